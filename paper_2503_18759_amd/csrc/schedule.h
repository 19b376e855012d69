// Schedule engine interface (host only).
#pragma once

#include <cstdint>
#include <vector>

namespace cpqr {

enum { STEP_TTM = 0, STEP_UPDATE = 1 };
enum { TREE_NONE = 0, TREE_STANDARD = 1, TREE_RESTRUCTURED = 2 };

struct Step {
  int kind;       // STEP_TTM or STEP_UPDATE
  uint32_t src;   // TTM: free-mode mask of the input; update: unused (0)
  int mode;       // TTM: contracted mode; update: updated mode
  bool operator==(const Step& o) const { return kind == o.kind && src == o.src && mode == o.mode; }
};

// Per-sweep step lists for `sweeps` sweeps.  Returns false on bad arguments.
bool build_schedule(int N, int tree, int sweeps, std::vector<std::vector<Step>>& out);

// Checks that every sweep updates every mode once and that every TTM input
// and every leaf only contains contractions with the current Q's.
bool validate_schedule(int N, const std::vector<std::vector<Step>>& sched);

// Intermediates (free-mode masks, X excluded) live across the boundary
// before sweep index `from` (0-based): those whose first access in sweeps
// from, from + 1, ... is a read, so that running those sweeps again needs
// their contents as they were at the boundary.
std::vector<uint32_t> live_intermediates(int N, const std::vector<std::vector<Step>>& sched, int from);

}  // namespace cpqr
