// Tuned launch shapes of the float32 TTM kernels (host only).
//
// The K split (waves per 64-row output tile) and the workgroups per CU of a
// TTM launch are picked by timing the candidates on the device (runtime.cpp).
// The results are kept per handle in memory and, across processes, in a JSON
// file:
//
//   {"format": 1, "device": "<gcnArchName>:<CUs>",
//    "entries": {"<key>": [ks, wpc], ...}}
//
// at $CPQR_TUNE_CACHE, else $XDG_CACHE_HOME/cpqr/ttm_tune.json, else
// $HOME/.cache/cpqr/ttm_tune.json.  CPQR_TUNE_CACHE=off keeps the results in
// memory only.  A file written for another device signature is ignored (and
// replaced on the next save); unreadable or malformed files are treated as
// empty.  Saving merges with the entries the file holds at that moment and
// replaces it by an atomic rename, so concurrent processes lose at most
// each other's newest entries, never the file.
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace cpqr {

struct TtmShape {
  int ks = 0;    // K split: 1, 2 or 4 (0: the launcher's own choice)
  int wpc = 0;   // workgroups per CU of the persistent grid: 1 or 2 (0: default)
};

class TuneCache {
 public:
  explicit TuneCache(int device);
  // A tuned shape for `key` (from this process or the file).
  bool find(const std::string& key, TtmShape* out);
  void put(const std::string& key, const TtmShape& s);
  // Writes new entries to the file (nothing when none were added or when
  // persistence is off).  Errors are ignored: the table is an optimisation.
  void save();
  const std::string& path() const { return path_; }
  const std::string& device() const { return device_; }

 private:
  void load();
  std::string path_, device_;
  std::map<std::string, TtmShape> mem_;
  bool loaded_ = false, dirty_ = false;
};

// Keys: one problem's TTM of shape [L, I, S] x R, and a batched group (the
// kernel class and every member's shape).
std::string ttm_key_single(int prec, int64_t L, int I, int64_t S, int R);
std::string ttm_key_batch(int prec, int nb, bool kc, const std::vector<std::array<int64_t, 4>>& shapes);

// File-format helpers (exposed for the host-only tests through cpqr.h).
std::string tune_cache_format(const std::string& device, const std::map<std::string, TtmShape>& entries);
bool tune_cache_parse(const std::string& text, const std::string& device,
                      std::map<std::string, TtmShape>* entries);

}  // namespace cpqr
