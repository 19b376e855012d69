// Dimension-tree schedules for the TTM chain of QR-based ALS (Section 3.1,
// Section 3.4 Tables 1-6).
//
// A schedule is a list of steps per sweep.  A TTM step contracts free mode m
// of the intermediate Y{F} (F = bitmask of modes still at full size; all bits
// set is X itself) with Q_m^T and produces Y{F \ m}; an update step consumes
// the leaf Y{n} to update factor n.  Intermediates are identified by their
// free-mode set, so the runtime keeps one buffer per set.
//
//  * none:         every leaf is contracted directly from X (ascending modes).
//  * standard:     the dimension tree of Figure 1 (Tables 1 and 4): split off
//                  the largest mode recursively; an order-3 subtree's second
//                  branch contracts its middle mode before its first
//                  (Table 1, cost 3 = 2 I1 I3 R^2); larger subtrees contract
//                  their remaining modes in ascending order.
//  * restructured: sweep 1 is a standard sweep.  Each later sweep (i) finishes
//                  the two-mode end of the previous sweep's last chain with
//                  the mode updated last, (ii) walks back up that chain and
//                  turns each level's unused free mode into a leaf by
//                  contracting the level's other free modes, most recently
//                  updated first, and (iii) performs one TTM on X for the
//                  most recently updated mode, contracts the other modes
//                  already updated in this sweep (most recent first) down to
//                  a two-mode intermediate, and updates its two modes
//                  (smaller index first).  This reproduces the cost tables of
//                  Section 3.4 for orders 3 and 4 and the update orders
//                  described in Section 3.1.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "schedule.h"

namespace cpqr {

namespace {

inline uint32_t bit(int m) { return 1u << m; }

std::vector<int> modes_of(uint32_t mask, int N) {
  std::vector<int> v;
  for (int k = 0; k < N; ++k)
    if (mask & bit(k)) v.push_back(k);
  return v;
}

void standard_tree(const std::vector<int>& T, std::vector<Step>& out) {
  uint32_t mask = 0;
  for (int m : T) mask |= bit(m);
  const size_t p = T.size();
  if (p == 2) {
    out.push_back({STEP_TTM, mask, T[1]});
    out.push_back({STEP_UPDATE, 0, T[0]});
    out.push_back({STEP_TTM, mask, T[0]});
    out.push_back({STEP_UPDATE, 0, T[1]});
    return;
  }
  const int last = T.back();
  out.push_back({STEP_TTM, mask, last});
  standard_tree(std::vector<int>(T.begin(), T.end() - 1), out);
  std::vector<int> branch;
  if (p == 3) branch = {T[1], T[0]};
  else branch.assign(T.begin(), T.end() - 1);
  uint32_t cur = mask;
  for (int m : branch) {
    out.push_back({STEP_TTM, cur, m});
    cur &= ~bit(m);
  }
  out.push_back({STEP_UPDATE, 0, last});
}

}  // namespace

bool build_schedule(int N, int tree, int sweeps, std::vector<std::vector<Step>>& out) {
  out.clear();
  if (N < 2 || N > 8 || sweeps < 1) return false;
  if (tree != TREE_NONE && N < 3) return false;
  const uint32_t full = (N >= 32) ? 0xffffffffu : ((1u << N) - 1u);
  if (tree == TREE_NONE) {
    for (int k = 0; k < sweeps; ++k) {
      std::vector<Step> s;
      for (int n = 0; n < N; ++n) {
        uint32_t cur = full;
        for (int m = 0; m < N; ++m) {
          if (m == n) continue;
          s.push_back({STEP_TTM, cur, m});
          cur &= ~bit(m);
        }
        s.push_back({STEP_UPDATE, 0, n});
      }
      out.push_back(std::move(s));
    }
    return true;
  }
  if (tree != TREE_STANDARD && tree != TREE_RESTRUCTURED) return false;

  std::vector<int64_t> stamp(N, 0);
  int64_t clock = 0;
  std::vector<uint32_t> chain;
  std::vector<int> all(N);
  for (int k = 0; k < N; ++k) all[k] = k;

  for (int k = 1; k <= sweeps; ++k) {
    std::vector<Step> s;
    if (tree == TREE_STANDARD || k == 1) {
      standard_tree(all, s);
      for (const Step& st : s)
        if (st.kind == STEP_UPDATE) stamp[st.mode] = ++clock;
      chain.clear();
      if (N == 3) {
        chain.push_back(bit(0) | bit(2));
      } else {
        for (int j = 1; j <= N - 2; ++j) chain.push_back(full & ~((1u << j) - 1u));
      }
      out.push_back(std::move(s));
      continue;
    }
    std::vector<int> updated;
    auto update = [&](int n) {
      s.push_back({STEP_UPDATE, 0, n});
      stamp[n] = ++clock;
      updated.push_back(n);
    };
    auto by_recency = [&](std::vector<int> v) {
      std::sort(v.begin(), v.end(), [&](int x, int y) { return stamp[x] > stamp[y]; });
      return v;
    };
    // (i) the two-mode end of the previous chain
    const uint32_t Fm = chain.back();
    std::vector<int> fm = modes_of(Fm, N);
    const int u = stamp[fm[0]] > stamp[fm[1]] ? fm[0] : fm[1];
    const int a = (u == fm[0]) ? fm[1] : fm[0];
    s.push_back({STEP_TTM, Fm, u});
    update(a);
    // (ii) walk back up the chain
    for (int j = (int)chain.size() - 2; j >= 0; --j) {
      const uint32_t Fj = chain[j];
      const uint32_t cmask = Fj & ~chain[j + 1];
      int c = -1;
      for (int m = 0; m < N; ++m)
        if (cmask & bit(m)) c = m;
      std::vector<int> others;
      for (int m : modes_of(Fj, N))
        if (m != c) others.push_back(m);
      uint32_t cur = Fj;
      for (int m : by_recency(others)) {
        s.push_back({STEP_TTM, cur, m});
        cur &= ~bit(m);
      }
      update(c);
    }
    // (iii) one TTM on X and the new chain
    const int mr = updated.back();
    uint32_t cur = full;
    s.push_back({STEP_TTM, cur, mr});
    cur &= ~bit(mr);
    std::vector<uint32_t> nchain{cur};
    std::vector<int> rest;
    for (int m : updated)
      if (m != mr) rest.push_back(m);
    for (int m : by_recency(rest)) {
      s.push_back({STEP_TTM, cur, m});
      cur &= ~bit(m);
      nchain.push_back(cur);
    }
    std::vector<int> pq = modes_of(cur, N);
    s.push_back({STEP_TTM, cur, pq[1]});
    update(pq[0]);
    s.push_back({STEP_TTM, cur, pq[0]});
    update(pq[1]);
    chain = nchain;
    out.push_back(std::move(s));
  }
  return true;
}

bool validate_schedule(int N, const std::vector<std::vector<Step>>& sched) {
  const uint32_t full = (1u << N) - 1u;
  std::vector<int> version(N, 0);
  // contracted versions per cached intermediate (by mask)
  std::vector<std::vector<int>> cache(1u << N);
  std::vector<bool> present(1u << N, false);
  present[full] = true;
  cache[full].assign(N, -1);
  for (const auto& sweep : sched) {
    std::vector<int> seen(N, 0);
    for (const Step& st : sweep) {
      if (st.kind == STEP_TTM) {
        if (!present[st.src] || !(st.src & (1u << st.mode))) return false;
        const auto& v = cache[st.src];
        for (int k = 0; k < N; ++k)
          if (v[k] >= 0 && v[k] != version[k]) return false;
        const uint32_t dst = st.src & ~(1u << st.mode);
        cache[dst] = v;
        cache[dst][st.mode] = version[st.mode];
        present[dst] = true;
      } else {
        const uint32_t leaf = 1u << st.mode;
        if (!present[leaf]) return false;
        const auto& v = cache[leaf];
        for (int k = 0; k < N; ++k) {
          if (k == st.mode) continue;
          if (v[k] != version[k]) return false;
        }
        version[st.mode]++;
        seen[st.mode]++;
      }
    }
    for (int k = 0; k < N; ++k)
      if (seen[k] != 1) return false;
  }
  return true;
}

std::vector<uint32_t> live_intermediates(int N, const std::vector<std::vector<Step>>& sched, int from) {
  const uint32_t full = (1u << N) - 1u;
  std::vector<char> first(1u << N, 0);   // 0: not accessed yet, 'r' or 'w'
  std::vector<uint32_t> live;
  for (size_t k = from < 0 ? 0 : (size_t)from; k < sched.size(); ++k)
    for (const Step& st : sched[k]) {
      const uint32_t rd = st.kind == STEP_TTM ? st.src : (1u << st.mode);
      if (rd != full && !first[rd]) {
        first[rd] = 'r';
        live.push_back(rd);
      }
      if (st.kind == STEP_TTM) {
        const uint32_t d = st.src & ~(1u << st.mode);
        if (!first[d]) first[d] = 'w';
      }
    }
  return live;
}

}  // namespace cpqr
