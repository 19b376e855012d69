// Host runtime and C ABI of the gfx950 CP-ALS-QR library.
//
// cpqr_als_qr runs Algorithm 2 / Algorithm 3 of arXiv 2503.18759 on one GPU:
// every step of the sweep (TTMs, Khatri-Rao QR, Y_(n) Q0, extrapolation,
// triangular solve, normalisation, factor QR, fit, activation rule) is a
// kernel launch on the handle's stream; the host only walks the schedule and
// reads results back at the end (or after each sweep when a tolerance is
// set).  Sweeps with the same step list are captured once into a HIP graph
// and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cpqr.h"
#include "kernels.h"
#include "mlp.h"
#include "schedule.h"
#include "tune_cache.h"

using namespace cpqr;

namespace {

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct cpqr_handle {
  int device = 0;
  hipStream_t user_stream = nullptr;  // stream given at creation (may be the null stream)
  hipStream_t stream = nullptr;       // stream the library launches on
  bool own_stream = false;
  hipEvent_t ready = nullptr;
  // second stream (default priority) for the Z QR branch of captured sweeps
  hipStream_t side = nullptr;
  // more streams (default priority) for the independent groups of a
  // batched sweep, which the captured graph runs as parallel branches
  std::vector<hipStream_t> pool;
  std::string err;
  std::map<std::string, DevBuf> bufs;
  bool busy = false;                  // a session is using the workspace
  // tuned launch shapes of float32 TTMs (in memory, and in the JSON file
  // of tune_cache.h), created at the first tuning
  std::unique_ptr<TuneCache> tune;
};

namespace {

// Make the work stream wait for everything already queued on the user's stream.
hipError_t order_after_user(cpqr_handle* h) {
  if (!h->own_stream) return hipSuccess;
  hipError_t e = hipEventRecord(h->ready, h->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(h->stream, h->ready, 0);
}

cpqr_status fail(cpqr_handle* h, cpqr_status s, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return s;
}

#define HIP_TRY(h, call)                                                                  \
  do {                                                                                    \
    hipError_t e__ = (call);                                                              \
    if (e__ != hipSuccess)                                                                \
      return fail((h), CPQR_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e__), \
                  __FILE__, __LINE__);                                                    \
  } while (0)

// Workspace buffer `name` with at least `bytes` bytes (grown on demand).
cpqr_status ws(cpqr_handle* h, const std::string& name, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  DevBuf& b = h->bufs[name];
  if (b.bytes < bytes) {
    if (b.ptr) HIP_TRY(h, hipFree(b.ptr));
    b.ptr = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b.ptr = nullptr;
      return fail(h, CPQR_ENOMEM, "device allocation of %zu bytes for %s failed", bytes, name.c_str());
    }
    b.bytes = bytes;
  }
  *out = b.ptr;
  return CPQR_OK;
}

#define WS(h, name, bytes, ptr)                                          \
  do {                                                                   \
    void* p__ = nullptr;                                                 \
    cpqr_status s__ = ws((h), (name), (bytes), &p__);                    \
    if (s__ != CPQR_OK) return s__;                                      \
    (ptr) = reinterpret_cast<decltype(ptr)>(p__);                        \
  } while (0)

// Back-to-back launches per timed level-1 TTM (CPQR_FLAG_TIME_KERNELS).
constexpr int kTimeReps = 8;

// Seeded N(0,1) initial factors (the "Initialize" step of Algorithms 2 and 3
// leaves the initialisation open).  Uniforms come from SplitMix64 (Steele,
// Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
// 2014, with the finaliser of Vigna's splitmix64.c): output j (0-based) of the
// sequence seeded with s is mix(s + (j + 1) * 0x9E3779B97F4A7C15), mapped to
// (0, 1) as ((z >> 11) + 0.5) 2^-53.  Entry e of the factors (modes in order,
// each I_n x R column-major, e counting across modes) is the Box-Muller
// normal sqrt(-2 ln u(2e)) cos(2 pi u(2e + 1)).
uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double unit_open(uint64_t z) { return ((double)(z >> 11) + 0.5) * 0x1.0p-53; }

std::vector<std::vector<double>> seeded_init_factors(uint64_t seed, const std::vector<int64_t>& dims, int R) {
  std::vector<std::vector<double>> out(dims.size());
  uint64_t e = 0;
  for (size_t k = 0; k < dims.size(); ++k) {
    out[k].resize((size_t)dims[k] * R);
    for (double& v : out[k]) {
      const double u1 = unit_open(splitmix64_at(seed, 2 * e));
      const double u2 = unit_open(splitmix64_at(seed, 2 * e + 1));
      v = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
      ++e;
    }
  }
  return out;
}

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Everything one decomposition needs on the device.
struct Problem {
  std::string prefix;     // workspace name prefix (one per problem of a batch)
  int N = 0, R = 0, prec = CPQR_PREC_FP32;
  std::vector<int64_t> dims;
  const void* X = nullptr;
  bool f64 = false;
  size_t elem = 4;
  int64_t M = 0;          // R^(N-1) rows of Z_n
  int P = 0;              // TSQR leaves
  int64_t leaf_rows = 0;
  StairPlan stair{};      // staircase Z_n QR (ok == false: dense TSQR)
  ZcolPlan zcol{};        // column-distributed staircase Z_n QR, compact Q0 (preferred)
  int* smap = nullptr;    // staircase row table of zqr_col (M x 2 ints)
  NestPlan nest{};        // nested two-factor Z_n QR (order >= 4 where neither plan above fits)
  int* nsmap = nullptr;   // its R^2-row staircase table
  double *nV = nullptr, *nMeta = nullptr, *nT = nullptr;   // per level: V, [Md, D, piv], T
  // Host-side bookkeeping of the sweep being enqueued, for reusing nested
  // levels: what each level's buffers hold (a signature of its remaining
  // modes and their factors' versions; 0: nothing valid) and the version of
  // every R factor (bumped when an update rewrites it)
  mutable std::vector<uint64_t> nest_sig;
  mutable std::vector<uint64_t> fac_ver;
  mutable uint64_t ver_clock = 0;
  std::map<uint32_t, TtmShape> ttm_ks;   // TTM step (src | mode << 16) -> launch shape
  int nchunks_max = 0;
  int Imax = 0;
  // device pointers
  std::vector<double*> A;      // factors (float64)
  std::vector<void*> Q;        // explicit Q_n in the TTM precision
  double* rf = nullptr;        // N x R x R R factors
  double* lambda = nullptr;
  std::vector<double*> q0buf;  // per mode: 2 x M x R (ping-pong): Q0, or V of the compact Q0
  std::vector<double*> q0meta; // per mode: 2 x (R^2 + 2R): [Md, D, piv] of the compact Q0
  double *tV = nullptr, *tT = nullptr, *tStack = nullptr, *tQtop = nullptr, *R0 = nullptr;
  // factor TSQR of modes with more than CPQR_MAX_FACTOR_ROWS rows (sized for
  // the largest such mode; fQ holds Q_n in float64 for the float32 chain)
  double *fV = nullptr, *fT = nullptr, *fStack = nullptr, *fQtop = nullptr, *fQ = nullptr;
  double *partial = nullptr, *Vbuf = nullptr, *qnbuf = nullptr;
  DevState* state = nullptr;
  double* fit_hist = nullptr;
  double* norm_part = nullptr;
  std::map<uint32_t, void*> inter;   // intermediates by free-mode mask
  // buffers that carry state from one sweep to the next besides the Q0
  // halves and the intermediates (part of the learned extrapolation's
  // checkpoint), and the checkpoint copies by live buffer
  std::vector<std::pair<void*, size_t>> carried;
  std::map<const void*, void*> shadow;
  double* beta_sched = nullptr;   // device copy of cpqr_options.beta_schedule (iters values) or null
  int sched_len = 0;
};

int64_t inter_elems(const Problem& p, uint32_t mask) {
  int64_t n = 1;
  for (int k = 0; k < p.N; ++k) n *= (mask & (1u << k)) ? p.dims[k] : p.R;
  return n;
}

}  // namespace

struct cpqr_session {
  cpqr_handle* h = nullptr;
  cpqr_options opts;
  Problem p;
  std::vector<std::vector<Step>> sched;
  int64_t nelem = 0;
  double nx2 = 0.0;
  int k = 0;                  // sweeps enqueued
  bool stopped = false;       // tolerance reached
  double ttm_flops = 0, ttm_bytes = 0, l1_bytes = 0, l1_flops = 0;
  int l1_count = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  bool t0_recorded = false;
  std::vector<hipEvent_t> evs;        // timing pairs of the level-1 TTMs
  std::vector<hipEvent_t> fork_evs;   // fork/join events of captured sweeps
  std::map<std::string, hipGraphExec_t> graphs;
  // CPQR_FLAG_TIME_PHASES: events at the kernel-group boundaries of a sweep,
  // the phase of the interval each one closes, and the accumulated times
  std::vector<hipEvent_t> ph_ev;
  std::vector<int> ph_lab;
  double phase[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // learned extrapolation
  float* mlp_w = nullptr;        // device weights
  float* mlp_io = nullptr;       // device features (CPQR_MLP_FEATURES) + output (1)
  bool learned_on = false;       // beta from the MLP in force
  bool fallback = false;         // a check failed: paper beta from then on
  double beta_learned = 0.0;
  double fit_accept = 0.0;       // explicit fit at the checkpoint
  int ckpt_k = 0;                // sweep of the checkpoint
  int next_check = 0;            // sweep of the next check
  int check_gap = 0;             // sweeps from the checkpoint to the next check
  int fallback_sweep = 0;
  ~cpqr_session() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    for (hipEvent_t e : fork_evs) (void)hipEventDestroy(e);
    for (hipEvent_t e : ph_ev) (void)hipEventDestroy(e);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  }
};

namespace {

cpqr_status setup(cpqr_handle* h, Problem& p, int iters,
                  const std::vector<std::vector<Step>>& sched) {
  const int N = p.N, R = p.R;
  p.A.resize(N);
  p.Q.resize(N);
  p.q0buf.resize(N);
  p.Imax = 0;
  for (int k = 0; k < N; ++k) {
    WS(h, p.prefix + "A" + std::to_string(k), (size_t)p.dims[k] * R * 8, p.A[k]);
    WS(h, p.prefix + "Q" + std::to_string(k), (size_t)p.dims[k] * R * p.elem, p.Q[k]);
    if (p.dims[k] > p.Imax) p.Imax = (int)p.dims[k];
  }
  WS(h, p.prefix + "rf", (size_t)N * R * R * 8, p.rf);
  WS(h, p.prefix + "lambda", (size_t)R * 8, p.lambda);
  p.M = ipow(R, N - 1);
  // the two-level TSQR's buffers, unless the nested QR takes every Z_n and
  // the TSQR has no plan at this size
  const TsqrPlan pl = tsqr_plan(p.M, R);
  if (!pl.ok && !p.nest.ok) return fail(h, CPQR_EUNSUPPORTED, "no Z QR plan for %lld x %d", (long long)p.M, R);
  p.leaf_rows = pl.ok ? pl.leaf_rows : 0;
  p.P = pl.ok ? pl.P : 0;
  for (int k = 0; k < N; ++k) WS(h, p.prefix + "q0_" + std::to_string(k), (size_t)2 * p.M * R * 8, p.q0buf[k]);
  p.q0meta.assign(N, nullptr);
  if (p.zcol.ok) {
    // staircase row table, and the reflector buffers cleared once: zqr_col
    // writes only the rows of each column's live chunks, the rest stay zero
    std::vector<int> tab((size_t)2 * p.M);
    stair_table(R, N - 1, p.M, tab.data());
    WS(h, p.prefix + "smap", tab.size() * sizeof(int), p.smap);
    HIP_TRY(h, hipMemcpy(p.smap, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
    for (int k = 0; k < N; ++k) {
      WS(h, p.prefix + "q0meta_" + std::to_string(k), (size_t)2 * (R * R + 2 * R) * 8, p.q0meta[k]);
      HIP_TRY(h, hipMemsetAsync(p.q0buf[k], 0, (size_t)2 * p.M * R * 8, h->stream));
      HIP_TRY(h, hipMemsetAsync(p.q0meta[k], 0, (size_t)2 * (R * R + 2 * R) * 8, h->stream));
    }
  }
  if (p.nest.ok) {
    // the levels' staircase table and reflector buffers (cleared once, as above)
    const int64_t R2 = (int64_t)R * R;
    const int L = p.nest.L;
    std::vector<int> tab((size_t)2 * R2);
    stair_table(R, 2, R2, tab.data());
    WS(h, p.prefix + "nsmap", tab.size() * sizeof(int), p.nsmap);
    HIP_TRY(h, hipMemcpy(p.nsmap, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
    WS(h, p.prefix + "nestV", (size_t)L * R2 * R * 8, p.nV);
    WS(h, p.prefix + "nestMeta", (size_t)L * (R2 + 2 * R) * 8, p.nMeta);
    WS(h, p.prefix + "nestT", (size_t)(L - 1) * R2 * 8, p.nT);
    HIP_TRY(h, hipMemsetAsync(p.nV, 0, (size_t)L * R2 * R * 8, h->stream));
  }
  if (pl.ok) {
    WS(h, p.prefix + "tsqrV", (size_t)p.P * p.leaf_rows * R * 8, p.tV);
    WS(h, p.prefix + "tsqrT", (size_t)p.P * R * R * 8, p.tT);
    WS(h, p.prefix + "tsqrS", (size_t)p.P * R * R * 8, p.tStack);
    WS(h, p.prefix + "tsqrQ", (size_t)p.P * R * R * 8, p.tQtop);
  }
  WS(h, p.prefix + "R0", (size_t)R * R * 8, p.R0);
  if (p.Imax > CPQR_MAX_FACTOR_ROWS) {
    // a smaller mode can take more, shorter leaves than a larger one, so the
    // buffers take the maximum over every tall mode's plan
    int64_t vrows = 0, pmax = 0;
    for (int k = 0; k < N; ++k) {
      if (p.dims[k] <= CPQR_MAX_FACTOR_ROWS) continue;
      const TsqrPlan fp = tsqr_plan(p.dims[k], R);
      if (!fp.ok) return fail(h, CPQR_EUNSUPPORTED, "no TSQR plan for a %lld x %d factor", (long long)p.dims[k], R);
      vrows = std::max<int64_t>(vrows, (int64_t)fp.P * fp.leaf_rows);
      pmax = std::max<int64_t>(pmax, fp.P);
    }
    WS(h, p.prefix + "ftsqrV", (size_t)vrows * R * 8, p.fV);
    WS(h, p.prefix + "ftsqrT", (size_t)pmax * R * R * 8, p.fT);
    WS(h, p.prefix + "ftsqrS", (size_t)pmax * R * R * 8, p.fStack);
    WS(h, p.prefix + "ftsqrQ", (size_t)pmax * R * R * 8, p.fQtop);
    if (!p.f64) WS(h, p.prefix + "ftsqrQ64", (size_t)p.Imax * R * 8, p.fQ);
  }
  int nch = 1;
  for (int k = 0; k < N; ++k) {
    const int c = apply_num_chunks(p.M, (int)p.dims[k]);
    if (c > nch) nch = c;
  }
  p.nchunks_max = nch;
  WS(h, p.prefix + "partial", (size_t)nch * 2 * p.Imax * R * 8, p.partial);
  WS(h, p.prefix + "V", (size_t)2 * p.Imax * R * 8, p.Vbuf);
  WS(h, p.prefix + "qn", (size_t)CPQR_QN_WORDS * 8, p.qnbuf);
  WS(h, p.prefix + "state", sizeof(DevState), p.state);
  // State that sweeps hand on besides the Q0 halves and the intermediates:
  // factors, Q_n, R factors, lambda and the device state.
  p.carried.clear();
  for (int k = 0; k < N; ++k) {
    p.carried.push_back({p.A[k], (size_t)p.dims[k] * R * 8});
    p.carried.push_back({p.Q[k], (size_t)p.dims[k] * R * p.elem});
  }
  p.carried.push_back({p.rf, (size_t)N * R * R * 8});
  p.carried.push_back({p.lambda, (size_t)R * 8});
  p.carried.push_back({p.state, sizeof(DevState)});
  WS(h, p.prefix + "fit_hist", (size_t)(iters > 0 ? iters : 1) * 8, p.fit_hist);
  WS(h, p.prefix + "norm_part", 4096 * 8, p.norm_part);
  // intermediates used by the schedule
  const uint32_t full = (1u << N) - 1u;
  for (const auto& sw : sched)
    for (const Step& st : sw)
      if (st.kind == STEP_TTM) {
        const uint32_t dst = st.src & ~(1u << st.mode);
        if (!p.inter.count(dst)) {
          void* ptr = nullptr;
          WS(h, p.prefix + "Y" + std::to_string(dst), (size_t)inter_elems(p, dst) * p.elem, ptr);
          p.inter[dst] = ptr;
        }
      }
  (void)full;
  return CPQR_OK;
}

// TTM of one schedule step: input (X or a cached intermediate), output
// intermediate and the [L, I, S] view around the contracted mode.
TtmArgs ttm_step_args(const Problem& p, const Step& st) {
  const uint32_t full = (1u << p.N) - 1u;
  const void* in = (st.src == full) ? p.X : p.inter.at(st.src);
  void* out = p.inter.at(st.src & ~(1u << st.mode));
  int64_t L = 1, S = 1;
  for (int k = 0; k < p.N; ++k) {
    const int64_t d = (st.src & (1u << k)) ? p.dims[k] : p.R;
    if (k < st.mode) L *= d;
    if (k > st.mode) S *= d;
  }
  return TtmArgs{(const float*)in, (const float*)p.Q[st.mode], (float*)out, L, S,
                 (int)p.dims[st.mode], p.R};
}

hipError_t launch_ttm_step(const Problem& p, const Step& st, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr) {
  const TtmArgs a = ttm_step_args(p, st);
  if (p.f64)
    return launch_ttm_f64((const double*)a.in, (const double*)a.Q, (double*)a.out, a.L, a.I, a.S, a.R, s,
                          ev0, ev1);
  const auto k = p.ttm_ks.find(st.src | ((uint32_t)st.mode << 16));
  const TtmShape sh = k == p.ttm_ks.end() ? TtmShape{} : k->second;
  return launch_ttm_f32(a.in, a.Q, a.out, a.L, a.I, a.S, a.R, p.prec == CPQR_PREC_BF16X3, s, ev0, ev1, sh.ks,
                        sh.wpc);
}

// Launch shape of every float32 TTM step of the schedule: the K split
// (waves per output tile: 1, 2 or 4, as the shape allows) and the
// workgroups per CU of the persistent grid (1 or 2).  Each shape is timed once
// (one warm-up and three launches per candidate, output redirected to scratch
// so that no cached intermediate is touched) and the fastest is kept in the
// handle's table, which tune_cache.h also keeps on disk, so that later
// processes on the same kind of device skip the timing.  The best shape
// depends on the shape and on the memory system, so it is measured rather
// than assumed.
TuneCache& handle_tune(cpqr_handle* h) {
  if (!h->tune) h->tune.reset(new TuneCache(h->device));
  return *h->tune;
}

cpqr_status tune_ttm_steps(cpqr_handle* h, Problem& p, const std::vector<std::vector<Step>>& sched) {
  if (p.f64) return CPQR_OK;
  hipStream_t s = h->stream;
  TuneCache& tc = handle_tune(h);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  for (const auto& sw : sched)
    for (const Step& st : sw) {
      if (st.kind != STEP_TTM) continue;
      const uint32_t key = st.src | ((uint32_t)st.mode << 16);
      if (p.ttm_ks.count(key)) continue;
      const TtmArgs a = ttm_step_args(p, st);
      const std::string name = ttm_key_single(p.prec, a.L, a.I, a.S, a.R);
      TtmShape best;
      if (tc.find(name, &best)) {
        p.ttm_ks[key] = best;
        continue;
      }
      const unsigned opts = ttm_ks_options(a.L, a.I, a.S, a.R);
      if (opts == 0) {   // not an MFMA shape: the launcher decides
        p.ttm_ks[key] = TtmShape{};
        continue;
      }
      float* out = nullptr;
      WS(h, "tune:ttm_out", (size_t)(a.L * a.S * a.R) * 4 + 256, out);
      if (!e0) {
        HIP_TRY(h, hipEventCreate(&e0));
        HIP_TRY(h, hipEventCreate(&e1));
      }
      float best_ms = 1e30f;
      const bool bf = p.prec == CPQR_PREC_BF16X3;
      for (int b = 0; b < 3; ++b) {
        if (!(opts & (1u << b))) continue;
        for (int wpc = 1; wpc <= 2; ++wpc) {
          const int ks = 1 << b;
          HIP_TRY(h, launch_ttm_f32(a.in, a.Q, out, a.L, a.I, a.S, a.R, bf, s, nullptr, nullptr, ks, wpc));
          HIP_TRY(h, hipEventRecord(e0, s));
          for (int r = 0; r < 3; ++r)
            HIP_TRY(h, launch_ttm_f32(a.in, a.Q, out, a.L, a.I, a.S, a.R, bf, s, nullptr, nullptr, ks, wpc));
          HIP_TRY(h, hipEventRecord(e1, s));
          HIP_TRY(h, hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms) {
            best_ms = ms;
            best = TtmShape{ks, wpc};
          }
        }
      }
      tc.put(name, best);
      p.ttm_ks[key] = best;
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  tc.save();
  return CPQR_OK;
}

// The closing plain sweep of CPQR_FLAG_CLOSING_PLAIN (1-based sweep k).
bool closing_sweep(const cpqr_options* o, int k) {
  return (o->flags & CPQR_FLAG_CLOSING_PLAIN) && k == o->iters;
}

// Arguments of the mode-n update of sweep k (Z QR, Y*Q0, finish).  Q0 of
// the sweep and of the previous sweep are the two halves of the mode's
// ping-pong buffer.
void update_args(const Problem& p, int n, int sweep_k, bool last, const cpqr_options* o, TsqrArgs* t,
                 ApplyArgs* a, FinishArgs* f) {
  const int R = p.R;
  double* q0cur = p.q0buf[n] + (size_t)(sweep_k % 2) * p.M * R;
  double* q0prev = (sweep_k >= 2) ? p.q0buf[n] + (size_t)((sweep_k - 1) % 2) * p.M * R : nullptr;
  t->N = p.N;
  t->n = n;
  t->R = R;
  t->rf = p.rf;
  t->src = nullptr;
  t->M = p.M;
  t->P = p.P;
  t->V = p.tV;
  t->T = p.tT;
  t->stack = p.tStack;
  t->R0 = p.R0;
  t->Qtop = p.tQtop;
  t->Q0 = q0cur;
  a->Y = p.inter.at(1u << n);
  a->y_f64 = p.f64;
  a->L = ipow(R, n);
  a->I = (int)p.dims[n];
  a->S = ipow(R, p.N - 1 - n);
  a->R = R;
  a->Q0 = q0cur;
  a->Q0prev = (o->extrapolate != CPQR_EXTRAP_OFF) ? q0prev : nullptr;
  a->partial = p.partial;
  a->V = p.Vbuf;
  a->nchunks = apply_num_chunks(p.M, a->I);
  a->state = p.state;
  if (p.zcol.ok) {
    const size_t mw = (size_t)R * R + 2 * R;
    a->meta_p = p.q0meta[n] + (size_t)(sweep_k % 2) * mw;
    a->meta_q = a->Q0prev ? p.q0meta[n] + (size_t)((sweep_k - 1) % 2) * mw : nullptr;
  }
  f->I = (int)p.dims[n];
  f->R = R;
  f->V = p.Vbuf;
  f->qn = p.qnbuf;
  f->R0 = p.R0;
  f->A = p.A[n];
  f->lambda = p.lambda;
  f->Rn = p.rf + (size_t)n * R * R;
  f->q64 = p.f64 ? (double*)p.Q[n] : nullptr;
  f->q32 = p.f64 ? nullptr : (float*)p.Q[n];
  f->state = p.state;
  f->fit_hist = p.fit_hist;
  f->alpha = o->alpha;
  f->delta = o->switch_delta;
  f->fixed_beta = o->fixed_beta;
  // the learned mode drives the same device-side beta state as the paper's rule
  f->extrap = (o->extrapolate != CPQR_EXTRAP_OFF && !closing_sweep(o, sweep_k)) ? 1 : 0;
  f->last_in_sweep = last ? 1 : 0;
  f->beta_sched = p.beta_sched;
  f->sched_len = p.sched_len;
}

// Factor QR of a mode with more than CPQR_MAX_FACTOR_ROWS rows: two-level
// TSQR of A_n (explicit source), then the float32 Q_n and the R_n check
// (state == nullptr: no check, for the initial factors).
hipError_t launch_tall_factor_qr(const Problem& p, int n, DevState* state, hipStream_t s) {
  const int R = p.R;
  const int I = (int)p.dims[n];
  const TsqrPlan fp = tsqr_plan(I, R);
  if (!fp.ok) return hipErrorInvalidValue;
  double* Rn = p.rf + (size_t)n * R * R;
  double* q64 = p.f64 ? (double*)p.Q[n] : p.fQ;
  TsqrArgs t{};
  t.N = 0;
  t.n = 0;
  t.R = R;
  t.rf = nullptr;
  t.src = p.A[n];
  t.M = I;
  t.P = fp.P;
  t.V = p.fV;
  t.T = p.fT;
  t.stack = p.fStack;
  t.R0 = Rn;
  t.Qtop = p.fQtop;
  t.Q0 = q64;
  hipError_t e = launch_tsqr(t, s);
  if (e != hipSuccess) return e;
  return launch_tall_factor_tail(I, R, q64, p.f64 ? nullptr : (float*)p.Q[n], Rn, state, s);
}

StairArgs stair_args(const TsqrArgs& t) {
  return StairArgs{t.N, t.n, t.R, t.M, t.rf, t.R0, t.Q0, 1};
}

// The nested Z QR of an order >= 4 update (NestPlan): the levels' staircase
// QRs, each reading the previous level's T, then the explicit Q0.
hipError_t launch_zqr_nested(const Problem& p, const TsqrArgs& t, hipStream_t s) {
  const int R = p.R, L = p.nest.L, n = t.n;
  const int64_t R2 = (int64_t)R * R;
  const size_t mw = (size_t)R2 + 2 * R;
  int m[CPQR_MAX_ORDER];   // remaining modes, ascending
  int nm = 0;
  for (int k = 0; k < p.N; ++k)
    if (k != n) m[nm++] = k;
  NestArgs na{};
  na.L = L;
  na.R = R;
  na.M = p.M;
  na.Q0 = t.Q0;
  // Level k (0-based) reads R_{m_1} .. R_{m_{k+2}} only.  Within a sweep, a
  // level whose buffers were written from the same factors at the same
  // versions (an earlier update with the same first remaining modes, none
  // of them rewritten since) is kept; the last level always runs, as it
  // writes R0.
  uint64_t sig[CPQR_MAX_ORDER] = {};
  int k0 = 0;
  if ((int)p.nest_sig.size() == L && (int)p.fac_ver.size() == p.N) {
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
      for (int b = 0; b < 8; ++b) {
        hsh ^= (v >> (8 * b)) & 0xff;
        hsh *= 1099511628211ull;
      }
    };
    mix((uint64_t)m[0]);
    mix(p.fac_ver[m[0]]);
    for (int k = 0; k < L; ++k) {
      mix((uint64_t)m[k + 1]);
      mix(p.fac_ver[m[k + 1]]);
      sig[k] = hsh | 1u;
    }
    while (k0 < L - 1 && p.nest_sig[k0] == sig[k0]) ++k0;
  }
  for (int k = 0; k < L; ++k) {
    na.V[k] = p.nV + (size_t)k * R2 * R;
    na.meta[k] = p.nMeta + (size_t)k * mw;
  }
  for (int k = k0; k < L; ++k) {
    ZcolArgs za{};
    za.N = 3;
    za.R = R;
    za.M = R2;
    za.smap = p.nsmap;
    za.V = p.nV + (size_t)k * R2 * R;
    za.meta = p.nMeta + (size_t)k * mw;
    za.R0 = (k + 1 < L) ? p.nT + (size_t)k * R2 : t.R0;
    za.active = 1;
    if (k == 0) {
      // W_1 = R_{m_2} (.) R_{m_1}: the first two remaining factors of the
      // full array, read as the order-3 array at t.rf (or t.rf + R^2)
      // without mode za.n
      if (n == 0) {
        za.rf = t.rf + R2;   // m_1 = 1, m_2 = 2
        za.n = 2;
      } else {
        za.rf = t.rf;        // m_1 = 0, m_2 = 1 (n >= 2) or 2 (n = 1)
        za.n = (n == 1) ? 1 : 2;
      }
    } else {
      // W_{k+1} = R_{m_{k+2}} (.) T_k
      za.rf = p.nT + (size_t)(k - 1) * R2;
      za.n = 2;
      za.rf_hi = t.rf + (size_t)m[k + 1] * R2;
    }
    hipError_t e = launch_zqr_col(p.nest.zp, za, s);
    if (e != hipSuccess) return e;
    if ((int)p.nest_sig.size() == L) p.nest_sig[k] = sig[k];
  }
  return launch_form_q0_nested(na, s);
}

// The Z QR of a mode update on the path its problem takes: the
// column-distributed staircase kernel (compact Q0), the one-workgroup
// staircase kernel, the nested two-factor QRs, or the two-level TSQR.
hipError_t launch_zqr_any(const Problem& p, const TsqrArgs& t, const ApplyArgs& a, hipStream_t s) {
  if (p.nest.ok) return launch_zqr_nested(p, t, s);
  if (p.zcol.ok)
    return launch_zqr_col(p.zcol, ZcolArgs{t.N, t.n, t.R, t.M, t.rf, p.smap, t.R0, t.Q0,
                                           const_cast<double*>(a.meta_p), 1}, s);
  return p.stair.ok ? launch_zqr_stair(p.stair, stair_args(t), s) : launch_tsqr(t, s);
}

// The QR Z_n = Q0 R0 of a mode update.  It reads only the R factors, so it
// may run beside the TTMs that produce the same update's Y_(n).
hipError_t launch_zqr(const Problem& p, int n, int sweep_k, bool last, const cpqr_options* o, hipStream_t s) {
  TsqrArgs t;
  ApplyArgs a;
  FinishArgs f;
  update_args(p, n, sweep_k, last, o, &t, &a, &f);
  return launch_zqr_any(p, t, a, s);
}

// One mode update; with zqr_done the Z QR has been enqueued already (on a
// branch that the stream has joined).  With tail given, a Q_n kernel that
// only the following TTMs need is left to the caller (*tail_pending set,
// its arguments in *tail).
// Phases of the time breakdown of Section 4.2 (cpqr_result.phase_seconds).
enum { PH_TTM = 0, PH_QR = 1, PH_Q0 = 2, PH_APPLY = 3, PH_OTHER = 4 };
// Records a phase boundary: the interval that ends here belongs to `phase`.
using PhaseMark = std::function<hipError_t(int phase)>;

hipError_t launch_update(const Problem& p, int n, int sweep_k, bool last, const cpqr_options* o,
                         hipStream_t s, bool zqr_done = false, FinishArgs* tail = nullptr,
                         bool* tail_pending = nullptr, const PhaseMark* mark = nullptr) {
  TsqrArgs t;
  ApplyArgs a;
  FinishArgs f;
  update_args(p, n, sweep_k, last, o, &t, &a, &f);
  hipError_t e = hipSuccess;
  auto at = [&](int phase) { return mark ? (*mark)(phase) : hipSuccess; };
  if (!zqr_done) {
    if ((e = at(PH_OTHER)) != hipSuccess) return e;
    e = launch_zqr_any(p, t, a, s);
    if (e != hipSuccess) return e;
    if ((e = at(PH_Q0)) != hipSuccess) return e;
  }
  if ((e = at(PH_OTHER)) != hipSuccess) return e;
  e = launch_apply(a, s);
  if (e != hipSuccess) return e;
  if ((e = at(PH_APPLY)) != hipSuccess) return e;
  if ((e = at(PH_OTHER)) != hipSuccess) return e;
  if (p.dims[n] <= CPQR_MAX_FACTOR_ROWS) {
    if (tail == nullptr) e = launch_finish(f, s);
    else {
      *tail = f;
      e = launch_finish_head(f, s, tail_pending);
    }
  } else {
    e = launch_finish_tall(f, s);
    if (e == hipSuccess) e = launch_tall_factor_qr(p, n, p.state, s);
  }
  if (e != hipSuccess) return e;
  return at(PH_QR);
}

std::string sweep_key(const std::vector<Step>& sw, int parity, bool extrap) {
  std::string k = std::to_string(parity) + (extrap ? "e" : "p");
  for (const Step& s : sw) {
    k += ":" + std::to_string(s.kind) + "," + std::to_string(s.src) + "," + std::to_string(s.mode);
  }
  return k;
}

// Host-side argument checks shared by cpqr_als_qr and cpqr_check_args.
cpqr_status check_args(cpqr_handle* h, const cpqr_tensor* X, int rank, const cpqr_options* o) {
  if (!X || !o) return fail(h, CPQR_EINVAL, "null argument");
  const int N = X->order;
  if (N < 2 || N > CPQR_MAX_ORDER) return fail(h, CPQR_EINVAL, "order must be in [2, %d]", CPQR_MAX_ORDER);
  if (!X->dims || !X->data) return fail(h, CPQR_EINVAL, "null tensor dims or data");
  if (rank < 1) return fail(h, CPQR_EINVAL, "rank must be >= 1");
  if (o->iters < 1) return fail(h, CPQR_EINVAL, "iters must be >= 1");
  if (o->tree < 0 || o->tree > 2) return fail(h, CPQR_EINVAL, "bad tree");
  if (N == 2 && o->tree != CPQR_TREE_NONE) return fail(h, CPQR_EINVAL, "order 2 needs tree=none");
  if (o->extrapolate < 0 || o->extrapolate > 2) return fail(h, CPQR_EINVAL, "bad extrapolation mode");
  if (o->extrapolate == CPQR_EXTRAP_LEARNED && !o->mlp_weights)
    return fail(h, CPQR_EINVAL, "learned extrapolation needs mlp_weights");
  if (o->prec < 0 || o->prec > 2) return fail(h, CPQR_EINVAL, "bad precision");
  if (X->dtype != CPQR_DTYPE_F32 && X->dtype != CPQR_DTYPE_F64) return fail(h, CPQR_EINVAL, "bad dtype");
  if ((o->prec == CPQR_PREC_FP64) != (X->dtype == CPQR_DTYPE_F64))
    return fail(h, CPQR_EINVAL, "FP64 precision needs a float64 tensor; FP32/BF16X3 need float32");
  if (!(o->tol >= 0.0) || !(o->alpha == o->alpha) || !(o->switch_delta >= 0.0) || !(o->fixed_beta >= 0.0))
    return fail(h, CPQR_EINVAL, "bad tol/alpha/switch_delta/fixed_beta");
  if ((o->flags & CPQR_FLAG_TIME_PHASES) && (o->flags & CPQR_FLAG_TIME_KERNELS))
    return fail(h, CPQR_EINVAL, "CPQR_FLAG_TIME_PHASES and CPQR_FLAG_TIME_KERNELS exclude each other");
  for (int k = 0; k < N; ++k) {
    if (X->dims[k] < 1) return fail(h, CPQR_EINVAL, "dims must be >= 1");
    // init_factors == NULL: seeded N(0,1) factors (seeded_init_factors)
    if (o->init_factors && !o->init_factors[k]) return fail(h, CPQR_EINVAL, "null init factor %d", k);
  }
  if (rank > 32) return fail(h, CPQR_EUNSUPPORTED, "rank > 32 is not supported by this build");
  // A mode smaller than the rank keeps min(I_k, R) nonzero rows of R_k, so
  // Z_n has prod_{k != n} min(I_k, R) nonzero rows; fewer than R means P^(n)
  // is rank-deficient and the least-squares update is not unique.
  for (int n = 0; n < N; ++n) {
    int64_t rows = 1;
    for (int k = 0; k < N; ++k)
      if (k != n) rows = std::min<int64_t>(rows * std::min<int64_t>(X->dims[k], rank), (int64_t)rank);
    if (rows < rank)
      return fail(h, CPQR_EUNSUPPORTED, "mode %d: the other modes give prod min(I_k, R) < rank %d rows of Z_n", n, rank);
  }
  for (int k = 0; k < N; ++k) {
    // modes above the single-workgroup factor QR go through the two-level
    // TSQR, which bounds their size
    if (X->dims[k] > CPQR_MAX_FACTOR_ROWS && (X->dims[k] > INT32_MAX || !tsqr_plan(X->dims[k], rank).ok))
      return fail(h, CPQR_EUNSUPPORTED, "mode %d of size %lld is beyond the two-level factor TSQR at rank %d", k,
                  (long long)X->dims[k], rank);
  }
  // Z_n of R^(N-1) rows: the nested two-factor QR covers every order up to
  // qr_max_order at R <= 32; CPQR_FLAG_DENSE_ZQR asks for the two-level TSQR,
  // which bounds R^(N-1)
  if (N > qr_max_order(rank))
    return fail(h, CPQR_EUNSUPPORTED, "order %d is beyond the Z QR kernels at rank %d", N, rank);
  if ((o->flags & CPQR_FLAG_DENSE_ZQR) && !tsqr_plan(ipow(rank, N - 1), rank).ok)
    return fail(h, CPQR_EUNSUPPORTED, "R^(N-1) too large for a two-level TSQR at this rank");
  if (o->prec == CPQR_PREC_BF16X3)
    for (int k = 0; k < N; ++k)
      if (!ttm_mfma_supported((int)X->dims[k], rank)) return fail(h, CPQR_EUNSUPPORTED, "bf16x3 TTM limits");

  return CPQR_OK;
}

}  // namespace

extern "C" {

const char* cpqr_status_string(int s) {
  switch (s) {
    case CPQR_OK: return "CPQR_OK";
    case CPQR_EINVAL: return "CPQR_EINVAL";
    case CPQR_EUNSUPPORTED: return "CPQR_EUNSUPPORTED";
    case CPQR_ENOMEM: return "CPQR_ENOMEM";
    case CPQR_EHIP: return "CPQR_EHIP";
    case CPQR_ERANKDEF: return "CPQR_ERANKDEF";
    case CPQR_ENONFINITE: return "CPQR_ENONFINITE";
    default: return "CPQR_UNKNOWN";
  }
}

cpqr_status cpqr_create(cpqr_handle** handle, int device, void* stream) {
  if (!handle) return CPQR_EINVAL;
  *handle = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return CPQR_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return CPQR_EHIP;
  }
  cpqr_handle* h = new cpqr_handle();
  h->device = device;
  h->user_stream = (hipStream_t)stream;
  if (h->user_stream == nullptr) {
    // graphs cannot be captured on the null stream: launch on a private
    // stream (default priority) ordered after the null stream at each call
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return CPQR_EHIP;
    }
    h->own_stream = true;
  } else {
    h->stream = h->user_stream;
  }
  if (hipEventCreateWithFlags(&h->ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return CPQR_EHIP;
  }
  *handle = h;
  return CPQR_OK;
}

cpqr_status cpqr_destroy(cpqr_handle* h) {
  if (!h) return CPQR_EINVAL;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  for (auto& kv : h->bufs)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  if (h->ready) (void)hipEventDestroy(h->ready);
  if (h->side) (void)hipStreamDestroy(h->side);
  for (hipStream_t q : h->pool) (void)hipStreamDestroy(q);
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return CPQR_OK;
}

const char* cpqr_last_error(const cpqr_handle* h) { return h ? h->err.c_str() : noalloc_last_error(); }

cpqr_status cpqr_schedule(int order, int tree, int sweeps, int* orders_out, int* steps_out,
                          int max_steps, int* n_steps, double* flops_out) {
  if (order < 2 || order > 8 || sweeps < 1 || tree < 0 || tree > 2) return CPQR_EINVAL;
  std::vector<std::vector<Step>> sched;
  if (!build_schedule(order, tree, sweeps, sched)) return CPQR_EINVAL;
  int total = 0;
  for (const auto& sw : sched) total += (int)sw.size();
  if (n_steps) *n_steps = total;
  if (steps_out && max_steps < total) return CPQR_EINVAL;
  int idx = 0;
  if (flops_out)
    for (int i = 0; i < (1 << order) * order; ++i) flops_out[i] = 0.0;
  for (size_t k = 0; k < sched.size(); ++k) {
    int u = 0;
    for (const Step& st : sched[k]) {
      if (steps_out) {
        steps_out[3 * idx + 0] = st.kind;
        steps_out[3 * idx + 1] = (int)st.src;
        steps_out[3 * idx + 2] = st.mode;
      }
      ++idx;
      if (st.kind == STEP_UPDATE) {
        if (orders_out) orders_out[k * order + u] = st.mode;
        ++u;
      } else if (flops_out) {
        flops_out[(size_t)st.src * order] += 2.0;
      }
    }
  }
  return CPQR_OK;
}

cpqr_status cpqr_ttm(cpqr_handle* h, int prec, int order, const int64_t* dims, int mode, int rank,
                     const void* in, const void* q, void* out) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!dims || !in || !q || !out) return fail(h, CPQR_EINVAL, "null pointer");
  if (order < 1 || order > 16 || mode < 0 || mode >= order || rank < 1)
    return fail(h, CPQR_EINVAL, "bad order/mode/rank");
  if (prec < 0 || prec > 2) return fail(h, CPQR_EINVAL, "bad precision");
  int64_t L = 1, S = 1;
  for (int k = 0; k < order; ++k) {
    if (dims[k] < 1) return fail(h, CPQR_EINVAL, "dims must be >= 1");
    if (k < mode) L *= dims[k];
    if (k > mode) S *= dims[k];
  }
  const int64_t I = dims[mode];
  if (I > (1 << 30)) return fail(h, CPQR_EUNSUPPORTED, "mode size too large");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  if (prec == CPQR_PREC_FP64) {
    HIP_TRY(h, launch_ttm_f64((const double*)in, (const double*)q, (double*)out, L, (int)I, S, rank, h->stream));
  } else {
    if (prec == CPQR_PREC_BF16X3 && !ttm_mfma_supported((int)I, rank))
      return fail(h, CPQR_EUNSUPPORTED, "bf16x3 TTM needs rank <= 64 and roundup(I,32) * roundup(R,16) * 4 <= 160 KiB");
    HIP_TRY(h, launch_ttm_f32((const float*)in, (const float*)q, (float*)out, L, (int)I, S, rank,
                              prec == CPQR_PREC_BF16X3, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return CPQR_OK;
}

cpqr_status cpqr_qr(cpqr_handle* h, int64_t M, int R, const double* A, double* Q, double* Rout) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!A || !Q || !Rout) return fail(h, CPQR_EINVAL, "null pointer");
  if (R < 1 || M < R) return fail(h, CPQR_EINVAL, "need 1 <= R <= M");
  if (R > 32) return fail(h, CPQR_EUNSUPPORTED, "R > 32");
  const TsqrPlan pl = tsqr_plan(M, R);
  if (!pl.ok) return fail(h, CPQR_EUNSUPPORTED, "M too large for a two-level TSQR at this R");
  const int64_t leaf = pl.leaf_rows;
  const int64_t P = pl.P;
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  TsqrArgs t;
  t.N = 0;
  t.n = 0;
  t.R = R;
  t.rf = nullptr;
  t.src = A;
  t.M = M;
  t.P = (int)P;
  WS(h, "qr_V", (size_t)P * leaf * R * 8, t.V);
  WS(h, "qr_T", (size_t)P * R * R * 8, t.T);
  WS(h, "qr_S", (size_t)P * R * R * 8, t.stack);
  WS(h, "qr_Q", (size_t)P * R * R * 8, t.Qtop);
  t.R0 = Rout;
  t.Q0 = Q;
  HIP_TRY(h, launch_tsqr(t, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return CPQR_OK;
}

cpqr_status cpqr_check_args(const cpqr_tensor* X, int rank, const cpqr_options* o) {
  return check_args(nullptr, X, rank, o);
}

}  // extern "C"

namespace {

cpqr_status checkpoint_shadows(cpqr_session* S, int c, std::vector<CopySeg>* save,
                               std::vector<CopySeg>* restore);

// Creates the device state of one decomposition (workspace names prefixed by
// `prefix`), computes ||X||^2 and the QRs of the initial factors.
cpqr_status session_create_impl(cpqr_handle* h, const cpqr_tensor* X, int rank, const cpqr_options* o,
                                const std::string& prefix, cpqr_session** out, bool batched = false) {
  *out = nullptr;
  {
    cpqr_status v = check_args(h, X, rank, o);
    if (v != CPQR_OK) return v;
  }
  const int N = X->order;
  std::unique_ptr<cpqr_session> ss(new cpqr_session());
  cpqr_session& S = *ss;
  S.h = h;
  S.opts = *o;
  S.opts.init_factors = nullptr;
  S.opts.mlp_weights = nullptr;
  S.opts.beta_schedule = nullptr;
  if (!build_schedule(N, o->tree, o->iters, S.sched) || !validate_schedule(N, S.sched))
    return fail(h, CPQR_EINVAL, "schedule construction failed");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  Problem& p = S.p;
  p.prefix = prefix;
  p.N = N;
  p.R = rank;
  p.prec = o->prec;
  p.dims.assign(X->dims, X->dims + N);
  p.X = X->data;
  p.f64 = (o->prec == CPQR_PREC_FP64);
  p.elem = p.f64 ? 8 : 4;
  if (!(o->flags & CPQR_FLAG_DENSE_ZQR)) {
    p.stair = stair_plan(N, rank);
    p.zcol = zcol_plan(N, rank);
    if (!p.stair.ok && !p.zcol.ok) p.nest = nest_plan(N, rank);
  }
  cpqr_status stt = setup(h, p, o->iters, S.sched);
  if (stt != CPQR_OK) return stt;
  S.nelem = 1;
  for (int k = 0; k < N; ++k) S.nelem *= p.dims[k];
  // ||X||^2 and the device state
  HIP_TRY(h, launch_sumsq(p.X, p.f64, S.nelem, p.norm_part, s));
  HIP_TRY(h, launch_state_init(p.state, p.norm_part, sumsq_blocks(S.nelem), s));
  // initial factors and their QRs (Algorithm 2, "Initialize"): the caller's,
  // or seeded N(0,1) ones
  std::vector<std::vector<double>> gen;
  if (!o->init_factors) gen = seeded_init_factors(o->seed, p.dims, rank);
  for (int k = 0; k < N; ++k) {
    const double* a0 = o->init_factors ? o->init_factors[k] : gen[k].data();
    HIP_TRY(h, hipMemcpyAsync(p.A[k], a0, (size_t)p.dims[k] * rank * 8, hipMemcpyHostToDevice, s));
    if (p.dims[k] > CPQR_MAX_FACTOR_ROWS)
      HIP_TRY(h, launch_tall_factor_qr(p, k, nullptr, s));
    else
      HIP_TRY(h, launch_factor_qr((int)p.dims[k], rank, p.A[k], p.rf + (size_t)k * rank * rank,
                                  p.f64 ? (double*)p.Q[k] : nullptr, p.f64 ? nullptr : (float*)p.Q[k], s));
  }
  HIP_TRY(h, launch_init_rank_check(p.rf, N, rank, p.dims.data(), p.state, s));
  DevState hs;
  HIP_TRY(h, hipMemcpyAsync(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  if (!(hs.nx2 > 0.0)) {
    if (hs.flags & FLAG_NONFINITE) return fail(h, CPQR_ENONFINITE, "tensor contains NaN or Inf");
    return fail(h, CPQR_EINVAL, "||X|| = 0");
  }
  if (hs.flags & FLAG_NONFINITE) return fail(h, CPQR_ENONFINITE, "tensor contains NaN or Inf");
  if (hs.flags & FLAG_RANKDEF)
    return fail(h, CPQR_ERANKDEF, "an initial factor has (numerically) dependent columns");
  S.nx2 = hs.nx2;
  stt = tune_ttm_steps(h, p, S.sched);
  if (stt != CPQR_OK) return stt;
  if (o->beta_schedule && o->extrapolate == CPQR_EXTRAP_PAPER) {
    WS(h, prefix + "beta_sched", (size_t)o->iters * sizeof(double), p.beta_sched);
    HIP_TRY(h, hipMemcpy(p.beta_sched, o->beta_schedule, (size_t)o->iters * sizeof(double),
                         hipMemcpyHostToDevice));
    p.sched_len = o->iters;
  }
  if (o->extrapolate == CPQR_EXTRAP_LEARNED) {
    WS(h, prefix + "mlp_w", CPQR_MLP_PARAMS * sizeof(float), S.mlp_w);
    WS(h, prefix + "mlp_io", (CPQR_MLP_FEATURES + 1) * sizeof(float), S.mlp_io);
    HIP_TRY(h, hipMemcpy(S.mlp_w, o->mlp_weights, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    // the checkpoint copies for every boundary the checks can fall on, so
    // that no sweep allocates
    for (int c = 2; c < o->iters; ++c) {
      stt = checkpoint_shadows(&S, c, nullptr, nullptr);
      if (stt != CPQR_OK) return stt;
    }
  }
  HIP_TRY(h, hipEventCreate(&S.t0));
  HIP_TRY(h, hipEventCreate(&S.t1));
  *out = ss.release();
  return CPQR_OK;
}

}  // namespace

extern "C" {

cpqr_status cpqr_session_create(cpqr_handle* h, const cpqr_tensor* X, int rank,
                                const cpqr_options* o, cpqr_session** out) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!out) return fail(h, CPQR_EINVAL, "null session pointer");
  *out = nullptr;
  if (h->busy) return fail(h, CPQR_EINVAL, "the handle already has a live session");
  cpqr_status st = session_create_impl(h, X, rank, o, "", out);
  if (st == CPQR_OK) h->busy = true;
  return st;
}

}  // extern "C"

namespace {

// Enqueues sweep k (graph replay, or kernel by kernel) and counts its TTM work.
// Runs sweep k (1-based).  capture_only: only capture (and keep) the sweep's
// graph if it is not there yet, without running it.
cpqr_status run_sweep(cpqr_session* S, int k, bool capture_only = false) {
  cpqr_handle* h = S->h;
  hipStream_t s = h->stream;
  const cpqr_options* o = &S->opts;
  Problem& p = S->p;
  const int N = p.N;
  const bool timing = (o->flags & CPQR_FLAG_TIME_KERNELS) != 0;
  const bool phases = (o->flags & CPQR_FLAG_TIME_PHASES) != 0;
  const bool use_graph = !timing && !phases && !(o->flags & CPQR_FLAG_NO_GRAPH);
  const uint32_t full = (1u << N) - 1u;
  const auto& sw = S->sched[k - 1];
  if (capture_only && !use_graph) return CPQR_OK;
  // phase timing: an event at every kernel-group boundary, kernel by kernel
  size_t ph_n = 0;
  const PhaseMark mark = [&](int phase) -> hipError_t {
    if (ph_n == S->ph_ev.size()) {
      hipEvent_t ev;
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return e;
      S->ph_ev.push_back(ev);
      S->ph_lab.push_back(PH_OTHER);
    }
    S->ph_lab[ph_n] = phase;
    return hipEventRecord(S->ph_ev[ph_n++], s);
  };
  for (const Step& st : sw)
    if (st.kind == STEP_TTM && !capture_only) {
      const int64_t in = inter_elems(p, st.src);
      const int64_t outn = in / p.dims[st.mode] * p.R;
      S->ttm_flops += 2.0 * in * p.R;
      S->ttm_bytes += (double)(in + outn) * p.elem;
      if (st.src == full) {
        S->l1_bytes += (double)(in + outn) * p.elem;
        S->l1_flops += 2.0 * in * p.R;
        ++S->l1_count;
      }
    }
  int last_update = -1;
  for (size_t i = 0; i < sw.size(); ++i)
    if (sw[i].kind == STEP_UPDATE) last_update = (int)i;
  // In a captured sweep each update's Z QR (the one-workgroup staircase
  // kernel, or the TSQR's few workgroups) is forked onto the side stream as
  // soon as the previous update is enqueued, so that it runs beside the TTMs
  // producing the same update's Y_(n); the update joins the branch before its
  // product with Q0.  (Measured at 256^3 rank 32: forking every update beats
  // forking only those behind a level-1 TTM; the fork and join cost less
  // than a level-2 TTM.)
  bool fork = use_graph;
  if (fork && h->side == nullptr &&
      hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    h->side = nullptr;
    fork = false;
  }
  // fork and join events of the captured branches, created before capture
  std::vector<hipEvent_t> fev;
  size_t fnext = 0;
  auto make_fork_events = [&]() -> hipError_t {
    for (const Step& st : sw) {
      if (st.kind != STEP_UPDATE) continue;
      for (int r = 0; r < 2; ++r) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        S->fork_evs.push_back(ev);
        fev.push_back(ev);
      }
    }
    return hipSuccess;
  };
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    if (p.nest.ok) {
      // nested levels are reused within a sweep only
      p.nest_sig.assign(p.nest.L, 0);
      p.fac_ver.assign(p.N, 0);
    }
    hipEvent_t join = nullptr;   // end of the forked Z QR of the next update
    bool forked = false;         // the next update's Z QR is on the side branch
    auto fork_next = [&](size_t from) -> hipError_t {
      size_t j = from;
      while (j < sw.size() && sw[j].kind != STEP_UPDATE) ++j;
      forked = false;
      if (j == sw.size()) return hipSuccess;
      if (fnext + 2 > fev.size()) return hipErrorInvalidValue;
      hipEvent_t a = fev[fnext++], b = fev[fnext++];
      hipError_t e;
      if ((e = hipEventRecord(a, q)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(h->side, a, 0)) != hipSuccess) return e;
      if ((e = launch_zqr(p, sw[j].mode, k, (int)j == last_update, o, h->side)) != hipSuccess) return e;
      if ((e = hipEventRecord(b, h->side)) != hipSuccess) return e;
      join = b;
      forked = true;
      return hipSuccess;
    };
    if (fork) {
      hipError_t e = fork_next(0);
      if (e != hipSuccess) return e;
    }
    if (phases) {
      hipError_t e = mark(-1);
      if (e != hipSuccess) return e;
    }
    for (size_t i = 0; i < sw.size(); ++i) {
      const Step& st = sw[i];
      hipError_t e;
      if (st.kind == STEP_TTM) {
        if (timing && st.src == full) {
          // The level-1 TTM is idempotent (it rewrites its output from X and
          // Q_m), so it is timed as a graph of kTimeReps back-to-back
          // launches between two events: the per-launch average then holds
          // no event or launch overhead.
          const std::string gk = "l1rep:" + std::to_string(st.src) + ":" + std::to_string(st.mode);
          auto itr = S->graphs.find(gk);
          if (itr == S->graphs.end()) {
            hipGraph_t g;
            if ((e = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
            hipError_t el = hipSuccess;
            for (int r = 0; r < kTimeReps && el == hipSuccess; ++r) el = launch_ttm_step(p, st, q);
            if ((e = hipStreamEndCapture(q, &g)) != hipSuccess) return e;
            if (el != hipSuccess) return el;
            hipGraphExec_t ge;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            itr = S->graphs.emplace(gk, ge).first;
          }
          hipEvent_t a, b;
          if ((e = hipEventCreate(&a)) != hipSuccess) return e;
          if ((e = hipEventCreate(&b)) != hipSuccess) return e;
          S->evs.push_back(a);
          S->evs.push_back(b);
          if ((e = hipEventRecord(a, q)) != hipSuccess) return e;
          if ((e = hipGraphLaunch(itr->second, q)) != hipSuccess) return e;
          if ((e = hipEventRecord(b, q)) != hipSuccess) return e;
        } else {
          if (phases && (e = mark(PH_OTHER)) != hipSuccess) return e;
          if ((e = launch_ttm_step(p, st, q)) != hipSuccess) return e;
          if (phases && (e = mark(PH_TTM)) != hipSuccess) return e;
        }
      } else if (fork) {
        const bool z = forked;
        if (z && (e = hipStreamWaitEvent(q, join, 0)) != hipSuccess) return e;
        // the next update's Z QR needs R_n only: fork it before the Q_n
        // kernel, which only the following TTMs wait for
        FinishArgs ft{};
        bool tail = false;
        if ((e = launch_update(p, st.mode, k, (int)i == last_update, o, q, z, &ft, &tail)) != hipSuccess)
          return e;
        if (p.nest.ok) p.fac_ver[st.mode] = ++p.ver_clock;   // R_n rewritten
        if ((e = fork_next(i + 1)) != hipSuccess) return e;
        if (tail && (e = launch_finish_tail(ft, q)) != hipSuccess) return e;
      } else {
        if ((e = launch_update(p, st.mode, k, (int)i == last_update, o, q, false, nullptr, nullptr,
                               phases ? &mark : nullptr)) != hipSuccess)
          return e;
        if (p.nest.ok) p.fac_ver[st.mode] = ++p.ver_clock;   // R_n rewritten
      }
    }
    return hipSuccess;
  };
  if (use_graph) {
    // sweeps with the same step list and Q0 ping-pong parity share a graph
    const std::string key = sweep_key(sw, k == 1 ? 2 : (k % 2), o->extrapolate != 0 && !closing_sweep(o, k));
    auto itg = S->graphs.find(key);
    if (itg == S->graphs.end()) {
      hipGraph_t g;
      if (fork) HIP_TRY(h, make_fork_events());
      HIP_TRY(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(s);
      hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess) return fail(h, CPQR_EHIP, "kernel launch during capture failed: %s", hipGetErrorString(e));
      if (e2 != hipSuccess) return fail(h, CPQR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
      hipGraphExec_t ge;
      hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess) return fail(h, CPQR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
      itg = S->graphs.emplace(key, ge).first;
    }
    if (capture_only) return CPQR_OK;
    HIP_TRY(h, hipGraphLaunch(itg->second, s));
  } else {
    hipError_t e = enqueue(s);
    if (e != hipSuccess) return fail(h, CPQR_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    if (phases && ph_n > 0) {
      HIP_TRY(h, hipEventSynchronize(S->ph_ev[ph_n - 1]));
      for (size_t i = 1; i < ph_n; ++i) {
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, S->ph_ev[i - 1], S->ph_ev[i]));
        const int lab = S->ph_lab[i];
        if (lab >= 0 && lab < 5) S->phase[lab] += ms * 1e-3;
      }
    }
  }
  return CPQR_OK;
}

// Checkpoint of the state after sweep c (1-based) for the learned
// extrapolation: everything sweeps c+1, c+2, ... read before they write it,
// that is the carried buffers, the Q0 half of sweep c of every mode (Q0^{k-1}
// of sweep c+1) with its compact-form metadata, and the intermediates live
// across the boundary.
cpqr_status checkpoint_bufs(cpqr_session* S, int c, std::vector<std::pair<void*, size_t>>* bufs) {
  Problem& p = S->p;
  *bufs = p.carried;
  const size_t mw = (size_t)p.R * p.R + 2 * p.R;
  for (int n = 0; n < p.N; ++n) {
    bufs->push_back({p.q0buf[n] + (size_t)(c % 2) * p.M * p.R, (size_t)p.M * p.R * 8});
    if (p.q0meta[n]) bufs->push_back({p.q0meta[n] + (size_t)(c % 2) * mw, mw * 8});
  }
  for (uint32_t m : live_intermediates(p.N, S->sched, c)) {
    auto it = p.inter.find(m);
    if (it == p.inter.end()) return fail(S->h, CPQR_EINVAL, "checkpoint: intermediate %u not allocated", m);
    bufs->push_back({it->second, (size_t)inter_elems(p, m) * p.elem});
  }
  return CPQR_OK;
}

// The copy of every buffer of the checkpoint after sweep c (allocated once).
cpqr_status checkpoint_shadows(cpqr_session* S, int c, std::vector<CopySeg>* save,
                               std::vector<CopySeg>* restore) {
  cpqr_handle* h = S->h;
  Problem& p = S->p;
  std::vector<std::pair<void*, size_t>> bufs;
  cpqr_status st = checkpoint_bufs(S, c, &bufs);
  if (st != CPQR_OK) return st;
  for (const auto& b : bufs) {
    auto it = p.shadow.find(b.first);
    if (it == p.shadow.end()) {
      void* sh = nullptr;
      WS(h, p.prefix + "ckpt" + std::to_string(p.shadow.size()), b.second, sh);
      it = p.shadow.emplace(b.first, sh).first;
    }
    if (save) save->push_back(CopySeg{b.first, it->second, (int64_t)b.second});
    if (restore) restore->push_back(CopySeg{it->second, b.first, (int64_t)b.second});
  }
  return CPQR_OK;
}

// Saves (save) or restores the checkpoint after sweep c: one launch per
// COPY_LIST_MAX buffers, on the library's stream.
cpqr_status checkpoint(cpqr_session* S, int c, bool save) {
  std::vector<CopySeg> segs;
  cpqr_status st = checkpoint_shadows(S, c, save ? &segs : nullptr, save ? nullptr : &segs);
  if (st != CPQR_OK) return st;
  HIP_TRY(S->h, launch_copy_list(segs.data(), (int)segs.size(), S->h->stream));
  return CPQR_OK;
}

// Fits of sweeps k-1 and k (1-based k >= 2).
cpqr_status read_fits(cpqr_session* S, int k, double* f) {
  cpqr_handle* h = S->h;
  HIP_TRY(h, hipMemcpyAsync(f, S->p.fit_hist + (k - 2), 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return CPQR_OK;
}

// Explicit fit 1 - ||X - K|| / ||X|| of the current factors, with lambda
// multiplied by lambda_scale (float64 accumulation).
cpqr_status explicit_fit(cpqr_session* S, double lambda_scale, double* fit) {
  cpqr_handle* h = S->h;
  Problem& p = S->p;
  std::vector<double*> fac(p.A.begin(), p.A.end());
  HIP_TRY(h, launch_residual(p.X, p.f64, p.N, p.dims.data(), fac.data(), p.lambda, p.R, p.norm_part, h->stream,
                             lambda_scale));
  const int nb = sumsq_blocks(S->nelem);
  std::vector<double> part(nb);
  HIP_TRY(h, hipMemcpyAsync(part.data(), p.norm_part, nb * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  double r2 = 0.0;
  for (double v : part) r2 += v;
  *fit = 1.0 - std::sqrt(r2) / std::sqrt(S->nx2);
  return CPQR_OK;
}

cpqr_status set_beta(cpqr_session* S, double beta, int beta_sweep) {
  cpqr_handle* h = S->h;
  DevState hs;
  HIP_TRY(h, hipMemcpyAsync(&hs, S->p.state, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  hs.active = 1;
  hs.beta = beta;
  hs.beta_sweep = beta_sweep;
  HIP_TRY(h, hipMemcpyAsync(S->p.state, &hs, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return CPQR_OK;
}

// The paper's beta table (Section 4.3), used for the fallback of a rejected
// learned sweep.
double paper_beta(double fit) {
  if (fit > 0.95) return 1.0 / 20000.0;
  if (fit > 0.90) return 1.0 / 2000.0;
  if (fit > 0.70) return 1.0 / 500.0;
  return 1.0 / 250.0;
}

// Upper end of the training grid of the learned beta.
constexpr double kMaxLearnedBeta = 30.0;
// Sweeps from the learned beta's start (after sweep 2) to its first check;
// the gap between checks doubles after every passed check.
constexpr int kLearnedFirstCheck = 4;

// Learned beta after sweep 2 from the fits of sweeps 1 and 2 (features as in
// cpqr.h), evaluated by the MLP kernel.
cpqr_status learned_beta(cpqr_session* S, double f1, double f2, double* beta) {
  cpqr_handle* h = S->h;
  const Problem& p = S->p;
  double sumI = 0.0, minI = 1e300;
  for (int64_t d : p.dims) {
    sumI += (double)d;
    minI = std::min(minI, (double)d);
  }
  float x[CPQR_MLP_FEATURES] = {
      (float)f1, (float)f2, (float)(10.0 * (f2 - f1)),
      (float)(std::log10(std::max(1.0 - f2, 1e-12)) / 4.0), (float)(p.N / 5.0), (float)(p.R / 16.0),
      (float)(std::log2(sumI / p.N) / 8.0), (float)(p.R / minI)};
  HIP_TRY(h, hipMemcpyAsync(S->mlp_io, x, sizeof(x), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, launch_mlp_forward(S->mlp_w, S->mlp_io, 1, S->mlp_io + CPQR_MLP_FEATURES, h->stream));
  float y = 0.f;
  HIP_TRY(h, hipMemcpyAsync(&y, S->mlp_io + CPQR_MLP_FEATURES, sizeof(float), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  // y is u = g beta / (1 + g beta), g = 1 - 0.1 (the alpha of the training
  // runs): the momentum of the normalised eq. (19) update up to alpha / g
  constexpr double g = 0.9;
  constexpr double u_max = g * kMaxLearnedBeta / (1.0 + g * kMaxLearnedBeta);
  double u = (double)y;
  if (!(u > 0.0)) u = 0.0;
  if (u > u_max) u = u_max;
  *beta = std::min(u / (g * (1.0 - u)), kMaxLearnedBeta);
  return CPQR_OK;
}

}  // namespace

extern "C" {

cpqr_status cpqr_session_sweeps(cpqr_session* S, int nsweeps) {
  if (!S) return CPQR_EINVAL;
  cpqr_handle* h = S->h;
  h->err.clear();
  if (nsweeps < 0) return fail(h, CPQR_EINVAL, "nsweeps must be >= 0");
  if (S->stopped) return CPQR_OK;
  if (S->k + nsweeps > S->opts.iters)
    return fail(h, CPQR_EINVAL, "session was created for %d sweeps", S->opts.iters);
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  const cpqr_options* o = &S->opts;
  Problem& p = S->p;
  const bool learned = o->extrapolate == CPQR_EXTRAP_LEARNED;
  if (!S->t0_recorded) {
    HIP_TRY(h, hipEventRecord(S->t0, s));
    S->t0_recorded = true;
  }
  for (int it = 0; it < nsweeps; ++it) {
    const int k = S->k + 1;
    cpqr_status st;
    if ((st = run_sweep(S, k)) != CPQR_OK) return st;
    S->k = k;
    // the closing plain sweep's graph (another key when extrapolation is on)
    // is captured with the first sweep's, so that no later sweep pays for it
    if (k == 1 && closing_sweep(o, o->iters) && o->iters > 1 && (st = run_sweep(S, o->iters, true)) != CPQR_OK)
      return st;
    if (learned && k == 2 && !S->learned_on) {
      double f[2], b = 0.0;
      if ((st = read_fits(S, 2, f)) != CPQR_OK) return st;
      if ((st = explicit_fit(S, 1.0, &S->fit_accept)) != CPQR_OK) return st;
      if ((st = learned_beta(S, f[0], f[1], &b)) != CPQR_OK) return st;
      if ((st = set_beta(S, b, 2)) != CPQR_OK) return st;
      S->beta_learned = b;
      S->learned_on = true;
      S->ckpt_k = 2;
      S->check_gap = kLearnedFirstCheck;
      S->next_check = 2 + kLearnedFirstCheck;
      if (o->iters > 2 && (st = checkpoint(S, 2, true)) != CPQR_OK) return st;
    }
    bool tol_stop = false;
    if (o->tol > 0.0 && k >= 2) {
      DevState hs;
      HIP_TRY(h, hipMemcpyAsync(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
      double fk[2];
      HIP_TRY(h, hipMemcpyAsync(fk, p.fit_hist + (k - 2), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(h, hipStreamSynchronize(s));
      tol_stop = hs.flags || std::fabs(fk[1] - fk[0]) < o->tol;
    }
    if (learned && S->learned_on && !S->fallback && k > 2 &&
        (k == S->next_check || k == o->iters || tol_stop)) {
      // acceptance test on the explicit fit.  While beta is on, eq. (19)
      // scales each update by about 1 + (1 - alpha) beta (exactly at a fixed
      // point), which lambda carries and the factors' directions do not; the
      // fit is taken with lambda divided by that factor, so that it compares
      // with the checkpoint's.  The closing plain sweep needs no correction.
      double fx = 0.0;
      const double scale = closing_sweep(o, k) ? 1.0 : 1.0 / (1.0 + (1.0 - o->alpha) * S->beta_learned);
      if ((st = explicit_fit(S, scale, &fx)) != CPQR_OK) return st;
      if (fx > S->fit_accept) {
        S->fit_accept = fx;
        S->ckpt_k = k;
        S->check_gap *= 2;
        S->next_check = k + S->check_gap;
        if (k < o->iters && !tol_stop && (st = checkpoint(S, k, true)) != CPQR_OK) return st;
      } else {
        // back to the checkpoint; sweeps ckpt_k + 1 .. k again with the
        // paper's beta for the checkpoint's fit
        if ((st = checkpoint(S, S->ckpt_k, false)) != CPQR_OK) return st;
        if ((st = set_beta(S, paper_beta(S->fit_accept), S->ckpt_k)) != CPQR_OK) return st;
        S->fallback = true;
        S->fallback_sweep = S->ckpt_k + 1;
        for (int j = S->ckpt_k + 1; j <= k; ++j)
          if ((st = run_sweep(S, j)) != CPQR_OK) return st;
        tol_stop = false;
        if (o->tol > 0.0) {
          DevState hs;
          HIP_TRY(h, hipMemcpyAsync(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
          double fk[2];
          HIP_TRY(h, hipMemcpyAsync(fk, p.fit_hist + (k - 2), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
          HIP_TRY(h, hipStreamSynchronize(s));
          tol_stop = hs.flags || std::fabs(fk[1] - fk[0]) < o->tol;
        }
      }
    }
    if (tol_stop) {
      S->stopped = true;
      break;
    }
  }
  return CPQR_OK;
}

cpqr_status cpqr_tune_cache_check(const char* text, const char* device, int* entries) {
  if (!text || !device) return CPQR_EINVAL;
  std::map<std::string, TtmShape> e;
  if (!tune_cache_parse(text, device, &e)) return CPQR_EINVAL;
  if (entries) *entries = (int)e.size();
  return CPQR_OK;
}

cpqr_status cpqr_tune_cache_path(cpqr_handle* h, char* path, char* device, int cap) {
  if (!h) return CPQR_EINVAL;
  if (cap <= 0) return CPQR_OK;
  HIP_TRY(h, hipSetDevice(h->device));
  TuneCache& tc = handle_tune(h);
  auto put = [cap](char* dst, const std::string& v) {
    if (!dst) return;
    const size_t n = std::min(v.size(), (size_t)cap - 1);
    std::memcpy(dst, v.data(), n);
    dst[n] = '\0';
  };
  put(path, tc.path());
  put(device, tc.device());
  return CPQR_OK;
}

cpqr_status cpqr_session_sync(cpqr_session* S) {
  if (!S) return CPQR_EINVAL;
  cpqr_handle* h = S->h;
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return CPQR_OK;
}

cpqr_status cpqr_session_result(cpqr_session* S, cpqr_result* res) {
  if (!S || !res) return CPQR_EINVAL;
  cpqr_handle* h = S->h;
  h->err.clear();
  HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  Problem& p = S->p;
  const int N = p.N, rank = p.R;
  const int done = S->k;
  HIP_TRY(h, hipEventRecord(S->t1, s));
  HIP_TRY(h, hipEventSynchronize(S->t1));
  float ms = 0.f;
  if (S->t0_recorded) HIP_TRY(h, hipEventElapsedTime(&ms, S->t0, S->t1));
  double l1_sec = 0.0;
  for (size_t i = 0; i + 1 < S->evs.size(); i += 2) {
    float e = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&e, S->evs[i], S->evs[i + 1]));
    l1_sec += e * 1e-3 / kTimeReps;
  }
  DevState hs;
  HIP_TRY(h, hipMemcpy(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost));
  std::vector<double> fits(done > 0 ? done : 1);
  if (done > 0) HIP_TRY(h, hipMemcpy(fits.data(), p.fit_hist, (size_t)done * 8, hipMemcpyDeviceToHost));
  res->sweeps_done = done;
  if (res->fit_history)
    for (int k = 0; k < done; ++k) res->fit_history[k] = fits[k];
  if (hs.flags & FLAG_NONFINITE) return fail(h, CPQR_ENONFINITE, "non-finite value in the fit or lambda");
  if (hs.flags & FLAG_RANKDEF) return fail(h, CPQR_ERANKDEF, "zero column norm or zero diagonal in R0/R_n");
  if (res->factors)
    for (int k = 0; k < N; ++k)
      if (res->factors[k])
        HIP_TRY(h, hipMemcpy(res->factors[k], p.A[k], (size_t)p.dims[k] * rank * 8, hipMemcpyDeviceToHost));
  if (res->lambda) HIP_TRY(h, hipMemcpy(res->lambda, p.lambda, (size_t)rank * 8, hipMemcpyDeviceToHost));
  if (res->q_factors)
    for (int k = 0; k < N; ++k) {
      if (!res->q_factors[k]) continue;
      const size_t n = (size_t)p.dims[k] * rank;
      if (p.f64) {
        HIP_TRY(h, hipMemcpy(res->q_factors[k], p.Q[k], n * 8, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> q(n);
        HIP_TRY(h, hipMemcpy(q.data(), p.Q[k], n * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i) res->q_factors[k][i] = (double)q[i];
      }
    }
  if (res->sweep_orders)
    for (int k = 0; k < done; ++k) {
      int u = 0;
      for (const Step& st : S->sched[k])
        if (st.kind == STEP_UPDATE) res->sweep_orders[k * N + (u++)] = st.mode;
    }
  res->fit = hs.fit;
  res->beta = hs.active ? hs.beta : 0.0;
  res->beta_sweep = hs.active ? hs.beta_sweep : 0;
  res->ttm_flops = S->ttm_flops;
  res->ttm_bytes = S->ttm_bytes;
  res->seconds = ms * 1e-3;
  const bool timing = (S->opts.flags & CPQR_FLAG_TIME_KERNELS) != 0;
  res->l1_ttm_seconds = l1_sec;
  res->l1_ttm_launches = timing ? (int)(S->evs.size() / 2) : 0;
  res->l1_ttm_bytes = S->l1_count ? S->l1_bytes / S->l1_count : 0.0;
  res->l1_ttm_flops = S->l1_count ? S->l1_flops / S->l1_count : 0.0;
  res->beta_learned = S->beta_learned;
  res->learned_fallback_sweep = S->fallback_sweep;
  for (int i = 0; i < 5; ++i) res->phase_seconds[i] = S->phase[i];
  res->fit_explicit = std::nan("");
  if (S->opts.flags & CPQR_FLAG_EXPLICIT_FIT) {
    std::vector<double*> fac(p.A.begin(), p.A.end());
    HIP_TRY(h, launch_residual(p.X, p.f64, N, p.dims.data(), fac.data(), p.lambda, rank, p.norm_part, s));
    const int nb = sumsq_blocks(S->nelem);
    std::vector<double> part(nb);
    HIP_TRY(h, hipMemcpyAsync(part.data(), p.norm_part, nb * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    double r2 = 0.0;
    for (double v : part) r2 += v;
    res->fit_explicit = 1.0 - std::sqrt(r2) / std::sqrt(hs.nx2);
  }
  return CPQR_OK;
}

cpqr_status cpqr_session_destroy(cpqr_session* S) {
  if (!S) return CPQR_EINVAL;
  cpqr_handle* h = S->h;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  delete S;
  h->busy = false;
  return CPQR_OK;
}

cpqr_status cpqr_als_qr(cpqr_handle* h, const cpqr_tensor* X, int rank, const cpqr_options* o,
                        cpqr_result* res) {
  if (!h) return CPQR_EINVAL;
  if (!res) return fail(h, CPQR_EINVAL, "null argument");
  cpqr_session* S = nullptr;
  cpqr_status st = cpqr_session_create(h, X, rank, o, &S);
  if (st != CPQR_OK) return st;
  st = cpqr_session_sweeps(S, o->iters);
  if (st == CPQR_OK) st = cpqr_session_result(S, res);
  else {
    // keep the per-sweep fits reached before the failure
    const std::string msg = h->err;
    cpqr_result tmp = *res;
    tmp.factors = nullptr;
    tmp.lambda = nullptr;
    tmp.q_factors = nullptr;
    (void)cpqr_session_result(S, &tmp);
    res->sweeps_done = tmp.sweeps_done;
    h->err = msg;
  }
  std::string msg = h->err;
  cpqr_session_destroy(S);
  h->err = msg;
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
namespace {

void count_ttm(cpqr_session* S, const std::vector<Step>& sw) {
  Problem& p = S->p;
  const uint32_t full = (1u << p.N) - 1u;
  for (const Step& st : sw)
    if (st.kind == STEP_TTM) {
      const int64_t in = inter_elems(p, st.src);
      const int64_t outn = in / p.dims[st.mode] * p.R;
      S->ttm_flops += 2.0 * in * p.R;
      S->ttm_bytes += (double)(in + outn) * p.elem;
      if (st.src == full) {
        S->l1_bytes += (double)(in + outn) * p.elem;
        S->l1_flops += 2.0 * in * p.R;
        ++S->l1_count;
      }
    }
}

// One batched launch of a sweep's step list, with the byte offsets of its
// argument arrays inside the sweep's argument blob.
struct BatchItem {
  int kind = 0;                 // 0 TTM, 1 TSQR, 2 Y*Q0, 3 finish, 4 staircase Z QR,
                                // 6 explicit Q_n after column-layout finishes, 7 zqr_col
  std::string tune_sig;         // TTM: identifies the step for the autotuner
  std::vector<int> members;     // problem indices
  TtmBatch tb{};
  TsqrBatch qb{};
  ApplyBatch ab{};
  int fin_rmax = 0, fin_rpt = 0;
  bool fin_col = false;         // kind 3: finish_col (fin_rpt = its rows per lane)
  int step = -1;                // kind 0: index of the TTM step in the sweep
  StairPlan sp{};
  ZcolPlan zp{};
  size_t off[3] = {0, 0, 0};
};

struct BatchRun {
  cpqr_handle* h = nullptr;
  std::vector<cpqr_session*> S;
  std::map<std::string, hipGraphExec_t> graphs;
  std::vector<hipEvent_t> fork_evs;   // fork/join events of the captured sweeps
  ~BatchRun() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : fork_evs) (void)hipEventDestroy(e);
    for (cpqr_session* x : S) delete x;
  }
};

template <typename T>
size_t blob_put(std::vector<char>& blob, const std::vector<T>& v) {
  const size_t off = (blob.size() + 63) & ~size_t(63);
  blob.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

// TTM launch shape of a group at K split ks and wpc workgroups per CU; false
// if some member cannot use it.
bool ttm_group_shape(const std::vector<TtmArgs>& args, int ks, int wpc, unsigned* wgs, size_t* lds) {
  *wgs = 1;
  *lds = 0;
  for (const TtmArgs& a : args) {
    int k = ks;
    unsigned w = 0;
    size_t l = 0;
    if (!ttm_batch_shape(a.L == 1 ? a.S : a.L * a.S, a.I, a.R, &k, &w, &l, wpc)) return false;
    if (w > *wgs) *wgs = w;
    if (l > *lds) *lds = l;
  }
  return true;
}

// Builds the launches of sweep k for every problem (grouped by the kernels'
// compile-time classes) and their argument blob.
void build_sweep_plan(BatchRun& B, int k, const std::vector<Step>& sw, const cpqr_options* o,
                      std::vector<BatchItem>* items, std::vector<char>* blob,
                      std::vector<std::vector<TtmArgs>>* ttm_host) {
  const int count = (int)B.S.size();
  const bool bf = o->prec == CPQR_PREC_BF16X3;
  int last_update = -1;
  for (size_t i = 0; i < sw.size(); ++i)
    if (sw[i].kind == STEP_UPDATE) last_update = (int)i;
  for (size_t i = 0; i < sw.size(); ++i) {
    const Step& st = sw[i];
    if (st.kind == STEP_TTM) {
      std::map<int, std::vector<int>> by_nb;
      for (int t = 0; t < count; ++t) by_nb[(B.S[t]->p.R + 15) / 16].push_back(t);
      for (auto& g : by_nb) {
        BatchItem it;
        it.kind = 0;
        it.members = g.second;
        std::vector<TtmArgs> args;
        bool vec = true, buf = true;
        for (int t : g.second) {
          args.push_back(ttm_step_args(B.S[t]->p, st));
          vec = vec && ttm_vec_legal(args.back());
          buf = buf && ttm_buf_legal(args.back());
        }
        std::vector<std::array<int64_t, 4>> shapes;
        for (const TtmArgs& a : args) shapes.push_back({a.L, (int64_t)a.I, a.S, (int64_t)a.R});
        it.tune_sig = ttm_key_batch(o->prec, g.first, args[0].L == 1, shapes);
        it.step = (int)i;
        it.tb.count = (int)args.size();
        it.tb.kc = args[0].L == 1;
        it.tb.vec = vec;
        it.tb.bf16x3 = bf;
        it.tb.buf = buf;
        it.tb.nb = g.first;
        TtmShape sh{1, 0};
        (void)handle_tune(B.h).find(it.tune_sig, &sh);
        it.tb.ks = sh.ks;
        if (!ttm_group_shape(args, it.tb.ks, sh.wpc, &it.tb.wgs, &it.tb.lds)) {
          it.tb.ks = 1;
          ttm_group_shape(args, 1, 0, &it.tb.wgs, &it.tb.lds);
        }
        it.off[0] = blob_put(*blob, args);
        ttm_host->push_back(args);
        items->push_back(it);
      }
    } else {
      const bool last = (int)i == last_update;
      std::vector<TsqrArgs> ts(count);
      std::vector<ApplyArgs> as(count);
      std::vector<FinishArgs> fs(count);
      // each problem's own alpha, switch_delta and fixed_beta (the batch
      // shares only the tree, extrapolation mode, precision and sweep count)
      for (int t = 0; t < count; ++t)
        update_args(B.S[t]->p, st.mode, k, last, &B.S[t]->opts, &ts[t], &as[t], &fs[t]);
      // column-distributed Z QR groups: its plan; staircase Z QR groups:
      // kernel shape; TSQR groups: rank class and plan
      std::map<std::pair<int, int>, std::vector<int>> zg;
      std::map<std::pair<int, int>, std::vector<int>> sg;
      std::map<std::tuple<int, int, int>, std::vector<int>> tg;
      for (int t = 0; t < count; ++t) {
        const ZcolPlan& zp = B.S[t]->p.zcol;
        if (zp.ok) {
          zg[{zp.rmax, zp.k}].push_back(t);
          continue;
        }
        const StairPlan& sp = B.S[t]->p.stair;
        if (sp.ok) {
          sg[{sp.rmax, sp.ns}].push_back(t);
          continue;
        }
        const TsqrPlan pl = tsqr_plan(ts[t].M, ts[t].R);
        tg[std::make_tuple(qr_rmax(ts[t].R), pl.leaf_rpt, pl.P > 1 ? pl.top_rpt : 0)].push_back(t);
      }
      // one launch per rank class and order: the group takes its largest
      // member's rows per lane (smaller members leave the extra rows zero)
      for (auto& g : zg) {
        BatchItem it;
        it.kind = 7;
        it.members = g.second;
        it.zp = B.S[g.second[0]]->p.zcol;
        for (int t : g.second)
          if (B.S[t]->p.zcol.rpl > it.zp.rpl) it.zp = B.S[t]->p.zcol;
        std::vector<ZcolArgs> za;
        for (int t : g.second) {
          const Problem& pp = B.S[t]->p;
          za.push_back(ZcolArgs{ts[t].N, ts[t].n, ts[t].R, ts[t].M, ts[t].rf, pp.smap, ts[t].R0, ts[t].Q0,
                                const_cast<double*>(as[t].meta_p), 1});
        }
        it.off[0] = blob_put(*blob, za);
        items->push_back(it);
      }
      for (auto& g : sg) {
        BatchItem it;
        it.kind = 4;
        it.members = g.second;
        it.sp = B.S[g.second[0]]->p.stair;
        std::vector<StairArgs> sa;
        for (int t : g.second) sa.push_back(stair_args(ts[t]));
        it.off[0] = blob_put(*blob, sa);
        items->push_back(it);
      }
      for (auto& g : tg) {
        BatchItem it;
        it.kind = 1;
        it.members = g.second;
        std::vector<LeafArgs> la;
        std::vector<TopArgs> ta;
        std::vector<FormArgs> fa;
        int Pmax = 1;
        unsigned chunks = 1;
        for (int t : g.second) {
          const TsqrPlan pl = tsqr_plan(ts[t].M, ts[t].R);
          LeafArgs l;
          TopArgs tp;
          FormArgs f;
          tsqr_args(ts[t], pl, &l, &tp, &f);
          la.push_back(l);
          ta.push_back(tp);
          fa.push_back(f);
          if (pl.P > Pmax) Pmax = pl.P;
          const unsigned c = (unsigned)((ts[t].M + 255) / 256);
          if (c > chunks) chunks = c;
        }
        it.qb = TsqrBatch{(int)g.second.size(), std::get<0>(g.first), std::get<1>(g.first),
                          std::get<2>(g.first), Pmax, std::get<2>(g.first) > 0 ? 1 : 0, chunks,
                          nullptr, nullptr, nullptr};
        it.off[0] = blob_put(*blob, la);
        it.off[1] = blob_put(*blob, ta);
        it.off[2] = blob_put(*blob, fa);
        items->push_back(it);
      }
      // Y*Q0 groups: rank class
      std::map<int, std::vector<int>> ag;
      for (int t = 0; t < count; ++t) ag[qr_rmax(as[t].R)].push_back(t);
      for (auto& g : ag) {
        BatchItem it;
        it.kind = 2;
        it.members = g.second;
        std::vector<ApplyDev> ad;
        unsigned ib = 1, nc = 1, rb = 1;
        for (int t : g.second) {
          ad.push_back(apply_dev(as[t]));
          ib = std::max(ib, apply_iblocks(as[t].I));
          nc = std::max(nc, (unsigned)as[t].nchunks);
          rb = std::max(rb, apply_reduce_blocks(as[t].I, as[t].R));
        }
        it.ab = ApplyBatch{(int)g.second.size(), g.first, false, ib, nc, rb, nullptr};
        it.off[0] = blob_put(*blob, ad);
        items->push_back(it);
      }
      // finish groups: the column-distributed kernel (factors of at most
      // 256 rows) by rank class and rows per lane, the row-distributed one
      // by rank class and rows per thread; then the explicit Q_n of the
      // column-layout groups (kind 6), which the next update's Z QR does not
      // wait for
      // (column-layout groups: one per rank class at the largest member's
      // rows per lane)
      std::map<std::tuple<int, int, int>, std::vector<int>> fg;
      std::map<int, int> col_rpl_max;
      for (int t = 0; t < count; ++t) {
        const int rm = qr_rmax(fs[t].R), cr = finish_col_rpl(fs[t].I);
        if (cr > 0 && fs[t].qn != nullptr) {
          fg[std::make_tuple(1, rm, 0)].push_back(t);
          col_rpl_max[rm] = std::max(col_rpl_max[rm], cr);
        } else {
          fg[std::make_tuple(0, rm, factor_rpt(fs[t].I))].push_back(t);
        }
      }
      std::vector<BatchItem> tails;
      for (auto& g : fg) {
        BatchItem it;
        it.kind = 3;
        it.members = g.second;
        std::vector<FinishArgs> fv;
        for (int t : g.second) fv.push_back(fs[t]);
        it.fin_col = std::get<0>(g.first) == 1;
        it.fin_rmax = std::get<1>(g.first);
        it.fin_rpt = it.fin_col ? col_rpl_max[it.fin_rmax] : std::get<2>(g.first);
        it.off[0] = blob_put(*blob, fv);
        items->push_back(it);
        if (it.fin_col) {
          BatchItem tl = it;
          tl.kind = 6;
          tails.push_back(tl);
        }
      }
      for (const BatchItem& tl : tails) items->push_back(tl);
    }
  }
}

hipError_t launch_item(const BatchItem& it, const char* base, hipStream_t s) {
  switch (it.kind) {
    case 0: {
      TtmBatch b = it.tb;
      b.args = reinterpret_cast<const TtmArgs*>(base + it.off[0]);
      return launch_ttm_f32_batched(b, s);
    }
    case 1: {
      TsqrBatch b = it.qb;
      b.leaf = reinterpret_cast<const LeafArgs*>(base + it.off[0]);
      b.top = reinterpret_cast<const TopArgs*>(base + it.off[1]);
      b.form = reinterpret_cast<const FormArgs*>(base + it.off[2]);
      return launch_tsqr_batched(b, s);
    }
    case 2: {
      ApplyBatch b = it.ab;
      b.args = reinterpret_cast<const ApplyDev*>(base + it.off[0]);
      return launch_apply_batched(b, s);
    }
    case 4:
      return launch_zqr_stair_batched(it.sp, (int)it.members.size(),
                                      reinterpret_cast<const StairArgs*>(base + it.off[0]), s);
    case 6:
      return launch_form_qn_batched((int)it.members.size(), it.fin_rmax,
                                    reinterpret_cast<const FinishArgs*>(base + it.off[0]), s);
    case 7:
      return launch_zqr_col_batched(it.zp, (int)it.members.size(),
                                    reinterpret_cast<const ZcolArgs*>(base + it.off[0]), s);
    default:
      if (it.fin_col)
        return launch_finish_col_batched((int)it.members.size(), it.fin_rmax, it.fin_rpt,
                                         reinterpret_cast<const FinishArgs*>(base + it.off[0]), s);
      return launch_finish_batched((int)it.members.size(), it.fin_rmax, it.fin_rpt,
                                   reinterpret_cast<const FinishArgs*>(base + it.off[0]), s);
  }
}

// Autotuner: for every TTM group not tuned yet, times the launch shapes that
// fit (K split 1, 2 or 4 waves per tile; 1 or 2 workgroups per CU) with
// outputs redirected to scratch memory, so that no cached intermediate is
// disturbed, and keeps the fastest (in the handle's table and its file).
cpqr_status tune_ttm(BatchRun& B, std::vector<BatchItem>& items,
                     const std::vector<std::vector<TtmArgs>>& ttm_host) {
  cpqr_handle* h = B.h;
  hipStream_t s = h->stream;
  TuneCache& tc = handle_tune(h);
  size_t ti = 0;
  for (BatchItem& it : items) {
    if (it.kind != 0) continue;
    const std::vector<TtmArgs>& args = ttm_host[ti++];
    TtmShape known;
    if (tc.find(it.tune_sig, &known)) {
      it.tb.ks = known.ks;
      if (!ttm_group_shape(args, known.ks, known.wpc, &it.tb.wgs, &it.tb.lds)) {
        it.tb.ks = 1;
        ttm_group_shape(args, 1, 0, &it.tb.wgs, &it.tb.lds);
      }
      continue;
    }
    std::vector<TtmArgs> scratch = args;
    size_t total = 0;
    for (const TtmArgs& a : args) total += (size_t)(a.L * a.S * a.R) * 4 + 256;
    char* out = nullptr;
    WS(h, "batch:tune_out", total, out);
    size_t pos = 0;
    for (TtmArgs& a : scratch) {
      a.out = reinterpret_cast<float*>(out + pos);
      pos += ((size_t)(a.L * a.S * a.R) * 4 + 255) & ~size_t(255);
    }
    TtmArgs* dargs = nullptr;
    WS(h, "batch:tune_args", scratch.size() * sizeof(TtmArgs), dargs);
    HIP_TRY(h, hipMemcpy(dargs, scratch.data(), scratch.size() * sizeof(TtmArgs), hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    TtmShape best{1, 0};
    float best_ms = 1e30f;
    for (int ks : {1, 2, 4})
      for (int wpc = 1; wpc <= 2; ++wpc) {
        TtmBatch b = it.tb;
        b.ks = ks;
        if (!ttm_group_shape(args, ks, wpc, &b.wgs, &b.lds)) continue;
        b.args = dargs;
        HIP_TRY(h, launch_ttm_f32_batched(b, s));
        HIP_TRY(h, hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) HIP_TRY(h, launch_ttm_f32_batched(b, s));
        HIP_TRY(h, hipEventRecord(e1, s));
        HIP_TRY(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = TtmShape{ks, wpc};
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tc.put(it.tune_sig, best);
    it.tb.ks = best.ks;
    ttm_group_shape(args, best.ks, best.wpc, &it.tb.wgs, &it.tb.lds);
  }
  tc.save();
  return CPQR_OK;
}

}  // namespace

extern "C" {

cpqr_status cpqr_als_qr_batched(cpqr_handle* h, int count, const cpqr_tensor* Xs, const int* ranks,
                                const cpqr_options* opts, cpqr_result* results) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (count < 1 || !Xs || !ranks || !opts || !results)
    return fail(h, CPQR_EINVAL, "batched: count >= 1 and non-null arrays required");
  if (h->busy) return fail(h, CPQR_EINVAL, "the handle already has a live session");
  const cpqr_options& o0 = opts[0];
  for (int t = 0; t < count; ++t) {
    cpqr_status v = check_args(h, &Xs[t], ranks[t], &opts[t]);
    if (v != CPQR_OK) {
      const std::string m = h->err;
      return fail(h, v, "batched problem %d: %s", t, m.c_str());
    }
    const cpqr_options& o = opts[t];
    if (Xs[t].order != Xs[0].order || o.tree != o0.tree || o.extrapolate != o0.extrapolate ||
        o.prec != o0.prec || o.iters != o0.iters)
      return fail(h, CPQR_EINVAL, "batched problem %d: order and options must match problem 0", t);
    if (o.tol != 0.0) return fail(h, CPQR_EINVAL, "batched runs a fixed number of sweeps: tol must be 0");
    // the batched driver factors Z_n of order >= 4 by the two-level TSQR
    if (!tsqr_plan(ipow(ranks[t], Xs[t].order - 1), ranks[t]).ok)
      return fail(h, CPQR_EUNSUPPORTED, "batched problem %d: R^(N-1) too large for the batched Z QR", t);
  }
  if (o0.prec == CPQR_PREC_FP64) return fail(h, CPQR_EUNSUPPORTED, "batched: FP32 or BF16X3 TTMs only");
  for (int t = 0; t < count; ++t)
    for (int k = 0; k < Xs[t].order; ++k)
      if (Xs[t].dims[k] > CPQR_MAX_FACTOR_ROWS)
        return fail(h, CPQR_EUNSUPPORTED, "batched problem %d: mode size > %d", t, CPQR_MAX_FACTOR_ROWS);
  if (o0.extrapolate == CPQR_EXTRAP_LEARNED)
    return fail(h, CPQR_EUNSUPPORTED, "batched: learned extrapolation is not supported");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  BatchRun B;
  B.h = h;
  h->busy = true;
  struct Unbusy { cpqr_handle* h; ~Unbusy() { h->busy = false; } } unbusy{h};
  for (int t = 0; t < count; ++t) {
    cpqr_session* S = nullptr;
    cpqr_status st = session_create_impl(h, &Xs[t], ranks[t], &opts[t], "b" + std::to_string(t) + ":", &S, true);
    if (st != CPQR_OK) {
      const std::string m = h->err;
      return fail(h, st, "batched problem %d: %s", t, m.c_str());
    }
    B.S.push_back(S);
  }
  for (cpqr_session* S : B.S) {
    HIP_TRY(h, hipEventRecord(S->t0, s));
    S->t0_recorded = true;
  }
  const auto& sched = B.S[0]->sched;
  for (int k = 1; k <= o0.iters; ++k) {
    const auto& sw = sched[k - 1];
    const std::string key = sweep_key(sw, k == 1 ? 2 : (k % 2), o0.extrapolate != 0);
    auto itg = B.graphs.find(key);
    if (itg == B.graphs.end()) {
      std::vector<BatchItem> items;
      std::vector<char> blob;
      std::vector<std::vector<TtmArgs>> ttm_host;
      build_sweep_plan(B, k, sw, &o0, &items, &blob, &ttm_host);
      cpqr_status ts = tune_ttm(B, items, ttm_host);
      if (ts != CPQR_OK) return ts;
      char* dblob = nullptr;
      WS(h, "batch:args:" + key, blob.size() + 64, dblob);
      HIP_TRY(h, hipMemcpy(dblob, blob.data(), blob.size(), hipMemcpyHostToDevice));
      // As in the single-problem sweep, each update's Z QR groups (kinds 1,
      // 4 and 7, contiguous in the plan) run beside the TTM groups of the
      // same update, forked after the previous update's finish groups and
      // joined before the update's first Y*Q0 group.  The groups of one
      // phase (the Z QR groups, the Y*Q0 groups, the finish groups, the Q_n
      // groups) are independent, one per kernel class, so each runs on a
      // branch of its own: the phase then takes as long as its slowest
      // group instead of their sum.
      // items i and j belong to one phase of independent groups
      auto same_phase = [&](size_t i, size_t j) {
        auto cls = [&](size_t x) { return items[x].kind == 4 || items[x].kind == 7 ? 1 : items[x].kind; };
        if (cls(i) != cls(j)) return false;
        return cls(i) != 0 || items[i].step == items[j].step;   // TTM groups of one step
      };
      size_t width = 1;
      for (size_t i = 0; i < items.size();) {
        size_t j = i + 1;
        while (j < items.size() && same_phase(i, j)) ++j;
        width = std::max(width, j - i);
        i = j;
      }
      bool bfork = (h->side != nullptr) ||
                   (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess);
      // the Z QR branches (h->side and pool[0, width - 1)) run beside the
      // main stream while the previous update's Q_n groups do: the other
      // phases take pool[width - 1, 2 width - 1)
      while (bfork && h->pool.size() + 1 < 2 * width) {
        hipStream_t q = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
          bfork = false;
          break;
        }
        h->pool.push_back(q);
      }
      if (!bfork) (void)hipGetLastError();
      // events: two per item are more than the branches can use
      std::vector<hipEvent_t> bev;
      if (bfork) {
        for (size_t r = 0; r < 2 * items.size() + 2; ++r) {
          hipEvent_t ev;
          HIP_TRY(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
          B.fork_evs.push_back(ev);
          bev.push_back(ev);
        }
      }
      const size_t ni = items.size();
      auto is_qr = [&](size_t i) { return items[i].kind == 1 || items[i].kind == 4 || items[i].kind == 7; };
      auto branch = [&](size_t r, bool qr) {
        return qr ? (r == 0 ? h->side : h->pool[r - 1]) : h->pool[width - 1 + r];
      };
      hipGraph_t g;
      HIP_TRY(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      size_t qr_end = 0, bnext = 0;   // end of the forked QR groups; next free event
      std::vector<hipEvent_t> joins;  // ends of the forked QR branches
      auto next_ev = [&]() -> hipEvent_t { return bnext < bev.size() ? bev[bnext++] : nullptr; };
      // items [j, j2) on branches of their own, forked from the main stream;
      // the events marking their ends are appended to *ends
      auto run_branches = [&](size_t j, size_t j2, bool qr, std::vector<hipEvent_t>* ends) -> hipError_t {
        hipEvent_t a = next_ev();
        if (!a) return hipErrorInvalidValue;
        hipError_t ee;
        if ((ee = hipEventRecord(a, s)) != hipSuccess) return ee;
        for (size_t q = j; q < j2; ++q) {
          hipStream_t br = branch(q - j, qr);
          hipEvent_t en = next_ev();
          if (!en) return hipErrorInvalidValue;
          if ((ee = hipStreamWaitEvent(br, a, 0)) != hipSuccess) return ee;
          if ((ee = launch_item(items[q], dblob, br)) != hipSuccess) return ee;
          if ((ee = hipEventRecord(en, br)) != hipSuccess) return ee;
          ends->push_back(en);
        }
        return hipSuccess;
      };
      auto fork_from = [&](size_t from) -> hipError_t {
        size_t j = from;
        while (j < ni && !is_qr(j) && items[j].kind != 2) ++j;
        if (j == ni || !is_qr(j)) return hipSuccess;
        size_t j2 = j;
        while (j2 < ni && is_qr(j2)) ++j2;
        qr_end = j2;
        return run_branches(j, j2, true, &joins);
      };
      if (bfork) e = fork_from(0);
      for (size_t i = 0; i < ni && e == hipSuccess;) {
        if (bfork && is_qr(i) && i < qr_end) {   // already on the side branches
          ++i;
          continue;
        }
        if (bfork && items[i].kind == 2 && !joins.empty()) {
          for (hipEvent_t je : joins)
            if ((e = hipStreamWaitEvent(s, je, 0)) != hipSuccess) break;
          joins.clear();
          if (e != hipSuccess) break;
        }
        // a run of independent groups of one phase: parallel branches
        size_t i2 = i + 1;
        if (bfork && (items[i].kind == 0 || items[i].kind == 2 || items[i].kind == 3 || items[i].kind == 6))
          while (i2 < ni && same_phase(i, i2)) ++i2;
        if (i2 - i > 1) {
          std::vector<hipEvent_t> ends;
          if ((e = run_branches(i, i2, false, &ends)) != hipSuccess) break;
          for (hipEvent_t en : ends)
            if ((e = hipStreamWaitEvent(s, en, 0)) != hipSuccess) break;
          if (e != hipSuccess) break;
        } else {
          if ((e = launch_item(items[i], dblob, s)) != hipSuccess) break;
        }
        if (bfork && items[i].kind == 3 && (i2 == ni || items[i2].kind != 3)) e = fork_from(i2);
        i = i2;
      }
      hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess) return fail(h, CPQR_EHIP, "batched launch during capture failed: %s", hipGetErrorString(e));
      if (e2 != hipSuccess) return fail(h, CPQR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
      hipGraphExec_t ge;
      hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess) return fail(h, CPQR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
      itg = B.graphs.emplace(key, ge).first;
    }
    HIP_TRY(h, hipGraphLaunch(itg->second, s));
    for (cpqr_session* S : B.S) {
      S->k = k;
      count_ttm(S, sw);
    }
  }
  HIP_TRY(h, hipStreamSynchronize(s));
  cpqr_status first = CPQR_OK;
  std::string first_msg;
  for (int t = 0; t < count; ++t) {
    cpqr_status st = cpqr_session_result(B.S[t], &results[t]);
    if (st != CPQR_OK && first == CPQR_OK) {
      first = st;
      first_msg = "batched problem " + std::to_string(t) + ": " + h->err;
    }
  }
  h->err = first_msg;
  return first;
}

// ---------------------------------------------------------------------- MLP
cpqr_status cpqr_mlp_forward(cpqr_handle* h, const float* w, const float* x, int n, float* y) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!w || !x || !y || n < 1) return fail(h, CPQR_EINVAL, "mlp_forward: null pointer or n < 1");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  float *dw, *dx, *dy;
  WS(h, "mlp:w", CPQR_MLP_PARAMS * sizeof(float), dw);
  WS(h, "mlp:x", (size_t)n * CPQR_MLP_FEATURES * sizeof(float), dx);
  WS(h, "mlp:y", (size_t)n * sizeof(float), dy);
  HIP_TRY(h, hipMemcpyAsync(dw, w, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(dx, x, (size_t)n * CPQR_MLP_FEATURES * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, launch_mlp_forward(dw, dx, n, dy, s));
  HIP_TRY(h, hipMemcpyAsync(y, dy, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  return CPQR_OK;
}

cpqr_status cpqr_mlp_grad(cpqr_handle* h, const float* w, const float* x, const float* y, int n,
                          float* loss, float* grad) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!w || !x || !y || !loss || !grad || n < 1) return fail(h, CPQR_EINVAL, "mlp_grad: null pointer or n < 1");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  const int chunks = mlp_grad_chunks(n, MLP_GRAD_PER_WAVE);
  float *dw, *dx, *dy, *part, *lpart, *dg, *dl;
  WS(h, "mlp:w", CPQR_MLP_PARAMS * sizeof(float), dw);
  WS(h, "mlp:x", (size_t)n * CPQR_MLP_FEATURES * sizeof(float), dx);
  WS(h, "mlp:y", (size_t)n * sizeof(float), dy);
  WS(h, "mlp:part", (size_t)chunks * CPQR_MLP_PARAMS * sizeof(float), part);
  WS(h, "mlp:lpart", (size_t)chunks * sizeof(float), lpart);
  WS(h, "mlp:g", (CPQR_MLP_PARAMS + 1) * sizeof(float), dg);
  dl = dg + CPQR_MLP_PARAMS;
  HIP_TRY(h, hipMemcpyAsync(dw, w, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(dx, x, (size_t)n * CPQR_MLP_FEATURES * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(dy, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, launch_mlp_grad(dw, dx, dy, nullptr, n, part, lpart, dg, dl, s));
  HIP_TRY(h, hipMemcpyAsync(grad, dg, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipMemcpyAsync(loss, dl, sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  return CPQR_OK;
}

cpqr_status cpqr_mlp_train(cpqr_handle* h, float* w, const float* x, const float* y, int n, int epochs,
                           int batch, float lr, uint64_t seed, float* loss_history) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!w || !x || !y || n < 1 || batch < 1 || epochs < 0)
    return fail(h, CPQR_EINVAL, "mlp_train: null pointer, n < 1, batch < 1 or epochs < 0");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  const int bmax = std::min(batch, n);
  const int chunks = std::max(mlp_grad_chunks(bmax, MLP_GRAD_PER_WAVE), mlp_grad_chunks(n, MLP_GRAD_PER_WAVE));
  float *dw, *dx, *dy, *part, *lpart, *dg, *dm, *dv;
  int* didx;
  WS(h, "mlp:w", CPQR_MLP_PARAMS * sizeof(float), dw);
  WS(h, "mlp:x", (size_t)n * CPQR_MLP_FEATURES * sizeof(float), dx);
  WS(h, "mlp:y", (size_t)n * sizeof(float), dy);
  WS(h, "mlp:part", (size_t)chunks * CPQR_MLP_PARAMS * sizeof(float), part);
  WS(h, "mlp:lpart", (size_t)chunks * sizeof(float), lpart);
  WS(h, "mlp:g", (CPQR_MLP_PARAMS + 1) * sizeof(float), dg);
  WS(h, "mlp:m", CPQR_MLP_PARAMS * sizeof(float), dm);
  WS(h, "mlp:v", CPQR_MLP_PARAMS * sizeof(float), dv);
  WS(h, "mlp:idx", (size_t)n * epochs * sizeof(int) + sizeof(int), didx);
  // seeded shuffles for every epoch (splitmix64 stream driving Fisher-Yates)
  std::vector<int> order((size_t)n * epochs);
  uint64_t st = seed;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  for (int e = 0; e < epochs; ++e) {
    int* o = order.data() + (size_t)e * n;
    for (int i = 0; i < n; ++i) o[i] = i;
    for (int i = n - 1; i > 0; --i) std::swap(o[i], o[next() % (uint64_t)(i + 1)]);
  }
  HIP_TRY(h, hipMemcpyAsync(dw, w, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(dx, x, (size_t)n * CPQR_MLP_FEATURES * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(dy, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
  if (epochs > 0)
    HIP_TRY(h, hipMemcpyAsync(didx, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(h, hipMemsetAsync(dm, 0, CPQR_MLP_PARAMS * sizeof(float), s));
  HIP_TRY(h, hipMemsetAsync(dv, 0, CPQR_MLP_PARAMS * sizeof(float), s));
  std::vector<float> losses(epochs > 0 ? epochs : 1);
  int t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int b0 = 0; b0 < n; b0 += bmax) {
      const int nb = std::min(bmax, n - b0);
      HIP_TRY(h, launch_mlp_grad(dw, dx, dy, didx + (size_t)e * n + b0, nb, part, lpart, dg,
                                 dg + CPQR_MLP_PARAMS, s));
      HIP_TRY(h, launch_mlp_adam(dw, dg, dm, dv, ++t, lr, 0.9f, 0.999f, 1e-8f, s));
    }
    // loss over all rows after the epoch
    HIP_TRY(h, launch_mlp_grad(dw, dx, dy, nullptr, n, part, lpart, dg, dg + CPQR_MLP_PARAMS, s));
    HIP_TRY(h, hipMemcpyAsync(&losses[e], dg + CPQR_MLP_PARAMS, sizeof(float), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(h, hipMemcpyAsync(w, dw, CPQR_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  if (loss_history)
    for (int e = 0; e < epochs; ++e) loss_history[e] = losses[e];
  return CPQR_OK;
}

}  // extern "C"
