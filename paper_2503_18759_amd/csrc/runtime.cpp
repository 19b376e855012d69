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

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cpqr.h"
#include "kernels.h"
#include "schedule.h"

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
  std::string err;
  std::map<std::string, DevBuf> bufs;
  bool busy = false;                  // a session is using the workspace
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

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Everything one decomposition needs on the device.
struct Problem {
  int N = 0, R = 0, prec = CPQR_PREC_FP32;
  std::vector<int64_t> dims;
  const void* X = nullptr;
  bool f64 = false;
  size_t elem = 4;
  int64_t M = 0;          // R^(N-1) rows of Z_n
  int P = 0;              // TSQR leaves
  int64_t leaf_rows = 0;
  int nchunks_max = 0;
  int Imax = 0;
  // device pointers
  std::vector<double*> A;      // factors (float64)
  std::vector<void*> Q;        // explicit Q_n in the TTM precision
  double* rf = nullptr;        // N x R x R R factors
  double* lambda = nullptr;
  std::vector<double*> q0buf;  // per mode: 2 x M x R (ping-pong)
  double *tV = nullptr, *tT = nullptr, *tStack = nullptr, *tQtop = nullptr, *R0 = nullptr;
  double *partial = nullptr, *Vbuf = nullptr;
  DevState* state = nullptr;
  double* fit_hist = nullptr;
  double* norm_part = nullptr;
  std::map<uint32_t, void*> inter;   // intermediates by free-mode mask
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
  std::vector<hipEvent_t> evs;
  std::map<std::string, hipGraphExec_t> graphs;
  ~cpqr_session() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
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
    WS(h, "A" + std::to_string(k), (size_t)p.dims[k] * R * 8, p.A[k]);
    WS(h, "Q" + std::to_string(k), (size_t)p.dims[k] * R * p.elem, p.Q[k]);
    if (p.dims[k] > p.Imax) p.Imax = (int)p.dims[k];
  }
  WS(h, "rf", (size_t)N * R * R * 8, p.rf);
  WS(h, "lambda", (size_t)R * 8, p.lambda);
  p.M = ipow(R, N - 1);
  const TsqrPlan pl = tsqr_plan(p.M, R);
  if (!pl.ok) return fail(h, CPQR_EUNSUPPORTED, "no TSQR plan for %lld x %d", (long long)p.M, R);
  p.leaf_rows = pl.leaf_rows;
  p.P = pl.P;
  for (int k = 0; k < N; ++k) WS(h, "q0_" + std::to_string(k), (size_t)2 * p.M * R * 8, p.q0buf[k]);
  WS(h, "tsqrV", (size_t)p.P * p.leaf_rows * R * 8, p.tV);
  WS(h, "tsqrT", (size_t)p.P * R * R * 8, p.tT);
  WS(h, "tsqrS", (size_t)p.P * R * R * 8, p.tStack);
  WS(h, "tsqrQ", (size_t)p.P * R * R * 8, p.tQtop);
  WS(h, "R0", (size_t)R * R * 8, p.R0);
  int nch = 1;
  for (int k = 0; k < N; ++k) {
    const int c = apply_num_chunks(p.M, (int)p.dims[k]);
    if (c > nch) nch = c;
  }
  p.nchunks_max = nch;
  WS(h, "partial", (size_t)nch * 2 * p.Imax * R * 8, p.partial);
  WS(h, "V", (size_t)2 * p.Imax * R * 8, p.Vbuf);
  WS(h, "state", sizeof(DevState), p.state);
  WS(h, "fit_hist", (size_t)(iters > 0 ? iters : 1) * 8, p.fit_hist);
  WS(h, "norm_part", 4096 * 8, p.norm_part);
  // intermediates used by the schedule
  const uint32_t full = (1u << N) - 1u;
  for (const auto& sw : sched)
    for (const Step& st : sw)
      if (st.kind == STEP_TTM) {
        const uint32_t dst = st.src & ~(1u << st.mode);
        if (!p.inter.count(dst)) {
          void* ptr = nullptr;
          WS(h, "Y" + std::to_string(dst), (size_t)inter_elems(p, dst) * p.elem, ptr);
          p.inter[dst] = ptr;
        }
      }
  (void)full;
  return CPQR_OK;
}

hipError_t launch_ttm_step(const Problem& p, const Step& st, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr) {
  const uint32_t full = (1u << p.N) - 1u;
  const void* in = (st.src == full) ? p.X : p.inter.at(st.src);
  void* out = p.inter.at(st.src & ~(1u << st.mode));
  int64_t L = 1, S = 1;
  for (int k = 0; k < p.N; ++k) {
    const int64_t d = (st.src & (1u << k)) ? p.dims[k] : p.R;
    if (k < st.mode) L *= d;
    if (k > st.mode) S *= d;
  }
  const int I = (int)p.dims[st.mode];
  if (p.f64)
    return launch_ttm_f64((const double*)in, (const double*)p.Q[st.mode], (double*)out, L, I, S, p.R, s,
                          ev0, ev1);
  return launch_ttm_f32((const float*)in, (const float*)p.Q[st.mode], (float*)out, L, I, S, p.R,
                        p.prec == CPQR_PREC_BF16X3, s, ev0, ev1);
}

hipError_t launch_update(const Problem& p, int n, int sweep_k, bool last, const cpqr_options* o,
                         hipStream_t s) {
  const int R = p.R;
  double* q0cur = p.q0buf[n] + (size_t)(sweep_k % 2) * p.M * R;
  double* q0prev = (sweep_k >= 2) ? p.q0buf[n] + (size_t)((sweep_k - 1) % 2) * p.M * R : nullptr;
  TsqrArgs t;
  t.N = p.N;
  t.n = n;
  t.R = R;
  t.rf = p.rf;
  t.src = nullptr;
  t.M = p.M;
  t.P = p.P;
  t.V = p.tV;
  t.T = p.tT;
  t.stack = p.tStack;
  t.R0 = p.R0;
  t.Qtop = p.tQtop;
  t.Q0 = q0cur;
  hipError_t e = launch_tsqr(t, s);
  if (e != hipSuccess) return e;
  ApplyArgs a;
  a.Y = p.inter.at(1u << n);
  a.y_f64 = p.f64;
  a.L = ipow(R, n);
  a.I = (int)p.dims[n];
  a.S = ipow(R, p.N - 1 - n);
  a.R = R;
  a.Q0 = q0cur;
  a.Q0prev = (o->extrapolate == CPQR_EXTRAP_PAPER) ? q0prev : nullptr;
  a.partial = p.partial;
  a.V = p.Vbuf;
  a.nchunks = apply_num_chunks(p.M, a.I);
  a.state = p.state;
  e = launch_apply(a, s);
  if (e != hipSuccess) return e;
  FinishArgs f;
  f.I = (int)p.dims[n];
  f.R = R;
  f.V = p.Vbuf;
  f.R0 = p.R0;
  f.A = p.A[n];
  f.lambda = p.lambda;
  f.Rn = p.rf + (size_t)n * R * R;
  f.q64 = p.f64 ? (double*)p.Q[n] : nullptr;
  f.q32 = p.f64 ? nullptr : (float*)p.Q[n];
  f.state = p.state;
  f.fit_hist = p.fit_hist;
  f.alpha = o->alpha;
  f.delta = o->switch_delta;
  f.fixed_beta = o->fixed_beta;
  f.extrap = o->extrapolate;
  f.last_in_sweep = last ? 1 : 0;
  return launch_finish(f, s);
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
  if (o->extrapolate < 0 || o->extrapolate > 1) return fail(h, CPQR_EINVAL, "bad extrapolation mode");
  if (o->prec < 0 || o->prec > 2) return fail(h, CPQR_EINVAL, "bad precision");
  if (X->dtype != CPQR_DTYPE_F32 && X->dtype != CPQR_DTYPE_F64) return fail(h, CPQR_EINVAL, "bad dtype");
  if ((o->prec == CPQR_PREC_FP64) != (X->dtype == CPQR_DTYPE_F64))
    return fail(h, CPQR_EINVAL, "FP64 precision needs a float64 tensor; FP32/BF16X3 need float32");
  if (!(o->tol >= 0.0) || !(o->alpha == o->alpha) || !(o->switch_delta >= 0.0) || !(o->fixed_beta >= 0.0))
    return fail(h, CPQR_EINVAL, "bad tol/alpha/switch_delta/fixed_beta");
  if (!o->init_factors) return fail(h, CPQR_EINVAL, "init_factors is required");
  for (int k = 0; k < N; ++k) {
    if (X->dims[k] < 1) return fail(h, CPQR_EINVAL, "dims must be >= 1");
    if (!o->init_factors[k]) return fail(h, CPQR_EINVAL, "null init factor %d", k);
  }
  if (rank > 32) return fail(h, CPQR_EUNSUPPORTED, "rank > 32 is not supported by this build");
  for (int k = 0; k < N; ++k) {
    if (X->dims[k] < rank) return fail(h, CPQR_EUNSUPPORTED, "mode %d has size %lld < rank %d", k, (long long)X->dims[k], rank);
    if (X->dims[k] > CPQR_MAX_FACTOR_ROWS)
      return fail(h, CPQR_EUNSUPPORTED, "mode size > %d is not supported by this build", CPQR_MAX_FACTOR_ROWS);
  }
  if (N > qr_max_order(rank) || !tsqr_plan(ipow(rank, N - 1), rank).ok)
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
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return CPQR_OK;
}

const char* cpqr_last_error(const cpqr_handle* h) { return h ? h->err.c_str() : ""; }

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
      return fail(h, CPQR_EUNSUPPORTED, "bf16x3 TTM needs rank <= 64 and I * roundup(R,16) * 4 <= 64 KiB");
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

cpqr_status cpqr_session_create(cpqr_handle* h, const cpqr_tensor* X, int rank,
                                const cpqr_options* o, cpqr_session** out) {
  if (!h) return CPQR_EINVAL;
  h->err.clear();
  if (!out) return fail(h, CPQR_EINVAL, "null session pointer");
  *out = nullptr;
  {
    cpqr_status v = check_args(h, X, rank, o);
    if (v != CPQR_OK) return v;
  }
  if (h->busy) return fail(h, CPQR_EINVAL, "the handle already has a live session");
  const int N = X->order;
  std::unique_ptr<cpqr_session> ss(new cpqr_session());
  cpqr_session& S = *ss;
  S.h = h;
  S.opts = *o;
  S.opts.init_factors = nullptr;
  if (!build_schedule(N, o->tree, o->iters, S.sched) || !validate_schedule(N, S.sched))
    return fail(h, CPQR_EINVAL, "schedule construction failed");
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, order_after_user(h));
  hipStream_t s = h->stream;
  Problem& p = S.p;
  p.N = N;
  p.R = rank;
  p.prec = o->prec;
  p.dims.assign(X->dims, X->dims + N);
  p.X = X->data;
  p.f64 = (o->prec == CPQR_PREC_FP64);
  p.elem = p.f64 ? 8 : 4;
  cpqr_status stt = setup(h, p, o->iters, S.sched);
  if (stt != CPQR_OK) return stt;
  S.nelem = 1;
  for (int k = 0; k < N; ++k) S.nelem *= p.dims[k];
  // ||X||^2 and the device state
  HIP_TRY(h, launch_sumsq(p.X, p.f64, S.nelem, p.norm_part, s));
  HIP_TRY(h, launch_state_init(p.state, p.norm_part, sumsq_blocks(S.nelem), s));
  // initial factors and their QRs (Algorithm 2, "Initialize")
  for (int k = 0; k < N; ++k) {
    HIP_TRY(h, hipMemcpyAsync(p.A[k], o->init_factors[k], (size_t)p.dims[k] * rank * 8,
                              hipMemcpyHostToDevice, s));
    HIP_TRY(h, launch_factor_qr((int)p.dims[k], rank, p.A[k], p.rf + (size_t)k * rank * rank,
                                p.f64 ? (double*)p.Q[k] : nullptr, p.f64 ? nullptr : (float*)p.Q[k], s));
  }
  DevState hs;
  HIP_TRY(h, hipMemcpyAsync(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  if (!(hs.nx2 > 0.0)) {
    if (hs.flags & FLAG_NONFINITE) return fail(h, CPQR_ENONFINITE, "tensor contains NaN or Inf");
    return fail(h, CPQR_EINVAL, "||X|| = 0");
  }
  S.nx2 = hs.nx2;
  HIP_TRY(h, hipEventCreate(&S.t0));
  HIP_TRY(h, hipEventCreate(&S.t1));
  h->busy = true;
  *out = ss.release();
  return CPQR_OK;
}

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
  const int N = p.N;
  const bool timing = (o->flags & CPQR_FLAG_TIME_KERNELS) != 0;
  const bool use_graph = !timing && !(o->flags & CPQR_FLAG_NO_GRAPH);
  const uint32_t full = (1u << N) - 1u;
  if (!S->t0_recorded) {
    HIP_TRY(h, hipEventRecord(S->t0, s));
    S->t0_recorded = true;
  }
  for (int it = 0; it < nsweeps; ++it) {
    const int k = S->k + 1;
    const auto& sw = S->sched[k - 1];
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
    int last_update = -1;
    for (size_t i = 0; i < sw.size(); ++i)
      if (sw[i].kind == STEP_UPDATE) last_update = (int)i;
    auto enqueue = [&](hipStream_t q) -> hipError_t {
      for (size_t i = 0; i < sw.size(); ++i) {
        const Step& st = sw[i];
        hipError_t e;
        if (st.kind == STEP_TTM) {
          if (timing && st.src == full) {
            hipEvent_t a, b;
            if ((e = hipEventCreate(&a)) != hipSuccess) return e;
            if ((e = hipEventCreate(&b)) != hipSuccess) return e;
            S->evs.push_back(a);
            S->evs.push_back(b);
            // events stamped by the kernel dispatch itself (start and end of the kernel)
            if ((e = launch_ttm_step(p, st, q, a, b)) != hipSuccess) return e;
          } else {
            if ((e = launch_ttm_step(p, st, q)) != hipSuccess) return e;
          }
        } else {
          if ((e = launch_update(p, st.mode, k, (int)i == last_update, o, q)) != hipSuccess) return e;
        }
      }
      return hipSuccess;
    };
    if (use_graph) {
      // sweeps with the same step list and Q0 ping-pong parity share a graph
      const std::string key = sweep_key(sw, k == 1 ? 2 : (k % 2), o->extrapolate != 0);
      auto itg = S->graphs.find(key);
      if (itg == S->graphs.end()) {
        hipGraph_t g;
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
      HIP_TRY(h, hipGraphLaunch(itg->second, s));
    } else {
      hipError_t e = enqueue(s);
      if (e != hipSuccess) return fail(h, CPQR_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    S->k = k;
    if (o->tol > 0.0 && k >= 2) {
      DevState hs;
      HIP_TRY(h, hipMemcpyAsync(&hs, p.state, sizeof(DevState), hipMemcpyDeviceToHost, s));
      double fk[2];
      HIP_TRY(h, hipMemcpyAsync(fk, p.fit_hist + (k - 2), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(h, hipStreamSynchronize(s));
      if (hs.flags || std::fabs(fk[1] - fk[0]) < o->tol) {
        S->stopped = true;
        break;
      }
    }
  }
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
    l1_sec += e * 1e-3;
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
