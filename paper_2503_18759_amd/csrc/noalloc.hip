// cpqr_qr_noalloc: the compact Householder QR of cpqr_qr (Section 2.4) for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  The two-level TSQR
// keeps its scratch (reflectors V, the T factors, the stack of leaf
// triangles and the explicit Q of the stack) in a file-scope device array
// instead of handle workspace; the caller passes A, Q and R.
//
// The array is a host-side stand-in in host code: its device address is
// looked up once per device with hipGetSymbolAddress (on the first call on
// that device, with that device current) and only that address is passed to
// the kernels.  Every call on one device shares that device's array, so calls
// that overlap on one device (two streams, or two host threads) race.  The
// TSQR writes every scratch entry before it reads it, so nothing needs to be
// cleared between calls.
#include <mutex>
#include <string>

#include "../../include/cpqr.h"
#include "common.h"
#include "kernels.h"

namespace {

// 4 MiB of float64: for 17 <= R <= 32 every size the two-level TSQR takes
// (M <= 8192 at R = 32); M <= 29,696 at R = 16 and M <= 59,904 at R = 8.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = CPQR_QR_NOALLOC_SCRATCH_BYTES / 8;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

thread_local std::string g_err;

cpqr_status fail(cpqr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

namespace cpqr {
// Message of the last failed cpqr_qr_noalloc call on this host thread (read
// through cpqr_last_error(NULL)).
const char* noalloc_last_error() { return g_err.c_str(); }
}  // namespace cpqr

extern "C" {

cpqr_status cpqr_qr_noalloc(int64_t M, int R, const double* A, double* Q, double* Rout, void* hip_stream) {
  g_err.clear();
  if (!A || !Q || !Rout) return fail(CPQR_EINVAL, "null pointer");
  if (R < 1 || M < R) return fail(CPQR_EINVAL, "need 1 <= R <= M");
  if (R > 32) return fail(CPQR_EUNSUPPORTED, "R > 32");
  const cpqr::TsqrPlan pl = cpqr::tsqr_plan(M, R);
  if (!pl.ok) return fail(CPQR_EUNSUPPORTED, "M too large for a two-level TSQR at this R");
  const int64_t P = pl.P, leaf = pl.leaf_rows;
  const int64_t nV = P * leaf * R, nT = P * R * R;
  const int64_t need = nV + 3 * nT;
  if (need > NOALLOC_SCRATCH_DOUBLES)
    return fail(CPQR_EUNSUPPORTED,
                "scratch of " + std::to_string(need * 8) + " bytes needed for M = " + std::to_string(M) +
                    ", R = " + std::to_string(R) + "; the no-allocation QR holds " +
                    std::to_string((long long)CPQR_QR_NOALLOC_SCRATCH_BYTES) + " bytes per device");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CPQR_EHIP, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CPQR_EUNSUPPORTED, "device index beyond 63");
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(CPQR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      }
      g_ptr[dev] = static_cast<double*>(p);
    }
    base = g_ptr[dev];
  }
  cpqr::TsqrArgs t;
  t.N = 0;
  t.n = 0;
  t.R = R;
  t.rf = nullptr;
  t.src = A;
  t.M = M;
  t.P = (int)P;
  t.V = base;
  t.T = base + nV;
  t.stack = base + nV + nT;
  t.Qtop = base + nV + 2 * nT;
  t.R0 = Rout;
  t.Q0 = Q;
  const hipError_t e = cpqr::launch_tsqr(t, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CPQR_EHIP, std::string("TSQR launch: ") + hipGetErrorString(e));
  }
  return CPQR_OK;
}

}  // extern "C"
