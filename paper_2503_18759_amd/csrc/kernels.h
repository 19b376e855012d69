// Internal launcher interface between the runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CPQR_MAX_ORDER 7
#define CPQR_MAX_FACTOR_ROWS 512   // largest mode size I_n handled by the factor QR kernels

namespace cpqr {

// Device-resident sweep state.  Written only by the kernels of a mode update
// so that whole sweeps can be replayed from a HIP graph without host reads.
struct DevState {
  double nx2;       // ||X||_F^2
  double beta;      // extrapolation weight (valid when active)
  double vpvu;      // <Vp, Vu> of the last mode update
  double vuvu;      // ||Vu||^2 of the last mode update
  double fit;       // fit after the last completed sweep
  int active;       // extrapolation active
  int beta_sweep;   // 1-based sweep after which beta was activated
  int sweep;        // number of completed sweeps
  int flags;        // error bits: 1 = zero lambda / R diagonal, 2 = non-finite
};

enum { FLAG_RANKDEF = 1, FLAG_NONFINITE = 2 };

// --- TTM ------------------------------------------------------------------
bool ttm_mfma_supported(int I, int R);
hipError_t launch_ttm_f32(const float* in, const float* Q, float* out, int64_t L, int I, int64_t S,
                          int R, bool bf16x3, hipStream_t st);
hipError_t launch_ttm_f64(const double* in, const double* Q, double* out, int64_t L, int I,
                          int64_t S, int R, hipStream_t st);

// --- QR -------------------------------------------------------------------
int qr_rmax(int R);
int64_t qr_leaf_rows(int R);   // largest TSQR leaf at rank R
// TSQR of an M x R matrix: leaves of leaf_rows rows (leaf_rpt rows per
// thread), P leaves, and a top block of top_rpt rows per thread (P > 1).
struct TsqrPlan {
  bool ok;
  int leaf_rpt;
  int64_t leaf_rows;
  int P;
  int top_rpt;
};
TsqrPlan tsqr_plan(int64_t M, int R);
int factor_rpt(int I);
int qr_max_order(int R);   // largest order whose Khatri-Rao QR fits the kernels at rank R

struct TsqrArgs {
  int N, n, R;          // order, skipped mode (Khatri-Rao source), rank
  const double* rf;     // N x R x R column-major R factors (Khatri-Rao source) or null
  const double* src;    // explicit M x R source matrix or null
  int64_t M;            // rows
  int P;                // number of leaves = ceil(M / leaf_rows)
  double* V;            // (P * leaf_rows) x R reflectors
  double* T;            // P x R x R
  double* stack;        // (P * R) x R leaf triangles
  double* R0;           // R x R output
  double* Qtop;         // (P * R) x R
  double* Q0;           // M x R output (explicit Q)
};
hipError_t launch_tsqr(const TsqrArgs& t, hipStream_t st);
hipError_t launch_factor_qr(int I, int R, const double* A, double* Rn, double* q64, float* q32,
                            hipStream_t st);

// --- mode update ------------------------------------------------------------
struct ApplyArgs {
  const void* Y;        // leaf Y{n}: float or double
  bool y_f64;
  int64_t L;            // R^n  (0-based n)
  int I;                // I_n
  int64_t S;            // R^(N-1-n)
  int R;
  const double* Q0;     // M x R
  const double* Q0prev; // M x R or null
  double* partial;      // nchunks x 2 x I x R
  double* V;            // 2 x I x R reduced [Vp | Vq]
  int nchunks;
  const DevState* state;
};
int apply_num_chunks(int64_t M, int I);
hipError_t launch_apply(const ApplyArgs& a, hipStream_t st);

struct FinishArgs {
  int I, R;
  const double* V;      // 2 x I x R  [Vp | Vq]
  const double* R0;     // R x R
  double* A;            // I x R factor out (float64)
  double* lambda;       // R out
  double* Rn;           // R x R out
  double* q64;          // I x R explicit Q (float64) or null
  float* q32;           // I x R explicit Q (float32) or null
  DevState* state;
  double* fit_hist;     // iters
  double alpha;
  double delta;
  double fixed_beta;    // > 0: use from sweep 2 on
  int extrap;           // 0 off, 1 paper
  int last_in_sweep;
};
hipError_t launch_finish(const FinishArgs& f, hipStream_t st);

// --- norms ----------------------------------------------------------------
// partial sums of squares into `part` (nblocks doubles); returns nblocks
int sumsq_blocks(int64_t n);
hipError_t launch_sumsq(const void* x, bool f64, int64_t n, double* part, hipStream_t st);
hipError_t launch_state_init(DevState* s, const double* part, int nparts, hipStream_t st);
hipError_t launch_residual(const void* x, bool f64, int N, const int64_t* dims_host,
                           double* const* factors, const double* lambda, int R, double* part,
                           hipStream_t st);

}  // namespace cpqr
