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
// ev0/ev1 (optional): events stamped with the kernel's own start and end
// (hipExtLaunchKernel), used to time single TTM launches.  ks: waves per
// output tile (K split 1, 2 or 4); 0, or a split this shape cannot use,
// takes the launcher's own choice.  wpc: workgroups per CU of the persistent
// grid (1 or 2; 0: the default, 2).
hipError_t launch_ttm_f32(const float* in, const float* Q, float* out, int64_t L, int I, int64_t S,
                          int R, bool bf16x3, hipStream_t st, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr, int ks = 0, int wpc = 0);
// K splits a float32 MFMA TTM of this shape can use (bit k set: split 1 << k).
unsigned ttm_ks_options(int64_t L, int I, int64_t S, int R);
hipError_t launch_ttm_f64(const double* in, const double* Q, double* out, int64_t L, int I,
                          int64_t S, int R, hipStream_t st, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);

// Batched float32 TTM: one launch over `count` problems (grid.y = problem).
// Every problem has the same layout class (L == 1 for all or for none) and
// ranks in the same 16-column class; `args` lives in device memory.
struct TtmArgs {
  const float* in;
  const float* Q;
  float* out;
  int64_t L, S;
  int I, R;
};
struct TtmBatch {
  int count;
  bool kc;          // L == 1 for every problem
  bool vec;         // 16-byte loads legal for every problem
  bool bf16x3;
  bool buf;         // every input below 2 GiB (buffer-resource loads)
  int nb;           // 16-column blocks (max rank / 16, rounded up)
  int ks;           // K split across the waves of a workgroup
  unsigned wgs;     // workgroups per problem (max over problems)
  size_t lds;       // bytes of LDS (max over problems)
  const TtmArgs* args;
};
// Host helper for building a TtmBatch: workgroups and LDS bytes for one
// problem of `rows` output rows at K split `ks` (0: the launcher's own
// choice, returned in *ks) and `wpc` workgroups per CU (0: default).  False
// if that split does not fit.
bool ttm_batch_shape(int64_t rows, int I, int R, int* ks, unsigned* wgs, size_t* lds, int wpc = 0);
hipError_t launch_ttm_f32_batched(const TtmBatch& b, hipStream_t st);
bool ttm_vec_legal(const TtmArgs& a);   // 16-byte loads (and stores) legal for this problem
bool ttm_buf_legal(const TtmArgs& a);   // input addressable through a buffer resource

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
// Message of the last failed cpqr_qr_noalloc call on this host thread.
const char* noalloc_last_error();

// Per-problem arguments of the TSQR kernels (one entry per problem of a
// batch; a single problem passes its entry by value).
struct LeafArgs {
  int N, n, R, P;             // order, skipped mode, rank, leaves of this problem
  const double* rf;           // N x R x R R factors or null
  const double* src;          // explicit M x R matrix or null
  int64_t M, ldv, ldstack;    // rows, leading dims of V and of the leaf-triangle stack
  double *V, *T, *stack;
  double *R0, *Qtop;          // non-null: single leaf, write R0 and the trivial Qtop
};
struct TopArgs {
  int R, active;              // active == 0: nothing to do (single leaf)
  int64_t rows;               // P * R
  const double* stack;
  double *R0, *Qtop;
};
struct FormArgs {
  int R, leaf_rows;
  int64_t M, ldv, ldq;
  const double *V, *T, *Qtop;
  double* Q0;
};
// Batched TSQR over `count` problems of one rank class (rmax) and one plan
// (leaf_rpt, top_rpt, Pmax leaves, chunks = max form_q0 workgroups); the
// argument arrays live in device memory.
struct TsqrBatch {
  int count, rmax, leaf_rpt, top_rpt, Pmax, any_top;
  unsigned chunks;
  const LeafArgs* leaf;
  const TopArgs* top;
  const FormArgs* form;
};
hipError_t launch_tsqr_batched(const TsqrBatch& b, hipStream_t st);
void tsqr_args(const TsqrArgs& t, const TsqrPlan& pl, LeafArgs* la, TopArgs* ta, FormArgs* fa);
// Khatri-Rao QR of Z_n in one workgroup, rows in staircase order (largest
// digit first).  Used when Z_n has at most 256 rows, or when its rows beyond
// the first 256 fit the narrow slices of an instantiated shape.
struct StairPlan {
  bool ok;
  int rmax;       // columns of slice 0
  int ns;         // narrow slices (0: all rows in slice 0)
};
StairPlan stair_plan(int N, int R);
struct StairArgs {
  int N, n, R;          // order, skipped mode, rank
  int64_t M;            // R^(N-1) rows of Z_n
  const double* rf;     // N x R x R column-major R factors
  double* R0;           // R x R output (column-major, diag >= 0)
  double* Q0;           // M x R output (column-major, Kolda row order)
  int active;           // 0: nothing to do (batched entries of other plans)
};
hipError_t launch_zqr_stair(const StairPlan& pl, const StairArgs& a, hipStream_t st);
hipError_t launch_zqr_stair_batched(const StairPlan& pl, int count, const StairArgs* args, hipStream_t st);
// Khatri-Rao QR of Z_n (at most 1024 rows) in the column-distributed layout,
// written in the compact form Q0 = (E - V T V1^T) D: V (M x R, Kolda rows),
// R0 (R x R, diag >= 0) and meta = [Md = T V1^T D (R x R), D (R), piv (R)].
struct ZcolPlan {
  bool ok;
  int rmax;     // column class
  int rpl;      // rows per lane (64-row chunks of the staircase)
  int nw;       // waves (4 or 8)
  int k;        // other modes (N - 1)
};
ZcolPlan zcol_plan(int N, int R);
struct ZcolArgs {
  int N, n, R;          // order, skipped mode, rank
  int64_t M;            // R^(N-1) rows of Z_n
  const double* rf;     // N x R x R column-major R factors
  const int* smap;      // M x 2 ints: Kolda row and packed digits of staircase row s
  double* R0;           // R x R out
  double* V;            // M x R out (Kolda row order)
  double* meta;         // R^2 + 2R doubles out
  int active;           // 0: nothing to do (batched entries of other plans)
  const double* rf_hi;  // non-null: the last remaining factor (the slowest digit) from here
};
// Staircase row table (host): out[2s] = Kolda row, out[2s+1] = digits (5 bits each).
void stair_table(int R, int K, int64_t M, int* out);
hipError_t launch_zqr_col(const ZcolPlan& pl, const ZcolArgs& a, hipStream_t st);
hipError_t launch_zqr_col_batched(const ZcolPlan& pl, int count, const ZcolArgs* args, hipStream_t st);
// Khatri-Rao QR of Z_n at order N >= 4 by nested two-factor QRs.  With the
// remaining modes m_1 < ... < m_{N-1}: W_1 = R_{m_2} (.) R_{m_1} = Q_1 T_1 and
// W_k = R_{m_{k+1}} (.) T_{k-1} = Q_k T_k (k = 2 .. L = N - 2), each an R^2-row
// staircase QR by zqr_col (compact Q_k).  Column c of Z_n is
// r_{m_{N-1},c} (x) ... (x) r_{m_2,c} (x) r_{m_1,c}, and replacing the two fastest
// factors by Q_k t_{k,c} level by level gives
//   Z_n = (I (x) Q_1)(I (x) Q_2) ... Q_L T_L,
// a product of matrices with orthonormal columns times an upper triangular
// T_L with diag >= 0: R0 = T_L and Q0 = that product (form_q0_nested).
struct NestPlan {
  bool ok;
  int L;          // levels (N - 2)
  ZcolPlan zp;    // plan of the two-factor staircase QRs
};
NestPlan nest_plan(int N, int R);
struct NestArgs {
  int L, R;
  int64_t M;                              // R^(N-1)
  const double* V[CPQR_MAX_ORDER];        // level k: R^2 x R reflectors (Kolda rows)
  const double* meta[CPQR_MAX_ORDER];     // level k: [Md, D, piv]
  double* Q0;                             // M x R out
};
hipError_t launch_form_q0_nested(const NestArgs& a, hipStream_t st);
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
  // compact Q0 (zqr_col): Q0 / Q0prev hold the reflectors V and these the
  // R^2 + 2R words [Md, D, piv] of each; null: Q0 / Q0prev are explicit
  const double* meta_p = nullptr;
  const double* meta_q = nullptr;
};
int apply_num_chunks(int64_t M, int I);
hipError_t launch_apply(const ApplyArgs& a, hipStream_t st);

// Device-side form of ApplyArgs (one entry per problem of a batch).
struct ApplyDev {
  const void* Y;
  int64_t L, S, chunk;
  int I, R, nchunks;
  const double* Q0;
  const double* Q0prev;
  double* partial;
  double* V;
  const DevState* state;
  const double* meta_p;
  const double* meta_q;
  int y_f64;
};
ApplyDev apply_dev(const ApplyArgs& a);
unsigned apply_iblocks(int I);
unsigned apply_reduce_blocks(int I, int R);
// Batched Y*Q0 over `count` problems of one rank class with the same Y type;
// grid extents are maxima over the batch.
struct ApplyBatch {
  int count, rmax;
  bool y_f64;
  unsigned iblocks, nchunks, rblocks;
  const ApplyDev* args;
};
hipError_t launch_apply_batched(const ApplyBatch& b, hipStream_t st);

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
  const double* beta_sched;  // device, sched_len values or null: beta of sweep k+1 = beta_sched[k]
  int sched_len;
  double* qn;           // workspace of CPQR_QN_WORDS doubles: reflectors, U, tau and signs
                        // handed from the factor QR to the Q_n kernel (half-row path)
};
static constexpr int CPQR_QN_WORDS = 256 * 32 + 2 * 32 * 32 + 2 * 32;
hipError_t launch_finish(const FinishArgs& f, hipStream_t st);
// launch_finish in two parts: the head (solve, lambda, factor QR, R_n, fit)
// and, when *tail is set, the explicit Q_n kernel, which only the TTMs of the
// next update wait for (the next update's Z QR needs only R_n).
hipError_t launch_finish_head(const FinishArgs& f, hipStream_t st, bool* tail);
hipError_t launch_finish_tail(const FinishArgs& f, hipStream_t st);
// One workgroup per problem; every problem of the batch has rank class rmax
// and factor rows-per-thread rpt.
hipError_t launch_finish_batched(int count, int rmax, int rpt, const FinishArgs* args, hipStream_t st);
// The column-distributed finish (factors of at most 256 rows, finish_col_rpl
// rows per lane: 1, 2 or 4; 0 beyond) for every problem of a batch, and the
// explicit Q_n that follows it.
int finish_col_rpl(int I);
hipError_t launch_finish_col_batched(int count, int rmax, int rpl, const FinishArgs* args, hipStream_t st);
hipError_t launch_form_qn_batched(int count, int rmax, const FinishArgs* args, hipStream_t st);
// A factor with more than CPQR_MAX_FACTOR_ROWS rows: solve, lambda, A and the
// fit in one streaming workgroup (f.Rn, f.q64, f.q32 unused); the factor QR is
// then launch_tsqr on A (explicit source) followed by the tail, which writes
// the float32 Q_n from the float64 one (q32 may be null) and checks R_n.
hipError_t launch_finish_tall(const FinishArgs& f, hipStream_t st);
hipError_t launch_tall_factor_tail(int I, int R, const double* q64, float* q32, const double* Rn,
                                   DevState* state, hipStream_t st);

// --- norms ----------------------------------------------------------------
// partial sums of squares into `part` (nblocks doubles); returns nblocks
int sumsq_blocks(int64_t n);
hipError_t launch_sumsq(const void* x, bool f64, int64_t n, double* part, hipStream_t st);
hipError_t launch_state_init(DevState* s, const double* part, int nparts, hipStream_t st);
// Flags FLAG_RANKDEF in *st if a mode's R factor (rf, N x R x R) has a
// diagonal entry that is relatively zero (rank_deficient) among its first
// min(dims[n], R) entries.
hipError_t launch_init_rank_check(const double* rf, int N, int R, const int64_t* dims, DevState* st,
                                  hipStream_t s);
// ||X - K||^2 partial sums (sumsq_blocks(n) of them) with the weights
// lambda multiplied by lambda_scale.
hipError_t launch_residual(const void* x, bool f64, int N, const int64_t* dims_host,
                           double* const* factors, const double* lambda, int R, double* part,
                           hipStream_t st, double lambda_scale = 1.0);

// Copies of device buffers in one launch per COPY_LIST_MAX of them (sizes in
// bytes, multiples of 4; buffers must not overlap).
constexpr int COPY_LIST_MAX = 32;
struct CopySeg {
  const void* src;
  void* dst;
  int64_t bytes;
};
hipError_t launch_copy_list(const CopySeg* segs, int n, hipStream_t st);

}  // namespace cpqr
