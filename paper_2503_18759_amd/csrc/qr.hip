// Householder QR kernels (Section 2.4 and Algorithm 2: the QR of every factor
// matrix and the QR decomposition Z_n = Q0 R0 of each mode update).
//
//  * zqr_leaf:  TSQR leaves of Z_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1
//               (Khatri-Rao of the R factors, rows in the Kolda order of the
//               remaining modes, smallest mode fastest).  Each workgroup
//               builds its block of rows from the R factors in LDS, factors it
//               and writes V, T and its R factor (into the stack of leaf
//               triangles).  Also used on an explicit matrix.
//  * zqr_top:   QR of the stacked leaf triangles; writes R0 (diag >= 0) and
//               the explicit Q of the stack with the sign fix applied.
//  * zqr_leaf_col, zqr_top_col: the same two steps by the column-distributed
//               Householder QR (eight waves own whole columns, two columns
//               per step) where they are faster (rank class 32 leaves, and
//               tops of up to 512 rows in rank class 32 or 1024 rows in 16).
//  * form_q0:   explicit Q0 rows of each leaf: Q0_p = E Qtop_p - V_p (T_p V_p1^T Qtop_p).
//  * factor_qr: QR of an I x R factor held by one workgroup; writes R_n and
//               the explicit Q_n in float64 / float32 / bf16 hi+lo.
#include "common.h"
#include "kernels.h"
#include "qr_device.h"
#include "colqr_device.h"

namespace cpqr {

// Largest number of other modes whose Khatri-Rao product can fit a two-level
// TSQR at this column count (R^N <= leaf_rows^2 with the smallest R of the
// class: R = 17 for 32 columns, 9 for 16, 2 for 8; capped by the order limit).
constexpr int qr_max_other_modes(int rmax) { return rmax >= 32 ? 3 : (rmax >= 16 ? 5 : CPQR_MAX_ORDER - 1); }
int qr_max_order(int R) { return qr_max_other_modes(qr_rmax(R)) + 1; }
// Levels of the nested Khatri-Rao QR at the largest order of the class.
constexpr int nest_max_levels(int rmax) { return qr_max_other_modes(rmax) - 1; }

// ----------------------------------------------------------------- leaves
// src == nullptr: build rows of Z from the R factors in `rf` (N x R x R,
// column-major, factor n skipped).  Otherwise read rows of the M x R
// column-major matrix `src`.
template <int RMAX, int RPT>
__global__ CPQR_QR_KERNEL(RMAX) void zqr_leaf(LeafArgs a0, const LeafArgs* __restrict__ batch) {
  const LeafArgs args = kernel_args(a0, batch, blockIdx.y);
  if ((int)blockIdx.x >= args.P) return;
  const int N = args.N, n = args.n, R = args.R;
  const gdouble* __restrict__ rf = (const gdouble*)args.rf;
  const gdouble* __restrict__ src = (const gdouble*)args.src;
  const int64_t M = args.M, ldstack = args.ldstack;
  gdouble* __restrict__ V = (gdouble*)args.V;
  gdouble* __restrict__ Tbuf = (gdouble*)args.T;
  gdouble* __restrict__ stack = (gdouble*)args.stack;
  gdouble* __restrict__ R0 = (gdouble*)args.R0;
  gdouble* __restrict__ Qtop = (gdouble*)args.Qtop;
  __shared__ QrSmem<RMAX> sm;
  __shared__ double srf[qr_max_other_modes(RMAX) * RMAX * RMAX];
  constexpr int B = QrCfg<RMAX>::NT * RPT;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int nm = (src == nullptr) ? N - 1 : 0;
  if (src == nullptr) {
    // R factors of the other modes (ascending mode order), zero-padded to
    // RMAX x RMAX so that columns c >= R of every product vanish
    for (int e = tid; e < nm * RMAX * RMAX; e += QrCfg<RMAX>::NT) {
      const int q = e / (RMAX * RMAX), rem = e % (RMAX * RMAX);
      const int i = rem % RMAX, c = rem / RMAX;
      const int mode = (q < n) ? q : q + 1;
      srf[e] = (i < R && c < R) ? rf[(int64_t)mode * R * R + i + (int64_t)R * c] : 0.0;
    }
    __syncthreads();
  }
  QrRow<RMAX> a[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = (int64_t)p * B + tid + QrCfg<RMAX>::NT * q;
    const bool in = row < M;
    if (src == nullptr) {
      // Z[row][c] = prod_k R_k[digit_k(row)][c], digits of row in base R with
      // the first remaining mode fastest
#pragma unroll
      for (int c = 0; c < RMAX; ++c) a[q].set(c, in ? 1.0 : 0.0);
      int64_t rr = row;
      for (int k = 0; k < nm; ++k) {
        const int d = (int)(rr % R);
        rr /= R;
        const double* rk = srf + k * RMAX * RMAX + d;
#pragma unroll
        for (int c = 0; c < RMAX; ++c) a[q].set(c, a[q].get(c) * rk[RMAX * c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) a[q].set(c, (in && c < R) ? src[row + M * c] : 0.0);
    }
  }
  block_qr<RMAX, RPT>(a, R, sm);
  // V rows (unit lower trapezoidal) for all B rows of the block
  const int64_t ldv = args.ldv;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int lr = tid + QrCfg<RMAX>::NT * q;
    const int64_t row = (int64_t)p * B + lr;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      if (c < R) {
        const double v = block_qr_v<RMAX>(a[q], lr, c, sm);
        V[row + ldv * c] = v;
      }
    }
  }
  if (R0 != nullptr) {
    // single leaf: this is the whole QR.  R0 = D R with D = sign(diag R) and
    // the (trivial) stack factor Qtop = D.
    if (tid < R) {
      const double sg = (sm.beta[tid] < 0.0) ? -1.0 : 1.0;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        if (c < R) {
          R0[tid + R * c] = sg * block_qr_r<RMAX>(a[0], tid, c, sm);
          Qtop[tid + R * c] = (c == tid) ? sg : 0.0;
        }
      }
    }
  } else if (tid < R) {
    // leaf R (no sign fix) into the stack of leaf triangles
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) stack[(int64_t)p * R + tid + ldstack * c] = block_qr_r<RMAX>(a[0], tid, c, sm);
  }
  for (int e = tid; e < R * R; e += QrCfg<RMAX>::NT) {
    const int k = e % R, c = e / R;
    Tbuf[(int64_t)p * R * R + e] = sm.T[k][c];
  }
}

// The same leaf by the column-distributed Householder QR with two columns
// per step (col_qr_pair: eight waves, RMAX / 8 columns each, every wave holds
// all B = 64 RPL rows of its columns), for rank class 32.  Same inputs and outputs as zqr_leaf:
// V rows, T, and the leaf's R in the stack (or, for a single leaf, R0 = D R
// and the trivial Qtop = D).
static constexpr int LEAF_COL_NW = 8;

template <int RMAX, int RPL>
__global__ __launch_bounds__(64 * LEAF_COL_NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
void zqr_leaf_col(LeafArgs a0, const LeafArgs* __restrict__ batch) {
  const LeafArgs args = kernel_args(a0, batch, blockIdx.y);
  if ((int)blockIdx.x >= args.P) return;
  using Cfg = ColCfg<RMAX, LEAF_COL_NW>;
  constexpr int CPW = Cfg::CPW, NT = Cfg::NT, B = 64 * RPL;
  const int N = args.N, n = args.n, R = args.R;
  const gdouble* __restrict__ rf = (const gdouble*)args.rf;
  const gdouble* __restrict__ src = (const gdouble*)args.src;
  const int64_t M = args.M, ldstack = args.ldstack, ldv = args.ldv;
  gdouble* __restrict__ V = (gdouble*)args.V;
  gdouble* __restrict__ Tbuf = (gdouble*)args.T;
  gdouble* __restrict__ stack = (gdouble*)args.stack;
  gdouble* __restrict__ R0 = (gdouble*)args.R0;
  gdouble* __restrict__ Qtop = (gdouble*)args.Qtop;
  __shared__ QrSmem<RMAX> sm;
  __shared__ double srf[qr_max_other_modes(RMAX) * RMAX * RMAX];
  __shared__ double xp[2][2][B];
  const int p = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = CPW * wave;
  const int nm = (src == nullptr) ? N - 1 : 0;
  if (src == nullptr) {
    // R factors of the other modes (ascending mode order), zero-padded to
    // RMAX x RMAX so that columns c >= R of every product vanish
    for (int e = tid; e < nm * RMAX * RMAX; e += NT) {
      const int q = e / (RMAX * RMAX), rem = e % (RMAX * RMAX);
      const int i = rem % RMAX, c = rem / RMAX;
      const int mode = (q < n) ? q : q + 1;
      srf[e] = (i < R && c < R) ? rf[(int64_t)mode * R * R + i + (int64_t)R * c] : 0.0;
    }
    __syncthreads();
  }
  // this wave's columns of the leaf's rows: Z[row][c] = prod_k R_k[digit_k(row)][c]
  // (digits of row in base R, first remaining mode fastest), or the source
  double a[RPL][CPW];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int pp = decltype(pc)::value;
    const int64_t row = (int64_t)p * B + lane + 64 * pp;
    const bool in = row < M;
    if (src == nullptr) {
      double v[CPW];
#pragma unroll
      for (int q = 0; q < CPW; ++q) v[q] = in ? 1.0 : 0.0;
      int64_t rr = row;
      for (int k = 0; k < nm; ++k) {
        const int d = (int)(rr % R);
        rr /= R;
        const double* rk = srf + k * RMAX * RMAX + d + RMAX * c0;
#pragma unroll
        for (int q = 0; q < CPW; ++q) v[q] *= rk[RMAX * q];
      }
#pragma unroll
      for (int q = 0; q < CPW; ++q) a[pp][q] = v[q];
    } else {
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = c0 + q;
        a[pp][q] = (in && c < R) ? src[row + M * c] : 0.0;
      }
    }
  });
  col_qr_pair<RMAX, RPL, LEAF_COL_NW>(a, R, xp, sm);
  if (wave == 0) block_qr_build_t_wave0<RMAX>(R, sm);
  // V rows (unit lower trapezoidal) for all B rows of the leaf
  static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const int c = c0 + q;
    const double sc_c = sm.scale[c < R ? c : 0];
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int pp = decltype(pc)::value;
      const int lr = lane + 64 * pp;
      const double v = (lr > c) ? a[pp][q] * sc_c : ((lr == c) ? 1.0 : 0.0);
      if (c < R) V[(int64_t)p * B + lr + ldv * c] = v;
    });
    // the leaf's R (rows 0..R-1 are lanes of chunk 0)
    if (lane < R && c < R) {
      const int i = lane;
      const double rr = (c > i) ? a[0][q] : ((c == i) ? sm.beta[i] : 0.0);
      if (R0 != nullptr) {
        // single leaf: R0 = D R and the trivial Qtop = D
        const double sg = (sm.beta[i] < 0.0) ? -1.0 : 1.0;
        R0[i + R * c] = sg * rr;
        Qtop[i + R * c] = (c == i) ? sg : 0.0;
      } else {
        stack[(int64_t)p * R + i + ldstack * c] = rr;
      }
    }
  });
  __syncthreads();   // T from wave 0
  for (int e = tid; e < R * R; e += NT) {
    const int k = e % R, c = e / R;
    Tbuf[(int64_t)p * R * R + e] = sm.T[k][c];
  }
}

// --------------------------------------------------------------------- top
// QR of the P*R x R stack.  Writes R0 (R x R column-major, diag >= 0) and
// Qtop (P*R x R column-major) = explicit Q of the stack times the sign fix.
template <int RMAX, int RPT>
__global__ CPQR_QR_KERNEL(RMAX) void zqr_top(TopArgs a0, const TopArgs* __restrict__ batch) {
  const TopArgs args = kernel_args(a0, batch, blockIdx.y);
  if (!args.active) return;
  const int R = args.R;
  const int64_t rows = args.rows;
  const gdouble* __restrict__ stack = (const gdouble*)args.stack;
  gdouble* __restrict__ R0 = (gdouble*)args.R0;
  gdouble* __restrict__ Qtop = (gdouble*)args.Qtop;
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  const int tid = threadIdx.x;
  QrRow<RMAX> a[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = tid + QrCfg<RMAX>::NT * q;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[q].set(c, (row < rows && c < R) ? stack[row + rows * c] : 0.0);
  }
  block_qr<RMAX, RPT>(a, R, sm);
  block_qr_publish<RMAX>(a[0], R, sm, wy, true);
  block_qr_wy_product<RMAX>(sm, wy, R, nullptr, 0);
  for (int e = tid; e < R * R; e += QrCfg<RMAX>::NT) {
    const int i = e % R, c = e / R;
    R0[e] = wy.Rm[i][c];
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = tid + QrCfg<RMAX>::NT * q;
    if (row < rows)
      block_qr_q_row<RMAX>(a[q], (int)row, R, sm, wy, [&](int c, double val) { Qtop[row + rows * c] = val; });
  }
}

// QR of the P*R x R stack by the same column-distributed scheme (eight
// waves, two columns per step).  Writes what zqr_top writes: R0 = D R and
// Qtop = Q D = (E - V T V1^T) D, E the first R columns of the identity.  With
// Md = T V1^T D (R x R, in LDS), row r of Qtop is e_r^T D - V[r][:] Md; the
// rows of V pass through LDS 64 at a time (the QR leaves them distributed by
// column), and each wave forms its own columns of Qtop for those rows.
template <int RMAX, int RPL>
__global__ __launch_bounds__(64 * LEAF_COL_NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
void zqr_top_col(TopArgs a0, const TopArgs* __restrict__ batch) {
  const TopArgs args = kernel_args(a0, batch, blockIdx.y);
  if (!args.active) return;
  using Cfg = ColCfg<RMAX, LEAF_COL_NW>;
  constexpr int CPW = Cfg::CPW, NT = Cfg::NT, MR = 64 * RPL;
  const int R = args.R;
  const int rows = (int)args.rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = CPW * wave;
  const gdouble* __restrict__ stack = (const gdouble*)args.stack;
  gdouble* __restrict__ gR0 = (gdouble*)args.R0;
  gdouble* __restrict__ gQ = (gdouble*)args.Qtop;
  __shared__ QrSmem<RMAX> sm;
  __shared__ double xp[2][2][MR];
  __shared__ double vb[2][64][RMAX + 1];   // 64 rows of V
  __shared__ double smd[RMAX][RMAX + 1];   // Md
  double a[RPL][CPW];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    const int row = lane + 64 * p;
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const int c = c0 + q;
      const bool in = row < rows && c < R;
      const double v = stack[in ? row + (int64_t)rows * c : 0];
      a[p][q] = in ? v : 0.0;
    });
  });
  col_qr_pair<RMAX, RPL, LEAF_COL_NW>(a, R, xp, sm);
  if (tid < RMAX) sm.sgn[tid] = (tid < R && sm.beta[tid] < 0.0) ? -1.0 : 1.0;
  // R0 = D R from the first R rows (chunk 0)
  static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const int c = c0 + q;
    if (lane < R && c < R) {
      const int j = lane;
      const double sg = (sm.beta[j] < 0.0) ? -1.0 : 1.0;
      const double rr = (c > j) ? a[0][q] : ((c == j) ? sm.beta[j] : 0.0);
      gR0[j + R * c] = sg * rr;
    }
  });
  // rows of V of chunk p (this wave's columns) into vb[p & 1]
  auto put_v = [&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    const int row = lane + 64 * p;
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const int c = c0 + q;
      const double sc_c = sm.scale[c < R ? c : 0];
      const double v = (row > c) ? a[p][q] * sc_c : ((row == c) ? 1.0 : 0.0);
      vb[p & 1][lane][c] = (c < R && row < rows) ? v : 0.0;
    });
  };
  if (wave == 0) block_qr_build_t_wave0<RMAX>(R, sm);
  put_v(std::integral_constant<int, 0>{});
  __syncthreads();
  // Md[m][c] = sgn_c sum_k T[m][k] V1[c][k]  (V1 = rows 0..R-1 of V, in vb[0])
  for (int e = tid; e < RMAX * RMAX; e += NT) {
    const int m = e % RMAX, c = e / RMAX;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < RMAX; ++k) acc = fma(sm.T[m][k], vb[0][c][k], acc);
    smd[m][c] = (m < R && c < R) ? acc * sm.sgn[c] : 0.0;
  }
  __syncthreads();
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    if constexpr (p > 0) {
      put_v(pc);
      __syncthreads();
    }
    const int row = lane + 64 * p;
    double v[RMAX];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) v[m] = vb[p & 1][lane][m];
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const int c = c0 + q;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < RMAX; ++m) acc = fma(v[m], smd[m][c], acc);
      const double e = (row == c) ? sm.sgn[c] : 0.0;
      if (row < rows && c < R) gQ[row + (int64_t)rows * c] = e - acc;
    });
  });
}

// The column-distributed top for stacks of up to `rows` rows (the largest
// stack of the launch): rank class 32 up to 512 rows, rank class 16 from 513
// to 1024 rows; false: zqr_top then.
static bool top_col_launch(int rm, int64_t rows, dim3 grid, const TopArgs& ta, const TopArgs* batch,
                           hipStream_t st) {
  const dim3 blk(64 * LEAF_COL_NW);
  if (rm == 32 && rows <= 256)
    hipLaunchKernelGGL((zqr_top_col<32, 4>), grid, blk, 0, st, ta, batch);
  else if (rm == 32 && rows <= 512)
    hipLaunchKernelGGL((zqr_top_col<32, 8>), grid, blk, 0, st, ta, batch);
  else if (rm == 16 && rows > 512 && rows <= 1024)
    hipLaunchKernelGGL((zqr_top_col<16, 16>), grid, blk, 0, st, ta, batch);
  else
    return false;
  return true;
}

// ------------------------------------------------------------------ form Q0
// One workgroup per 256-row chunk.  Chunk rows lie inside one leaf p.
template <int RMAX>
__global__ __launch_bounds__(QrCfg<RMAX>::NT) void form_q0(FormArgs a0, const FormArgs* __restrict__ batch) {
  const FormArgs args = kernel_args(a0, batch, blockIdx.y);
  const int R = args.R, leaf_rows = args.leaf_rows;
  const int64_t M = args.M, ldv = args.ldv, ldq = args.ldq;
  const gdouble* __restrict__ V = (const gdouble*)args.V;
  const gdouble* __restrict__ Tbuf = (const gdouble*)args.T;
  const gdouble* __restrict__ Qtop = (const gdouble*)args.Qtop;
  gdouble* __restrict__ Q0 = (gdouble*)args.Q0;
  if ((int64_t)blockIdx.x * QrCfg<RMAX>::NT >= M) return;
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  __shared__ double sQt[RMAX * RMAX];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * QrCfg<RMAX>::NT;
  const int p = (int)(row0 / leaf_rows);
  const int64_t leaf0 = (int64_t)p * leaf_rows;
  // V1 of the leaf, T of the leaf, Qtop block p (row-major in LDS)
  for (int e = tid; e < RMAX * RMAX; e += QrCfg<RMAX>::NT) {
    const int i = e / RMAX, c = e % RMAX;
    const bool in = i < R && c < R;
    wy.V1[i][c] = in ? V[leaf0 + i + ldv * c] : 0.0;
    sm.T[i][c] = in ? Tbuf[(int64_t)p * R * R + i + R * c] : 0.0;
    sQt[i * RMAX + c] = in ? Qtop[(int64_t)p * R + i + ldq * c] : 0.0;
  }
  __syncthreads();
  block_qr_wy_product<RMAX>(sm, wy, R, sQt, RMAX);
  const int64_t row = row0 + tid;
  if (row >= M) return;
  const int64_t lr = row - leaf0;
  // row of V in registers, then two columns per trip with the M entries of
  // a column adjacent in LDS (16-byte reads) and two partial sums per column
  double v[RMAX];
#pragma unroll
  for (int m = 0; m < RMAX; ++m) v[m] = (m < R) ? V[row + ldv * (m < R ? m : 0)] : 0.0;
  for (int c = 0; c < R; c += 2) {
    // c + 1 <= RMAX - 1 (R <= RMAX, RMAX even); M is zero in columns >= R
    double m0[RMAX], m1[RMAX];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) {
      m0[m] = wy.Mt[c][m];
      m1[m] = wy.Mt[c + 1][m];
    }
    double a0 = (lr < R) ? sQt[lr * RMAX + c] : 0.0, a1 = (lr < R) ? sQt[lr * RMAX + c + 1] : 0.0;
    double b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int m = 0; m < RMAX; m += 2) {
      a0 = fma(-v[m], m0[m], a0);
      a1 = fma(-v[m], m1[m], a1);
      b0 = fma(-v[m + 1], m0[m + 1], b0);
      b1 = fma(-v[m + 1], m1[m + 1], b1);
    }
    Q0[row + M * c] = a0 + b0;
    if (c + 1 < R) Q0[row + M * (c + 1)] = a1 + b1;
  }
}

// --------------------------------------------------------------- staircase
// Digits (d_0 .. d_{K-1}; d_0 indexes the first remaining mode) of staircase
// position s.  Shell m (largest digit m) holds positions [m^K, (m+1)^K);
// inside a shell the tuples come by the highest index h with d_h = m, from
// h = K-1 down to 0, then by the digits below h (base m+1, lowest fastest)
// and above h (base m).  Positions below (c+1)^K are exactly the tuples with
// every digit <= c, the profile of column c of Z_n.
__device__ __forceinline__ int ipow_i(int b, int e) {
  int p = 1;
  for (int k = 0; k < e; ++k) p *= b;
  return p;
}

// 32-bit arithmetic throughout (Z_n of this kernel has at most 1024 rows);
// the shell index comes from a float estimate of s^(1/K), corrected exactly.
template <int KMAX>
__device__ __forceinline__ void stair_digits(int s, int K, int (&d)[KMAX]) {
  int m = (int)__builtin_exp2f(__builtin_log2f((float)s + 0.5f) / (float)K);
  while (ipow_i(m + 1, K) <= s) ++m;
  while (m > 0 && ipow_i(m, K) > s) --m;
  int o = s - ipow_i(m, K);
  int h = K - 1;
  int lo = 1;
  for (; h >= 0; --h) {
    lo = ipow_i(m + 1, h);
    const int cnt = lo * ipow_i(m, K - 1 - h);
    if (o < cnt) break;
    o -= cnt;
  }
  int l = o % lo, u = o / lo;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    int dk = 0;
    if (k < h) {
      dk = l % (m + 1);
      l /= (m + 1);
    } else if (k == h) {
      dk = m;
    } else if (k < K) {
      dk = u % m;
      u /= m;
    }
    d[k] = dk;
  }
}

// One workgroup per problem: build Z_n in staircase order from the R
// factors, factor it (block_qr_stair) and write R0 (diag >= 0) and the
// explicit Q0 (sign-fixed, rows scattered back to the Kolda order).
template <int RMAX, int NS, int RT, int CS>
__global__ CPQR_QR_KERNEL(RMAX) void zqr_stair(StairArgs a0, const StairArgs* __restrict__ batch) {
  // arguments read directly: passing them through readfirstlane makes the
  // compiler spill this kernel's rows to the accumulation registers
  const StairArgs args = batch ? batch[blockIdx.x] : a0;
  if (!args.active) return;
  constexpr int NT = QrCfg<RMAX>::NT;
  constexpr int KMAX = qr_max_other_modes(RMAX);
  constexpr int NSA = NS > 0 ? NS : 1;
  const int N = args.N, n = args.n, R = args.R, K = N - 1;
  const int64_t M = args.M;
  __shared__ QrSmem<RMAX> sm;
  // the R factors are needed only to build Z_n; their LDS is reused for the
  // compact WY product afterwards
  __shared__ union StairLds {
    double srf[KMAX * RMAX * RMAX];
    QrWySmem<RMAX> wy;
  } u;
  const int tid = threadIdx.x;
  {
    // R factors of the other modes, zero-padded to RMAX x RMAX; a fixed trip
    // count with clamped indices so that all loads are in flight together
    constexpr int TRIPS = (KMAX * RMAX * RMAX + NT - 1) / NT;
    const gdouble* __restrict__ rf = (const gdouble*)args.rf;
    double val[TRIPS];
#pragma unroll
    for (int t = 0; t < TRIPS; ++t) {
      const int e = tid + NT * t;
      const int q = e / (RMAX * RMAX), rem = e % (RMAX * RMAX);
      const int i = rem % RMAX, c = rem / RMAX;
      const int mode = (q < n) ? q : q + 1;
      const bool in = (e < K * RMAX * RMAX) && i < R && c < R;
      const double x = rf[in ? (int64_t)mode * R * R + i + (int64_t)R * c : 0];
      val[t] = in ? x : 0.0;
    }
#pragma unroll
    for (int t = 0; t < TRIPS; ++t) {
      const int e = tid + NT * t;
      if (e < K * RMAX * RMAX) u.srf[e] = val[t];
    }
  }
  __syncthreads();
  // Z[row][c] = prod_{k < K} R_k[d_k][c]; branch-free over the KMAX digit
  // slots (unused slots read a valid entry and multiply by one), so that a
  // row's LDS reads are issued together rather than one per branch
  auto zval = [&](const int (&d)[KMAX], int c) __attribute__((always_inline)) {
    double v = 1.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const bool use = k < K;
      const double f = u.srf[(use ? k * RMAX * RMAX + d[k] : 0) + RMAX * c];
      v *= use ? f : 1.0;
    }
    return v;
  };
  QrStair<RMAX, NS, RT, CS> z;
  int64_t krow[NS + 1];   // Kolda row of each held row (-1: beyond M)
  {
    int d[KMAX];
    const int64_t s0 = tid;
    if (s0 < M) {
      stair_digits<KMAX>((int)s0, K, d);
      int64_t kr = 0, w = 1;
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k < K) {
          kr += d[k] * w;
          w *= R;
        }
      krow[0] = kr;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) z.a0.set(c, zval(d, c));
    } else {
      krow[0] = -1;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) z.a0.set(c, 0.0);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int64_t sq = (int64_t)NT * (q + 1) + tid;
      if (sq < M) {
        stair_digits<KMAX>((int)sq, K, d);
        int64_t kr = 0, w = 1;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
          if (k < K) {
            kr += d[k] * w;
            w *= R;
          }
        krow[q + 1] = kr;
#pragma unroll
        for (int c = 0; c < RT; ++c) z.at[q].set(c, zval(d, CS + c));
      } else {
        krow[q + 1] = -1;
#pragma unroll
        for (int c = 0; c < RT; ++c) z.at[q].set(c, 0.0);
      }
    }
  }
  (void)NSA;
  block_qr_stair<RMAX, NS, RT, CS>(z, R, K, M, sm);
  // R0 = D R with D = sign(diag R)
  if (tid < R) {
    const double sg = (sm.beta[tid] < 0.0) ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) ((gdouble*)args.R0)[tid + R * c] = sg * block_qr_r<RMAX>(z.a0, tid, c, sm);
  }
  __syncthreads();   // the R factors in LDS are dead from here on
  block_qr_publish<RMAX>(z.a0, R, sm, u.wy, true);
  block_qr_wy_product<RMAX>(sm, u.wy, R, nullptr, 0);
  gdouble* __restrict__ Q0 = (gdouble*)args.Q0;
  if constexpr (NS == 0) {
    if (krow[0] >= 0)
      block_qr_q_row<RMAX>(z.a0, tid, R, sm, u.wy, [&](int c, double val) { Q0[krow[0] + M * c] = val; });
  } else {
    // Rows of Q0 = (E - V M) diag(sgn), M = T V1^T, for the slice-0 row and
    // the narrow rows together.  A narrow row's v vanishes outside columns
    // [CS, CS+RT) of V, and M vanishes at (m, c) for m > c (V1 is unit lower
    // triangular), so a narrow row's entries in columns c < CS are exact
    // zeros.  From column CS on, each pair of M entries read from LDS serves
    // the slice-0 row and every narrow row.  The multiply-adds of each row
    // run in the same order as for a row on its own.
    double v0[RMAX];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) v0[m] = (m < R) ? block_qr_v<RMAX>(z.a0, tid, m, sm) : 0.0;
    double vn[NS][RT];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int m = 0; m < RT; ++m) vn[q][m] = (CS + m < R) ? z.at[q].get(m) * sm.scale[CS + m] : 0.0;
    const bool have0 = krow[0] >= 0;
    for (int c = 0; c < R; c += 2) {
      // c + 1 <= RMAX - 1 (R <= RMAX, RMAX even); M is zero in columns >= R
      double a0 = (tid == c) ? 1.0 : 0.0, a1 = (tid == c + 1) ? 1.0 : 0.0, b0 = 0.0, b1 = 0.0;
      // M is upper triangular (M[m][c] = 0 for m > c): reflector blocks past
      // c + 1 contribute exact zeros and are skipped
      constexpr int MB = CS < 8 ? CS : 8;
      static_assert(CS % MB == 0 && (RMAX - CS) % MB == 0 && RT % MB == 0, "blocks of reflectors");
#pragma unroll
      for (int mb = 0; mb < CS; mb += MB) {
        if (mb > c + 1) break;
        double m0[MB], m1[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          m0[m] = u.wy.Mt[c][mb + m];
          m1[m] = u.wy.Mt[c + 1][mb + m];
        }
#pragma unroll
        for (int m = 0; m < MB; m += 2) {
          a0 = fma(-v0[mb + m], m0[m], a0);
          a1 = fma(-v0[mb + m], m1[m], a1);
          b0 = fma(-v0[mb + m + 1], m0[m + 1], b0);
          b1 = fma(-v0[mb + m + 1], m1[m + 1], b1);
        }
      }
      double na0[NS], na1[NS], nb0[NS], nb1[NS];
#pragma unroll
      for (int q = 0; q < NS; ++q) na0[q] = na1[q] = nb0[q] = nb1[q] = 0.0;
      // from column CS on (the upper blocks are needed only then): the
      // slice-0 row and every narrow row share the M entries
#pragma unroll
      for (int mb = 0; mb < RMAX - CS; mb += MB) {
        if (CS + mb > c + 1) break;
        double m0[MB], m1[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          m0[m] = u.wy.Mt[c][CS + mb + m];
          m1[m] = u.wy.Mt[c + 1][CS + mb + m];
        }
#pragma unroll
        for (int m = 0; m < MB; m += 2) {
          a0 = fma(-v0[CS + mb + m], m0[m], a0);
          a1 = fma(-v0[CS + mb + m], m1[m], a1);
          b0 = fma(-v0[CS + mb + m + 1], m0[m + 1], b0);
          b1 = fma(-v0[CS + mb + m + 1], m1[m + 1], b1);
          if (mb + m < RT) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
              na0[q] = fma(-vn[q][mb + m], m0[m], na0[q]);
              na1[q] = fma(-vn[q][mb + m], m1[m], na1[q]);
              nb0[q] = fma(-vn[q][mb + m + 1], m0[m + 1], nb0[q]);
              nb1[q] = fma(-vn[q][mb + m + 1], m1[m + 1], nb1[q]);
            }
          }
        }
      }
      const double s0 = sm.sgn[c], s1 = sm.sgn[c + 1];
      if (have0) {
        Q0[krow[0] + M * c] = (a0 + b0) * s0;
        if (c + 1 < R) Q0[krow[0] + M * (c + 1)] = (a1 + b1) * s1;
      }
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (krow[q + 1] < 0) continue;
        // columns below CS: exact zeros
        const double q0v = (c >= CS) ? (na0[q] + nb0[q]) * s0 : 0.0;
        const double q1v = (c >= CS) ? (na1[q] + nb1[q]) * s1 : 0.0;
        Q0[krow[q + 1] + M * c] = q0v;
        if (c + 1 < R) Q0[krow[q + 1] + M * (c + 1)] = q1v;
      }
    }
  }
}

// ------------------------------------------------- column-distributed Z QR
// Householder QR of Z_n (at most 1024 rows, rows in staircase order) in the
// column-distributed layout of col_qr (colqr_device.h); the staircase bounds
// every column step to the rows of its column's profile, (j+1)^K.  The
// output is the compact form of Q0 rather than Q0 itself: with the sign fix
// D = sign(diag R), Q0 = (E - V T V1^T) D, where V holds the reflectors
// (unit lower trapezoidal, rows scattered back to the Kolda order), V1 its
// first R rows and E the first R columns of the identity in staircase order,
// i.e. the unit vectors of the Kolda rows piv_0 .. piv_{R-1} of the first R
// staircase rows.  Then Y_(n) Q0 = (Y_E - (Y_(n) V) Md) D... with Md = T V1^T D
// and Y_E = Y_(n)[:, piv] the product needs only Y_(n) V, which has the
// shape of Y_(n) Q0, and an R x R correction (apply_partial, apply_reduce).
// meta (R^2 + 2R doubles): Md (R x R column-major), the signs D, piv.
template <int RMAX, int RPL, int NW, int K>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
void zqr_col(ZcolArgs a0, const ZcolArgs* __restrict__ batch) {
  const ZcolArgs args = kernel_args(a0, batch, blockIdx.x);
  if (!args.active) return;
  // two columns per step where the pairs fit the waves
  constexpr bool PAIRS = ((RMAX / NW) % 2) == 0;
  using SC = StairCfg<RMAX, RPL, NW, K, PAIRS>;
  constexpr int CPW = SC::CPW, NT = 64 * NW, MR = SC::MR;
  const int n = args.n, R = args.R;
  const int M = (int)args.M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ QrSmem<RMAX> sm;
  // broadcast buffer: two published columns per step, double-buffered
  // (pairs), or the owner's columns packed, double-buffered
  __shared__ double xbuf[PAIRS ? 2 * 2 * 64 * RPL : 2 * SC::TOT * 64];
  __shared__ union ZcolLds {
    double srf[K * RMAX * RMAX];   // R factors of the other modes (Z build)
    double v1[RMAX][RMAX + 1];     // first R rows of V (epilogue)
  } u;
  __shared__ int skrow[64 * RPL];  // Kolda row of each staircase row, for the epilogue
  // Kolda row and digits of this lane's rows (all loads in flight together,
  // beside those of the R factors)
  typedef __attribute__((address_space(1))) const int2 gint2;
  const gint2* __restrict__ smap = (const gint2*)args.smap;
  int2 tab[RPL];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    const int s = lane + 64 * p;
    int2 t = make_int2(-1, 0);
    if (s < M) {
      t.x = smap[s].x;
      t.y = smap[s].y;
    }
    tab[p] = t;
  });
  {
    // R factors of the other modes (ascending mode order), zero-padded to
    // RMAX x RMAX so that columns c >= R of every product vanish
    const gdouble* __restrict__ rf = (const gdouble*)args.rf;
    for (int e = tid; e < K * RMAX * RMAX; e += NT) {
      const int q = e / (RMAX * RMAX), rem = e % (RMAX * RMAX);
      const int i = rem % RMAX, c = rem / RMAX;
      const int mode = (q < n) ? q : q + 1;
      const bool in = i < R && c < R;
      const gdouble* __restrict__ f =
          (q == K - 1 && args.rf_hi != nullptr) ? (const gdouble*)args.rf_hi : rf + (int64_t)mode * R * R;
      const double x = f[in ? i + (int64_t)R * c : 0];
      u.srf[e] = in ? x : 0.0;
    }
  }
  __syncthreads();
  // Z[s][c] = prod_k R_k[d_k(s)][c] for this wave's columns c = NW q + wave,
  // rows s = lane + 64 p < 64 L(q) in staircase order (digits from the
  // staircase table, 5 bits each)
  if (wave == 0) {
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      skrow[lane + 64 * p] = tab[p].x;
    });
  }
  double a[SC::TOT];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    const bool in = tab[p].x >= 0;
    const int dig = tab[p].y;
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      if constexpr (p < SC::L(q)) {
        const int c = SC::col(q, wave);
        double v = in ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) v *= u.srf[k * RMAX * RMAX + ((dig >> (5 * k)) & 31) + RMAX * c];
        a[SC::OFF(q) + p] = v;
      }
    });
  });
  __syncthreads();   // the R factors in LDS are dead from here on
  // rows in the profile of column j: min(M, (j+1)^K)
  auto prof = [&](int j) __attribute__((always_inline)) {
    int pw = 1;
#pragma unroll
    for (int k = 0; k < K; ++k) pw *= (j + 1);
    return pw < M ? pw : M;
  };
  if constexpr (PAIRS)
    col_qr_stair_pair<RMAX, RPL, NW, K>(a, R, prof, reinterpret_cast<double(*)[2][64 * RPL]>(xbuf), sm);
  else
    col_qr_stair<RMAX, RPL, NW, K>(a, R, prof, reinterpret_cast<double(*)[SC::TOT * 64]>(xbuf), sm);
  // R0 = D R and V1 into LDS (the first R rows are lanes 0..R-1 of chunk 0)
  gdouble* __restrict__ gR0 = (gdouble*)args.R0;
  gdouble* __restrict__ gV = (gdouble*)args.V;
  static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const int c = SC::col(q, wave);
    const double sc_c = sm.scale[c < R ? c : 0];
    if (lane < RMAX) {
      const int j = lane;
      const double sg = (j < R && sm.beta[j] < 0.0) ? -1.0 : 1.0;
      const double x = a[SC::OFF(q)];
      const double rr = (c > j) ? x : ((c == j) ? sm.beta[j] : 0.0);
      if (j < R && c < R) gR0[j + R * c] = sg * rr;
      const double v1 = (j > c) ? x * sc_c : ((j == c) ? 1.0 : 0.0);
      u.v1[j][c] = (j < R && c < R) ? v1 : 0.0;
    }
  });
  // the Kolda rows again (not held through the factorisation: from LDS)
  int krow[RPL];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    krow[p] = skrow[lane + 64 * p];
  });
  // wave 0 builds T while the other waves write their rows of V
  if (wave == 0) block_qr_build_t_wave0<RMAX>(R, sm);
  // V rows (Kolda order; rows beyond a column's live chunks stay zero in the
  // buffer from its set-up)
  static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const int c = SC::col(q, wave);
    const double sc_c = sm.scale[c < R ? c : 0];
    static_for<0, SC::L(q)>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      const int s = lane + 64 * p;
      const double v = (s > c) ? a[SC::OFF(q) + p] * sc_c : ((s == c) ? 1.0 : 0.0);
      if (krow[p] >= 0 && c < R) gV[krow[p] + (int64_t)M * c] = v;
    });
  });
  gdouble* __restrict__ meta = (gdouble*)args.meta;
  if (tid < R) {
    meta[R * R + R + tid] = (double)skrow[tid];
    meta[R * R + tid] = (sm.beta[tid] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  // Md = T V1^T D: Md[m][c] = sgn_c sum_k T[m][k] V1[c][k]
  for (int e = tid; e < R * R; e += NT) {
    const int m = e % R, c = e / R;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < RMAX; ++k) acc = fma(sm.T[m][k], u.v1[c][k], acc);
    meta[e] = acc * ((sm.beta[c] < 0.0) ? -1.0 : 1.0);
  }
}

// Staircase order of the rows of Z_n (the row order of zqr_stair): entry s
// holds the Kolda row of staircase position s and its K digits, 5 bits each
// (digit k = index into the k-th remaining mode).
void stair_table(int R, int K, int64_t M, int* out) {
  for (int64_t s = 0; s < M; ++s) {
    auto ipw = [](int64_t b, int e) { int64_t p = 1; for (int k = 0; k < e; ++k) p *= b; return p; };
    int m = 0;
    while (ipw(m + 1, K) <= s) ++m;
    int64_t o = s - ipw(m, K);
    int h = K - 1;
    int64_t lo = 1;
    for (; h >= 0; --h) {
      lo = ipw(m + 1, h);
      const int64_t cnt = lo * ipw(m, K - 1 - h);
      if (o < cnt) break;
      o -= cnt;
    }
    int64_t l = o % lo, up = o / lo;
    int64_t kr = 0, w = 1;
    int packed = 0;
    for (int k = 0; k < K; ++k) {
      int dk;
      if (k < h) { dk = (int)(l % (m + 1)); l /= (m + 1); }
      else if (k == h) dk = m;
      else { dk = (int)(up % m); up /= m; }
      kr += dk * w;
      w *= R;
      packed |= dk << (5 * k);
    }
    out[2 * s] = (int)kr;
    out[2 * s + 1] = packed;
  }
}

ZcolPlan zcol_plan(int N, int R) {
  ZcolPlan pl{};
  const int rm = qr_rmax(R);
  const int K = N - 1;
  if (rm == 0 || (K != 2 && K != 3)) return pl;
  int64_t M = 1;
  for (int k = 0; k < K; ++k) M *= R;
  if (M > 1024 || (K == 3 && rm == 32)) return pl;
  pl.ok = true;
  pl.rmax = rm;
  pl.k = K;
  pl.rpl = M <= 64 ? 1 : (M <= 128 ? 2 : (M <= 256 ? 4 : (M <= 512 ? 8 : 16)));
  // four waves (one per SIMD) up to 256 rows; eight (two per SIMD, half the
  // columns each) beyond, where the column steps are bound by instruction
  // issue
  pl.nw = (pl.rpl >= 8 || (pl.rpl == 4 && rm == 16 && K == 2)) ? 8 : 4;
  return pl;
}

static hipError_t zcol_launch(const ZcolPlan& pl, unsigned blocks, const ZcolArgs& a, const ZcolArgs* batch,
                              hipStream_t st) {
#define CPQR_ZC(RM, RP, NWV, KV) \
  hipLaunchKernelGGL((zqr_col<RM, RP, NWV, KV>), dim3(blocks), dim3(64 * NWV), 0, st, a, batch)
#define CPQR_ZC_RPL(RM, KV)                                                  \
  if (pl.rpl == 1) CPQR_ZC(RM, 1, (RM < 4 ? RM : 4), KV);                    \
  else if (pl.rpl == 2) CPQR_ZC(RM, 2, (RM < 4 ? RM : 4), KV);               \
  else if (pl.rpl == 4) CPQR_ZC(RM, 4, (RM < 4 ? RM : 4), KV);               \
  else if (pl.rpl == 8) CPQR_ZC(RM, 8, 8, KV);                               \
  else if (pl.rpl == 16) CPQR_ZC(RM, 16, 8, KV);                             \
  else return hipErrorInvalidValue;
  if (!pl.ok) return hipErrorInvalidValue;
  if (pl.k == 2) {
    if (pl.rmax == 8) { CPQR_ZC_RPL(8, 2) }
    else if (pl.rmax == 16 && pl.nw == 8 && pl.rpl == 4) CPQR_ZC(16, 4, 8, 2);
    else if (pl.rmax == 16) { CPQR_ZC_RPL(16, 2) }
    else if (pl.rmax == 32) { CPQR_ZC_RPL(32, 2) }
    else return hipErrorInvalidValue;
  } else if (pl.k == 3) {
    if (pl.rmax == 8) { CPQR_ZC_RPL(8, 3) }
    else if (pl.rmax == 16) { CPQR_ZC_RPL(16, 3) }
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef CPQR_ZC_RPL
#undef CPQR_ZC
  return hipGetLastError();
}

hipError_t launch_zqr_col(const ZcolPlan& pl, const ZcolArgs& a, hipStream_t st) {
  if (!pl.ok || a.M > 64 * pl.rpl || a.R > pl.rmax) return hipErrorInvalidValue;
  return zcol_launch(pl, 1, a, nullptr, st);
}

hipError_t launch_zqr_col_batched(const ZcolPlan& pl, int count, const ZcolArgs* args, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return zcol_launch(pl, (unsigned)count, ZcolArgs{}, args, st);
}

// ------------------------------------------------------- nested Khatri-Rao QR
NestPlan nest_plan(int N, int R) {
  NestPlan pl{};
  if (N < 4 || qr_rmax(R) == 0 || N - 2 > nest_max_levels(qr_rmax(R))) return pl;
  pl.zp = zcol_plan(3, R);
  if (!pl.zp.ok) return pl;
  pl.ok = true;
  pl.L = N - 2;
  return pl;
}

// Explicit Q0 of the nested QR.  In the compact form of zqr_col, Q_k =
// E_k D_k - V_k Md_k (E_k: the unit vectors of the Kolda rows piv_k).  Row
// r + R^2 t of Q0 (r: the digits of m_1 and m_2; t: those of m_3 .. m_{N-1},
// Kolda order) is Q_1[r, :] B_2(t_0) B_3(t_1) ... B_L(t_{L-2}), B_k(d) being
// rows dR .. dR + R - 1 of Q_k and t_i the base-R digits of t.  Workgroup
// (t, chunk, column group) stages the blocks of V_k, every Md_k, D_k and
// piv_k in LDS (all loads in flight together), forms its columns of
// P = B_2 ... B_L and W = Md_1 P there, then one row of its chunk per thread:
// Q0[r + R^2 t][c] = D_1[j] P[j][c] [r = piv_1(j)] - sum_m V_1[r][m] W[m][c].
// Columns of Q0 per workgroup of form_q0_nested.
static constexpr int FQ_CW = 8;

template <int RMAX>
__global__ __launch_bounds__(256) void form_q0_nested(NestArgs a) {
  constexpr int LM = nest_max_levels(RMAX);
  constexpr int LD = RMAX + 1;
  // level k >= 1: rows d_k R .. of V_k, then B_k; every level: Md_k.  All
  // R x R blocks are zero-padded to RMAX x RMAX so that the inner loops run
  // over RMAX terms, unrolled.
  __shared__ double vb[LM][RMAX][LD];
  __shared__ double md[LM][RMAX][LD];
  __shared__ double P[RMAX][LD], W[RMAX][LD];
  __shared__ double dv[LM][RMAX];
  __shared__ int pv[LM][RMAX];
  __shared__ int jof[RMAX * RMAX];   // j with piv_1(j) = r, else -1
  __shared__ int dig[LM];            // level k >= 1: digit t_{k-1} of t
  const int R = a.R, L = a.L, R2 = R * R;
  const int64_t t = blockIdx.x;
  const int tid = threadIdx.x;
  // sum_m x(m) y(m) over RMAX terms in four independent chains
  auto dot = [](auto x, auto y) __attribute__((always_inline)) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < RMAX; ++m) s[m & 3] = fma(x(m), y(m), s[m & 3]);
    return (s[0] + s[1]) + (s[2] + s[3]);
  };
  // this thread's row of V_1 (independent of everything below: in flight first)
  const int r = blockIdx.y * 256 + tid;
  double v[RMAX];
  {
    const gdouble* __restrict__ V1 = (const gdouble*)a.V[0];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) v[m] = (m < R && r < R2) ? V1[r + (int64_t)R2 * m] : 0.0;
  }
  if (tid == 0) {
    int64_t rem = t;
    for (int k = 1; k < LM; ++k) {
      dig[k] = (int)(rem % R);
      rem /= R;
    }
  }
  for (int e = tid; e < R2; e += 256) jof[e] = -1;
  for (int e = tid; e < RMAX * LD; e += 256) {
    (&P[0][0])[e] = 0.0;
    (&W[0][0])[e] = 0.0;
  }
  __syncthreads();
  // every level's blocks, loads in flight together
#pragma unroll
  for (int k = 0; k < LM; ++k) {
    if (k < L) {
      const gdouble* __restrict__ V = (const gdouble*)a.V[k];
      const gdouble* __restrict__ meta = (const gdouble*)a.meta[k];
      const int row0 = (k > 0) ? dig[k] * R : 0;
      constexpr int IT = (RMAX * RMAX + 255) / 256;
      double x[IT], y[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = tid + 256 * it;
        const int i = e % RMAX, c = e / RMAX;
        const bool in = e < RMAX * RMAX && i < R && c < R;
        x[it] = meta[in ? i + R * c : 0];
        y[it] = (k > 0) ? V[in ? row0 + i + (int64_t)R2 * c : 0] : 0.0;
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = tid + 256 * it;
        const int i = e % RMAX, c = e / RMAX;
        const bool in = e < RMAX * RMAX && i < R && c < R;
        if (e < RMAX * RMAX) {
          md[k][i][c] = in ? x[it] : 0.0;
          if (k > 0) vb[k][i][c] = in ? y[it] : 0.0;
        }
      }
      if (tid < RMAX) {
        const bool in = tid < R;
        const double d = meta[in ? R2 + tid : 0];
        const double pr = meta[in ? R2 + R + tid : 0];
        dv[k][tid] = in ? d : 0.0;
        pv[k][tid] = in ? (int)pr : -1;
      }
    }
  }
  __syncthreads();
  if (tid < R && pv[0][tid] >= 0 && pv[0][tid] < R2) jof[pv[0][tid]] = tid;
  // This workgroup writes the columns [cb, cb + FQ_CW) of Q0, which need
  // only those columns of P and W, and so only those of the last block.
  const int cb = blockIdx.z * FQ_CW;
  // B_k(d)[j][c] = [dR + j = piv_k(c)] D_k[c] - sum_m vb_k[j][m] Md_k[m][c]
  // (into W, then over vb_k; the last level on this workgroup's columns)
  for (int k = 1; k < L; ++k) {
    const int c0 = (k == L - 1) ? cb : 0;
    const int n = RMAX * ((k == L - 1) ? FQ_CW : RMAX);
    for (int e = tid; e < n; e += 256) {
      const int j = e % RMAX, c = c0 + e / RMAX;
      const double acc = dot([&](int m) { return vb[k][j][m]; }, [&](int m) { return md[k][m][c]; });
      W[j][c] = (j < R && c < R) ? (((pv[k][c] == dig[k] * R + j) ? dv[k][c] : 0.0) - acc) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < n; e += 256) vb[k][e % RMAX][c0 + e / RMAX] = W[e % RMAX][c0 + e / RMAX];
    __syncthreads();
  }
  // P = B_L, then P = B_k P for k = L - 1 .. 2 (1-based levels); columns
  // outside [cb, cb + FQ_CW) stay zero
  for (int e = tid; e < RMAX * FQ_CW; e += 256) P[e % RMAX][cb + e / RMAX] = vb[L - 1][e % RMAX][cb + e / RMAX];
  __syncthreads();
  for (int k = L - 2; k >= 1; --k) {
    for (int e = tid; e < RMAX * FQ_CW; e += 256) {
      const int j = e % RMAX, c = cb + e / RMAX;
      W[j][c] = dot([&](int m) { return vb[k][j][m]; }, [&](int m) { return P[m][c]; });
    }
    __syncthreads();
    for (int e = tid; e < RMAX * FQ_CW; e += 256) P[e % RMAX][cb + e / RMAX] = W[e % RMAX][cb + e / RMAX];
    __syncthreads();
  }
  // W = Md_1 P
  for (int e = tid; e < RMAX * FQ_CW; e += 256) {
    const int m = e % RMAX, c = cb + e / RMAX;
    W[m][c] = dot([&](int j) { return md[0][m][j]; }, [&](int j) { return P[j][c]; });
  }
  __syncthreads();
  if (r >= R2) return;
  const int j = jof[r];
  const double dj = (j >= 0) ? dv[0][j] : 0.0;
  gdouble* __restrict__ Q0 = (gdouble*)a.Q0;
  const int64_t row = r + (int64_t)R2 * t;
  // four columns at a time (independent chains)
  for (int c0 = cb; c0 < R && c0 < cb + FQ_CW; c0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < RMAX; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(v[m], W[m][(c0 + u) & (RMAX - 1)], acc[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u;
      if (c < R) Q0[row + a.M * c] = ((j >= 0) ? dj * P[j][c] : 0.0) - acc[u];
    }
  }
}

hipError_t launch_form_q0_nested(const NestArgs& a, hipStream_t st) {
  const int rm = qr_rmax(a.R);
  if (rm == 0 || a.L < 2 || a.L > nest_max_levels(rm)) return hipErrorInvalidValue;
  int64_t tails = 1;
  for (int k = 2; k <= a.L; ++k) tails *= a.R;
  if (a.M != tails * a.R * a.R) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tails, (unsigned)((a.R * a.R + 255) / 256), (unsigned)((a.R + FQ_CW - 1) / FQ_CW));
  if (rm == 8)
    hipLaunchKernelGGL((form_q0_nested<8>), grid, dim3(256), 0, st, a);
  else if (rm == 16)
    hipLaunchKernelGGL((form_q0_nested<16>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((form_q0_nested<32>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------- factor QR
// QR of the I x R float64 factor `A` (column-major) by one workgroup.
// Writes Rn (R x R col-major, diag >= 0) and the explicit Q in the requested
// forms (any pointer may be null).
template <int RMAX, int RPT>
__global__ CPQR_QR_KERNEL(RMAX) void factor_qr(
    int I, int R, const double* __restrict__ A, double* __restrict__ Rn, double* __restrict__ q64,
    float* __restrict__ q32) {
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  const int tid = threadIdx.x;
  QrRow<RMAX> a[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = tid + QrCfg<RMAX>::NT * q;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[q].set(c, (row < I && c < R) ? A[row + (int64_t)I * c] : 0.0);
  }
  block_qr<RMAX, RPT>(a, R, sm);
  block_qr_publish<RMAX>(a[0], R, sm, wy, true);
  block_qr_wy_product<RMAX>(sm, wy, R, nullptr, 0);
  for (int e = tid; e < R * R; e += QrCfg<RMAX>::NT) {
    const int i = e % R, c = e / R;
    Rn[e] = wy.Rm[i][c];
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = tid + QrCfg<RMAX>::NT * q;
    if (row < I)
      block_qr_q_row<RMAX>(a[q], row, R, sm, wy, [&](int c, double val) {
        if (q64) q64[row + (int64_t)I * c] = val;
        if (q32) q32[row + (int64_t)I * c] = (float)val;
      });
  }
}

// ---------------------------------------------------------------- launchers
int qr_rmax(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : (R <= 32 ? 32 : 0)); }
// largest rows-per-thread instantiated at this column count (register budget)
static int qr_max_rpt(int rmax) { return rmax == 8 ? 8 : (rmax == 16 ? 4 : 2); }

TsqrPlan tsqr_plan(int64_t M, int R) {
  TsqrPlan pl{};
  const int rm = qr_rmax(R);
  if (rm == 0 || M < R) return pl;
  const int maxr = qr_max_rpt(rm);
  for (int rpt = 1; rpt <= maxr; rpt *= 2) {
    const int64_t rows = (int64_t)QrCfg<32>::NT * rpt;
    const int64_t P = (M + rows - 1) / rows;
    int top = 0;
    if (P > 1) {
      for (int t = 1; t <= maxr; t *= 2)
        if ((int64_t)QrCfg<32>::NT * t >= P * R) { top = t; break; }
      if (top == 0) continue;
    }
    pl.ok = true;
    pl.leaf_rpt = rpt;
    pl.leaf_rows = rows;
    pl.P = (int)P;
    pl.top_rpt = top;
    return pl;
  }
  return pl;
}

int64_t qr_leaf_rows(int R) { return (int64_t)QrCfg<32>::NT * qr_max_rpt(qr_rmax(R)); }

// Instantiated (RMAX, RPT) pairs.
#define CPQR_QR_SWITCH(RMAXV, RPTV, BODY)                                              \
  do {                                                                                 \
    if (RMAXV == 32) {                                                                 \
      constexpr int RM = 32;                                                           \
      if (RPTV == 1) { constexpr int RP = 1; BODY; }                                   \
      else if (RPTV == 2) { constexpr int RP = 2; BODY; }                              \
      else return hipErrorInvalidValue;                                                \
    } else if (RMAXV == 16) {                                                          \
      constexpr int RM = 16;                                                           \
      if (RPTV == 1) { constexpr int RP = 1; BODY; }                                   \
      else if (RPTV == 2) { constexpr int RP = 2; BODY; }                              \
      else if (RPTV == 4) { constexpr int RP = 4; BODY; }                              \
      else return hipErrorInvalidValue;                                                \
    } else if (RMAXV == 8) {                                                           \
      constexpr int RM = 8;                                                            \
      if (RPTV == 1) { constexpr int RP = 1; BODY; }                                   \
      else if (RPTV == 2) { constexpr int RP = 2; BODY; }                              \
      else if (RPTV == 4) { constexpr int RP = 4; BODY; }                              \
      else if (RPTV == 8) { constexpr int RP = 8; BODY; }                              \
      else return hipErrorInvalidValue;                                                \
    } else {                                                                           \
      return hipErrorInvalidValue;                                                     \
    }                                                                                  \
  } while (0)

void tsqr_args(const TsqrArgs& t, const TsqrPlan& pl, LeafArgs* la, TopArgs* ta, FormArgs* fa) {
  const bool single = (t.P == 1);
  *la = LeafArgs{t.N, t.n, t.R, t.P, t.rf, t.src, t.M, (int64_t)t.P * pl.leaf_rows, (int64_t)t.P * t.R,
                 t.V, t.T, t.stack, single ? t.R0 : nullptr, single ? t.Qtop : nullptr};
  *ta = TopArgs{t.R, single ? 0 : 1, (int64_t)t.P * t.R, t.stack, t.R0, t.Qtop};
  *fa = FormArgs{t.R, (int)pl.leaf_rows, t.M, (int64_t)t.P * pl.leaf_rows, (int64_t)t.P * t.R,
                 t.V, t.T, t.Qtop, t.Q0};
}

// The column-distributed leaf for leaves of `rows` rows in rank class 32
// (measured: 37 against 58 us for 512-row leaves at rank 20; in rank class
// 16 with 1024-row leaves it only ties zqr_leaf); false: zqr_leaf then.
static bool leaf_col_launch(int rm, int64_t rows, dim3 grid, const LeafArgs& la, const LeafArgs* batch,
                            hipStream_t st) {
  const dim3 blk(64 * LEAF_COL_NW);
#define CPQR_LC(RMV, RPV)                                                             \
  if (rm == RMV && rows == 64 * RPV) {                                                \
    hipLaunchKernelGGL((zqr_leaf_col<RMV, RPV>), grid, blk, 0, st, la, batch);        \
    return true;                                                                      \
  }
  CPQR_LC(32, 4) CPQR_LC(32, 8)
#undef CPQR_LC
  return false;
}

hipError_t launch_tsqr(const TsqrArgs& t, hipStream_t st) {
  const TsqrPlan pl = tsqr_plan(t.M, t.R);
  if (!pl.ok || pl.P != t.P) return hipErrorInvalidValue;
  const int rm = qr_rmax(t.R);
  LeafArgs la;
  TopArgs ta;
  FormArgs fa;
  tsqr_args(t, pl, &la, &ta, &fa);
  if (!leaf_col_launch(rm, pl.leaf_rows, dim3(t.P), la, nullptr, st)) {
    CPQR_QR_SWITCH(rm, pl.leaf_rpt, {
      hipLaunchKernelGGL((zqr_leaf<RM, RP>), dim3(t.P), dim3(QrCfg<RM>::NT), 0, st, la, nullptr);
    });
  }
  if (t.P > 1 && !top_col_launch(rm, ta.rows, dim3(1), ta, nullptr, st)) {
    CPQR_QR_SWITCH(rm, pl.top_rpt, {
      hipLaunchKernelGGL((zqr_top<RM, RP>), dim3(1), dim3(QrCfg<RM>::NT), 0, st, ta, nullptr);
    });
  }
  CPQR_QR_SWITCH(rm, 1, {
    (void)RP;
    const unsigned chunks = (unsigned)((t.M + QrCfg<RM>::NT - 1) / QrCfg<RM>::NT);
    hipLaunchKernelGGL((form_q0<RM>), dim3(chunks), dim3(QrCfg<RM>::NT), 0, st, fa, nullptr);
  });
  return hipGetLastError();
}

hipError_t launch_tsqr_batched(const TsqrBatch& b, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  const dim3 nb(1, (unsigned)b.count);
  if (!leaf_col_launch(b.rmax, (int64_t)QrCfg<32>::NT * b.leaf_rpt, dim3((unsigned)b.Pmax, (unsigned)b.count),
                       LeafArgs{}, b.leaf, st)) {
    CPQR_QR_SWITCH(b.rmax, b.leaf_rpt, {
      hipLaunchKernelGGL((zqr_leaf<RM, RP>), dim3((unsigned)b.Pmax, (unsigned)b.count), dim3(QrCfg<RM>::NT), 0,
                         st, LeafArgs{}, b.leaf);
    });
  }
  if (b.any_top &&
      !top_col_launch(b.rmax, (int64_t)QrCfg<32>::NT * b.top_rpt, nb, TopArgs{}, b.top, st)) {
    CPQR_QR_SWITCH(b.rmax, b.top_rpt, {
      hipLaunchKernelGGL((zqr_top<RM, RP>), nb, dim3(QrCfg<RM>::NT), 0, st, TopArgs{}, b.top);
    });
  }
  CPQR_QR_SWITCH(b.rmax, 1, {
    (void)RP;
    hipLaunchKernelGGL((form_q0<RM>), dim3(b.chunks, (unsigned)b.count), dim3(QrCfg<RM>::NT), 0, st,
                       FormArgs{}, b.form);
  });
  return hipGetLastError();
}

// Shapes of zqr_stair: all rows in slice 0 (Z_n of at most 256 rows), and
// order 3 at ranks 17..32 (rows 289..1024; the first 16 columns vanish
// beyond row 256, the narrow slices hold columns 16..31 of rows 256..1023).
StairPlan stair_plan(int N, int R) {
  StairPlan pl{};
  const int rm = qr_rmax(R);
  if (rm == 0 || N < 2 || N - 1 > qr_max_other_modes(rm)) return pl;
  int64_t M = 1;
  for (int k = 0; k < N - 1; ++k) M *= R;
  if (M <= QrCfg<32>::NT) {
    pl.ok = true;
    pl.rmax = rm;
    pl.ns = 0;
  } else if (N == 3 && rm == 32 && M <= 4 * QrCfg<32>::NT) {
    pl.ok = true;
    pl.rmax = 32;
    pl.ns = 3;
  }
  return pl;
}

static hipError_t stair_launch(const StairPlan& pl, unsigned blocks, const StairArgs& a,
                               const StairArgs* batch, hipStream_t st) {
  if (!pl.ok) return hipErrorInvalidValue;
  if (pl.ns == 0) {
    if (pl.rmax == 8)
      hipLaunchKernelGGL((zqr_stair<8, 0, 4, 4>), dim3(blocks), dim3(QrCfg<8>::NT), 0, st, a, batch);
    else if (pl.rmax == 16)
      hipLaunchKernelGGL((zqr_stair<16, 0, 8, 8>), dim3(blocks), dim3(QrCfg<16>::NT), 0, st, a, batch);
    else if (pl.rmax == 32)
      hipLaunchKernelGGL((zqr_stair<32, 0, 16, 16>), dim3(blocks), dim3(QrCfg<32>::NT), 0, st, a, batch);
    else
      return hipErrorInvalidValue;
  } else if (pl.rmax == 32 && pl.ns == 3) {
    hipLaunchKernelGGL((zqr_stair<32, 3, 16, 16>), dim3(blocks), dim3(QrCfg<32>::NT), 0, st, a, batch);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zqr_stair(const StairPlan& pl, const StairArgs& a, hipStream_t st) {
  if (!pl.ok || a.M > (int64_t)QrCfg<32>::NT * (pl.ns + 1) || a.R > pl.rmax) return hipErrorInvalidValue;
  return stair_launch(pl, 1, a, nullptr, st);
}

hipError_t launch_zqr_stair_batched(const StairPlan& pl, int count, const StairArgs* args, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return stair_launch(pl, (unsigned)count, StairArgs{}, args, st);
}

int factor_rpt(int I) { return I <= QrCfg<32>::NT ? 1 : 2; }

hipError_t launch_factor_qr(int I, int R, const double* A, double* Rn, double* q64, float* q32,
                            hipStream_t st) {
  if (I > CPQR_MAX_FACTOR_ROWS) return hipErrorInvalidValue;
  CPQR_QR_SWITCH(qr_rmax(R), factor_rpt(I), {
    hipLaunchKernelGGL((factor_qr<RM, RP>), dim3(1), dim3(QrCfg<RM>::NT), 0, st, I, R, A, Rn, q64, q32);
  });
  return hipGetLastError();
}

}  // namespace cpqr
