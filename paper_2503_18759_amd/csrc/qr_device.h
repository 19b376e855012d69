// Workgroup-level Householder QR of a tall block held in registers, with the
// compact WY factor T (Section 2.4 asks for compact QRs of the factor
// matrices and of Z_n; the sign convention is a non-negative diagonal of R).
//
// Layout: NT threads; thread t owns block rows t + NT p (p < RPT) and keeps
// each row's RMAX columns in vector registers (QrRow), so that the column of
// the current reflector can be read with one indexed register move.  Rows
// outside the matrix must be zero.  For column j the workgroup reduces, over
// the rows below the pivot, the RMAX values  sum_i x_i a_i[s]  (s = j gives
// the squared tail norm, s > j the dot products with the trailing columns,
// s < j the dot products with the earlier reflectors, which build T).  Per
// column: one wave-level transpose reduction, one LDS exchange of the wave
// partials behind a single barrier, and the reflector scalars computed by
// every wave redundantly (so no second barrier is needed); the dot products
// of column j+1 are formed while column j's update is applied.
//
// Reflector convention: x = column j from row j down; if the part below the
// pivot is exactly zero the reflector is the identity (tau = 0); otherwise
// beta = -sign(x0) ||x||, v = x / (x0 - beta) with v_j = 1, tau = (beta - x0) / beta.
// Then H_1 ... H_R = I - V T V^T with T upper triangular.
//
// Storage after the factorisation: below the diagonal, column j keeps x (the
// column as it was when its reflector was formed); the reflector is
// v = x * scale_j with scale_j = 1 / (x0 - beta) kept in LDS.  The pivot row j
// holds R[j][c] for c > j; R[j][j] = beta_j is kept in LDS.
#pragma once

#include <type_traits>

#include "common.h"

namespace cpqr {

// Workgroup size of the QR kernels: 256 threads, one wave per SIMD, so that
// each wave may use the whole register file (architectural plus accumulation
// registers) to keep its rows of the block resident.
template <int RMAX>
struct QrCfg {
  static constexpr int NT = 256;
  static constexpr int NW = NT / 64;
};
static constexpr int QR_MAX_WAVES = 4;

// Kernel attributes of the QR kernels: the workgroup size above, and the
// register budget of one workgroup per CU (the factorisation keeps its whole
// block in registers).
#define CPQR_QR_KERNEL(RMAX)                        \
  __launch_bounds__(QrCfg<RMAX>::NT)                \
  __attribute__((amdgpu_waves_per_eu(1, 1)))

typedef double f64x8 __attribute__((ext_vector_type(8)));
typedef double f64x16 __attribute__((ext_vector_type(16)));

// One row of the block: RMAX doubles in one or two register vectors of at
// most 16 elements (the largest the indexed register moves handle).
template <int RMAX>
struct QrRow {
  static constexpr int HW = RMAX > 16 ? 16 : RMAX;
  static constexpr int NH = RMAX / HW;
  using Vec = typename std::conditional<HW == 16, f64x16, f64x8>::type;
  Vec h[NH];
  __device__ __forceinline__ double get(int c) const {
    if constexpr (NH == 1) return h[0][c];
    else return (c < HW) ? h[0][c & (HW - 1)] : h[1][c & (HW - 1)];
  }
  __device__ __forceinline__ void set(int c, double x) {
    if constexpr (NH == 1) h[0][c] = x;
    else {
      if (c < HW) h[0][c & (HW - 1)] = x;
      else h[1][c & (HW - 1)] = x;
    }
  }
};

// LDS used by the factorisation itself.
template <int RMAX>
struct QrSmem {
  double piv[2][RMAX];
  double red[2][QR_MAX_WAVES][RMAX];
  double w[QR_MAX_WAVES][RMAX];   // per-wave copy of w_c (zero for c <= j)
  double U[RMAX][RMAX + 1];    // U[m][j] = (V^T v_j)_m for m < j
  double T[RMAX][RMAX + 1];
  double tau[RMAX];
  double beta[RMAX];
  double scale[RMAX];
  double sgn[RMAX];
};

// LDS used to form an explicit Q from the compact WY form.
template <int RMAX>
struct QrWySmem {
  double V1[RMAX][RMAX + 1];   // first R rows of V (unit lower triangular)
  double Rm[RMAX][RMAX + 1];   // R factor (after the sign fix when requested)
  double W[RMAX][RMAX + 1];    // scratch R x R product
  double M[RMAX][RMAX + 1];    // T V1^T B
};

// Reflector scalars from q = x0^2 + st (st = squared norm below the pivot):
// nrm = sqrt(q), beta = -sign(x0) nrm, tau = (|x0| + nrm) / nrm and
// scale = 1 / (x0 - beta) = sign(x0) / (|x0| + nrm).  The hardware reciprocal
// square root and reciprocal are refined by two Newton steps each (full
// double precision from their ~2^-22 start); outside a safe exponent range
// the exact library square root and divisions are used instead.
__device__ __forceinline__ void qr_reflector_scalars(double x0, double st, double* tau, double* beta,
                                                     double* scale) {
  if (st == 0.0) {
    *tau = 0.0;
    *beta = x0;
    *scale = 0.0;
    return;
  }
  const double q = fma(x0, x0, st);
  const double ax = fabs(x0);
  double nrm, rn, rd;
  if (q > 1e-280 && q < 1e280) {
    double y = __builtin_amdgcn_rsq(q);
    const double hq = 0.5 * q;
    y = y * fma(-hq * y, y, 1.5);
    y = y * fma(-hq * y, y, 1.5);
    nrm = q * y;
    rn = y;
    const double den = ax + nrm;
    double r = __builtin_amdgcn_rcp(den);
    r = r * fma(-den, r, 2.0);
    r = r * fma(-den, r, 2.0);
    rd = r;
  } else {
    nrm = sqrt(q);
    rn = 1.0 / nrm;
    rd = 1.0 / (ax + nrm);
  }
  const bool neg = x0 < 0.0;
  *beta = neg ? nrm : -nrm;
  *tau = (ax + nrm) * rn;
  *scale = neg ? -rd : rd;
}

// Factor the block (R <= RMAX columns); see the storage note above.
template <int RMAX, int RPT>
__device__ __forceinline__ void block_qr(QrRow<RMAX> (&a)[RPT], int R, QrSmem<RMAX>& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = QrCfg<RMAX>::NT;
  constexpr int G = 64 / RMAX;
  // column 0: pivot row, x and the dot products
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sm.piv[0][c] = a[0].get(c);
  }
  double x[RPT];
  double part[RMAX];
#pragma unroll
  for (int p = 0; p < RPT; ++p) x[p] = (tid + NT * p > 0) ? a[p].get(0) : 0.0;
#pragma unroll
  for (int s = 0; s < RMAX; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < RPT; ++p) acc = fma(x[p], a[p].get(s), acc);
    part[s] = acc;
  }
  for (int j = 0; j < R; ++j) {
    const int buf = j & 1;
    wave_transpose_reduce<RMAX>(part);
    if ((lane % G) == 0) sm.red[buf][wave][lane / G] = part[0];
    __syncthreads();
    // every wave: lane c < RMAX gets tot_c = sum_{i>j} x_i a_i[c]
    double tot = 0.0;
    if (lane < RMAX) {
#pragma unroll
      for (int w = 0; w < QrCfg<RMAX>::NW; ++w) tot += sm.red[buf][w][lane];
    }
    const double st = __shfl(tot, j, 64);
    const double x0 = sm.piv[buf][j];
    double tau, beta, scale;
    qr_reflector_scalars(x0, st, &tau, &beta, &scale);
    if (lane < RMAX) {
      // c > j: w_c = a_j[c] + scale * sum_{i>j} x_i a_i[c]  (v^T a_c with v_j = 1)
      // m < j: u_m = (V^T v_j)_m = scale_m (x_m[j] + scale * sum_{i>j} x_i x_m[i])
      const double pc = sm.piv[buf][lane];
      const double wu = fma(scale, tot, pc);
      sm.w[wave][lane] = (lane > j) ? wu : 0.0;
      if (wave == 0) sm.U[lane][j] = (lane < j) ? wu * sm.scale[lane] : 0.0;
    }
    if (wave == 0 && lane == 0) {
      sm.tau[j] = tau;
      sm.beta[j] = beta;
      sm.scale[j] = scale;
    }
    // the wave reads back its own copy of w (same wave: ordering only)
    __builtin_amdgcn_wave_barrier();
    double wv[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) wv[c] = sm.w[wave][c];
    // rows below the pivot: a -= tau v w^T with v = x scale; the pivot row:
    // a -= tau w^T (v_j = 1); w vanishes for c <= j.  Column j+1 is updated
    // first, then the remaining columns together with the dot products of
    // column j+1.
    const int jn = j + 1;
    double coef[RPT], xn[RPT];
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int row = tid + NT * p;
      coef[p] = (row > j) ? tau * x[p] * scale : ((row == j) ? tau : 0.0);
    }
    const double wn = (jn < RMAX) ? sm.w[wave][jn < RMAX ? jn : 0] : 0.0;
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int row = tid + NT * p;
      const double an = (jn < RMAX) ? fma(-coef[p], wn, a[p].get(jn < RMAX ? jn : 0)) : 0.0;
      xn[p] = (row > jn) ? an : 0.0;
    }
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < RPT; ++p) {
        const double v = fma(-coef[p], wv[s], a[p].get(s));
        a[p].set(s, v);
        acc = fma(xn[p], v, acc);
      }
      part[s] = acc;
    }
#pragma unroll
    for (int p = 0; p < RPT; ++p) x[p] = xn[p];
    if (tid == jn && jn < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) sm.piv[buf ^ 1][c] = a[0].get(c);
    }
  }
  __syncthreads();
  // T (upper triangular), row by row: T[k][k] = tau_k,
  // T[k][j] = -tau_j sum_{m=k}^{j-1} T[k][m] U[m][j]  (j > k)
  for (int e = tid; e < RMAX * (RMAX + 1); e += NT) (&sm.T[0][0])[e] = 0.0;
  __syncthreads();
  if (tid < R) {
    const int k = tid;
    sm.T[k][k] = sm.tau[k];
    for (int j = k + 1; j < R; ++j) {
      double acc = 0.0;
      for (int m = k; m < j; ++m) acc = fma(sm.T[k][m], sm.U[m][j], acc);
      sm.T[k][j] = -sm.tau[j] * acc;
    }
  }
  __syncthreads();
}

// Element (row, c) of the reflector matrix V (unit lower trapezoidal) for a
// row held by this thread as a[p].
template <int RMAX, int RPT>
__device__ __forceinline__ double block_qr_v(const QrRow<RMAX> (&a)[RPT], int p, int row, int c,
                                             const QrSmem<RMAX>& sm) {
  return (row > c) ? a[p].get(c) * sm.scale[c] : ((row == c) ? 1.0 : 0.0);
}

// Element (j, c) of the R factor (before the sign fix), from the thread that
// holds row j in `row0`.
template <int RMAX>
__device__ __forceinline__ double block_qr_r(const QrRow<RMAX>& row0, int j, int c,
                                             const QrSmem<RMAX>& sm) {
  return (c > j) ? row0.get(c) : ((c == j) ? sm.beta[j] : 0.0);
}

// After block_qr: publish the first R rows of V and the R factor to LDS,
// optionally fixing signs so that diag(R) >= 0 (sm.sgn holds the signs).
template <int RMAX, int RPT>
__device__ __forceinline__ void block_qr_publish(const QrRow<RMAX> (&a)[RPT], int R, QrSmem<RMAX>& sm,
                                                 QrWySmem<RMAX>& wy, bool fix_sign) {
  const int tid = threadIdx.x;
  if (tid < RMAX) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R);
      wy.V1[tid][c] = in ? block_qr_v<RMAX, RPT>(a, 0, tid, c, sm) : 0.0;
    }
    double sg = 1.0;
    if (fix_sign && tid < R && sm.beta[tid] < 0.0) sg = -1.0;
    sm.sgn[tid] = sg;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R);
      wy.Rm[tid][c] = in ? sg * block_qr_r<RMAX>(a[0], tid, c, sm) : 0.0;
    }
  }
  __syncthreads();
}

// wy.M = T * (V1^T * B) where B (R x R) is row-major in LDS with leading
// dimension ldb, or B = I when B == nullptr.
template <int RMAX>
__device__ __forceinline__ void block_qr_wy_product(const QrSmem<RMAX>& sm, QrWySmem<RMAX>& wy, int R,
                                                    const double* B, int ldb) {
  const int tid = threadIdx.x;
  for (int e = tid; e < RMAX * RMAX; e += QrCfg<RMAX>::NT) {
    const int k = e / RMAX, c = e % RMAX;
    double acc = 0.0;
    if (k < R && c < R) {
      if (B == nullptr) {
        acc = wy.V1[c][k];
      } else {
        for (int i = k; i < R; ++i) acc = fma(wy.V1[i][k], B[i * ldb + c], acc);
      }
    }
    wy.W[k][c] = acc;
  }
  __syncthreads();
  for (int e = tid; e < RMAX * RMAX; e += QrCfg<RMAX>::NT) {
    const int k = e / RMAX, c = e % RMAX;
    double acc = 0.0;
    for (int m = k; m < R; ++m) acc = fma(sm.T[k][m], wy.W[m][c], acc);
    wy.M[k][c] = acc;
  }
  __syncthreads();
}

// Row `row` (block-local) of the explicit Q = (E - V M) * diag(sgn) with
// M = T V1^T: store(c, value) for c < R; run-time loop over c.
template <int RMAX, int RPT, typename Store>
__device__ __forceinline__ void block_qr_q_row(const QrRow<RMAX> (&a)[RPT], int p, int R,
                                               const QrSmem<RMAX>& sm, const QrWySmem<RMAX>& wy,
                                               Store&& store) {
  const int row = threadIdx.x + QrCfg<RMAX>::NT * p;
  double v[RMAX];
#pragma unroll
  for (int m = 0; m < RMAX; ++m) v[m] = (m < R) ? block_qr_v<RMAX, RPT>(a, p, row, m, sm) : 0.0;
  for (int c = 0; c < R; ++c) {
    double acc = (row == c) ? 1.0 : 0.0;
#pragma unroll
    for (int m = 0; m < RMAX; ++m) acc = fma(-v[m], wy.M[m][c], acc);
    store(c, acc * sm.sgn[c]);
  }
}

// Sum V doubles over the whole workgroup; every thread receives the totals.
// `red` is LDS scratch of NW x V doubles (NW = waves in the workgroup).
template <int V, int NW>
__device__ __forceinline__ void block_allreduce(double (&v)[V], double (*red)[V]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  wave_transpose_reduce<V>(v);
  constexpr int G = 64 / V;
  if ((lane % G) == 0) red[wave][lane / G] = v[0];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < V; ++s) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w][s];
    v[s] = t;
  }
  __syncthreads();
}

}  // namespace cpqr
