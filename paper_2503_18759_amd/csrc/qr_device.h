// Workgroup-level Householder QR of a tall block held in registers, with the
// compact WY factor T accumulated on the fly (Section 2.4 asks for compact QRs
// of the factor matrices and of Z_n; the sign convention is a non-negative
// diagonal of R).
//
// Layout: 256 threads; thread t owns block rows t + 256 p (p < RPT) and keeps
// the row's RMAX columns in a[p][0..RMAX).  Rows outside the matrix must be
// zero.  For column j the workgroup reduces, over the rows below the pivot,
// the R values  sum_i x_i a_i[s]  (s = j gives the squared tail norm, s > j
// the dot products with the trailing columns, s < j the dot products with the
// earlier reflectors, which build column j of T).  One wave-level transpose
// reduction, one LDS exchange and one barrier per column.
//
// Reflector convention: x = column j from row j down; if the part below the
// pivot is exactly zero the reflector is the identity (tau = 0); otherwise
// beta = -sign(x0) ||x||, v = x / (x0 - beta) with v_j = 1, tau = (beta - x0) / beta.
// Then H_1 ... H_R = I - V T V^T with T upper triangular.
#pragma once

#include "common.h"

namespace cpqr {

static constexpr int QR_THREADS = 256;
static constexpr int QR_WAVES = QR_THREADS / 64;

// LDS used by the factorisation itself.
template <int RMAX>
struct QrSmem {
  double piv[2][RMAX];
  double red[2][QR_WAVES][RMAX];
  double T[RMAX][RMAX + 1];
  double beta[RMAX];
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

// Factor the block in a[][] (R <= RMAX columns).  On return:
//   a[p][c] for rows i > c holds V[i][c]; the pivot row j holds beta_j at
//   column j and R[j][c] for c > j;  sm.T = T, sm.beta[j] = beta_j.
template <int RMAX, int RPT>
__device__ void block_qr(double (&a)[RPT][RMAX], int R, QrSmem<RMAX>& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < RMAX * (RMAX + 1); e += QR_THREADS) (&sm.T[0][0])[e] = 0.0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    if (j < R) {
      const int buf = j & 1;
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < RMAX; ++c) sm.piv[buf][c] = a[0][c];
      }
      double part[RMAX];
#pragma unroll
      for (int s = 0; s < RMAX; ++s) part[s] = 0.0;
#pragma unroll
      for (int p = 0; p < RPT; ++p) {
        const int row = tid + QR_THREADS * p;
        const double x = (row > j) ? a[p][j] : 0.0;
#pragma unroll
        for (int s = 0; s < RMAX; ++s) part[s] = fma(x, a[p][s], part[s]);
      }
      wave_transpose_reduce<RMAX>(part);
      constexpr int G = 64 / RMAX;
      if ((lane % G) == 0) sm.red[buf][wave][lane / G] = part[0];
      __syncthreads();
      double tot[RMAX], pv[RMAX];
#pragma unroll
      for (int s = 0; s < RMAX; ++s) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < QR_WAVES; ++w) t += sm.red[buf][w][s];
        tot[s] = t;
        pv[s] = sm.piv[buf][s];
      }
      const double x0 = pv[j], st = tot[j];
      double tau, beta, scale;
      if (st == 0.0) {
        tau = 0.0;
        beta = x0;
        scale = 0.0;
      } else {
        const double nrm = sqrt(fma(x0, x0, st));
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      double w[RMAX];
#pragma unroll
      for (int c = 0; c < RMAX; ++c) w[c] = (c > j) ? fma(scale, tot[c], pv[c]) : 0.0;
#pragma unroll
      for (int p = 0; p < RPT; ++p) {
        const int row = tid + QR_THREADS * p;
        if (row > j) {
          const double v = a[p][j] * scale;
          a[p][j] = v;
          const double tv = tau * v;
#pragma unroll
          for (int c = j + 1; c < RMAX; ++c) a[p][c] = fma(-tv, w[c], a[p][c]);
        } else if (row == j) {
          a[p][j] = beta;
#pragma unroll
          for (int c = j + 1; c < RMAX; ++c) a[p][c] = fma(-tau, w[c], a[p][c]);
        }
      }
      // column j of T:  T[k][j] = -tau sum_{m<j} T[k][m] u_m,  u_m = (V^T v_j)_m
      if (tid < j) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < j; ++m) acc = fma(sm.T[tid][m], fma(scale, tot[m], pv[m]), acc);
        sm.T[tid][j] = -tau * acc;
      }
      if (tid == j) {
        sm.T[j][j] = tau;
        sm.beta[j] = beta;
      }
    }
  }
  __syncthreads();
}

// After block_qr: publish the first R rows of V and the R factor to LDS,
// optionally fixing signs so that diag(R) >= 0 (sm.sgn holds the signs).
template <int RMAX, int RPT>
__device__ void block_qr_publish(const double (&a)[RPT][RMAX], int R, QrSmem<RMAX>& sm,
                                 QrWySmem<RMAX>& wy, bool fix_sign) {
  const int tid = threadIdx.x;
  if (tid < RMAX) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R);
      wy.V1[tid][c] = !in ? 0.0 : (c < tid ? a[0][c] : (c == tid ? 1.0 : 0.0));
    }
    double sg = 1.0;
    if (fix_sign && tid < R && sm.beta[tid] < 0.0) sg = -1.0;
    sm.sgn[tid] = sg;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R) && (c >= tid);
      wy.Rm[tid][c] = in ? sg * a[0][c] : 0.0;
    }
  }
  __syncthreads();
}

// wy.M = T * (V1^T * B) where B (R x R) is row-major in LDS with leading
// dimension ldb, or B = I when B == nullptr.
template <int RMAX>
__device__ void block_qr_wy_product(const QrSmem<RMAX>& sm, QrWySmem<RMAX>& wy, int R,
                                    const double* B, int ldb) {
  const int tid = threadIdx.x;
  for (int e = tid; e < RMAX * RMAX; e += QR_THREADS) {
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
  for (int e = tid; e < RMAX * RMAX; e += QR_THREADS) {
    const int k = e / RMAX, c = e % RMAX;
    double acc = 0.0;
    for (int m = k; m < R; ++m) acc = fma(sm.T[k][m], wy.W[m][c], acc);
    wy.M[k][c] = acc;
  }
  __syncthreads();
}

// Row i (block-local) of the explicit Q = (E - V M) with E the first R
// columns of the identity, M = T V1^T (B = I case), times the sign fix.
template <int RMAX, int RPT>
__device__ inline void block_qr_q_row(const double (&a)[RPT][RMAX], int p, int R,
                                      const QrSmem<RMAX>& sm, const QrWySmem<RMAX>& wy,
                                      double (&q)[RMAX]) {
  const int row = threadIdx.x + QR_THREADS * p;
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = (row == c) ? 1.0 : 0.0;
#pragma unroll
  for (int m = 0; m < RMAX; ++m) {
    const double v = (row > m) ? a[p][m] : ((row == m) ? 1.0 : 0.0);
    if (m < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) q[c] = fma(-v, wy.M[m][c], q[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] *= sm.sgn[c];
}

}  // namespace cpqr

namespace cpqr {

// Sum V doubles over the whole workgroup; every thread receives the totals.
// `red` is LDS scratch of QR_WAVES x V doubles.
template <int V>
__device__ void block_allreduce(double (&v)[V], double (*red)[V]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  wave_transpose_reduce<V>(v);
  constexpr int G = 64 / V;
  if ((lane % G) == 0) red[wave][lane / G] = v[0];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < V; ++s) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < QR_WAVES; ++w) t += red[w][s];
    v[s] = t;
  }
  __syncthreads();
}

}  // namespace cpqr
