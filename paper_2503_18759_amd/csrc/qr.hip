// Householder QR kernels (Section 2.4 / Algorithm 2, lines "QR of the factor
// matrices" and "QR decomposition Z_n = Q0 R0").
//
//  * zqr_leaf:  TSQR leaves of Z_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1
//               (Khatri-Rao of the R factors, rows in the Kolda order of the
//               remaining modes, smallest mode fastest).  Each workgroup
//               builds its block of rows from the R factors in LDS, factors it
//               and writes V, T and its R factor (into the stack of leaf
//               triangles).  Also used on an explicit matrix.
//  * zqr_top:   QR of the stacked leaf triangles; writes R0 (diag >= 0) and
//               the explicit Q of the stack with the sign fix applied.
//  * form_q0:   explicit Q0 rows of each leaf: Q0_p = E Qtop_p - V_p (T_p V_p1^T Qtop_p).
//  * factor_qr: QR of an I x R factor held by one workgroup; writes R_n and
//               the explicit Q_n in float64 / float32 / bf16 hi+lo.
#include "common.h"
#include "kernels.h"
#include "qr_device.h"

namespace cpqr {

// ----------------------------------------------------------------- leaves
// src == nullptr: build rows of Z from the R factors in `rf` (N x R x R,
// column-major, factor n skipped).  Otherwise read rows of the M x R
// column-major matrix `src`.
template <int RMAX, int RPT>
__global__ __launch_bounds__(QR_THREADS) void zqr_leaf(
    int N, int n, int R, const double* __restrict__ rf, const double* __restrict__ src,
    int64_t M, double* __restrict__ V, double* __restrict__ Tbuf, double* __restrict__ stack,
    int64_t ldstack) {
  __shared__ QrSmem<RMAX> sm;
  __shared__ double srf[(CPQR_MAX_ORDER - 1) * RMAX * RMAX];
  constexpr int B = QR_THREADS * RPT;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  int modes[CPQR_MAX_ORDER];
  int nm = 0;
  if (src == nullptr) {
    for (int k = 0; k < N; ++k)
      if (k != n) modes[nm++] = k;
    for (int e = tid; e < nm * R * R; e += QR_THREADS) {
      const int q = e / (R * R), rem = e % (R * R);
      srf[e] = rf[(int64_t)modes[q] * R * R + rem];
    }
    __syncthreads();
  }
  double a[RPT][RMAX];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = (int64_t)p * B + tid + QR_THREADS * q;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[q][c] = 0.0;
    if (row < M) {
      if (src == nullptr) {
        // digits of row in base R, first remaining mode fastest
        int dig[CPQR_MAX_ORDER];
        int64_t rr = row;
        for (int k = 0; k < nm; ++k) {
          dig[k] = (int)(rr % R);
          rr /= R;
        }
#pragma unroll
        for (int c = 0; c < RMAX; ++c) {
          if (c < R) {
            double prod = 1.0;
            for (int k = 0; k < nm; ++k) prod *= srf[k * R * R + dig[k] + R * c];
            a[q][c] = prod;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < RMAX; ++c)
          if (c < R) a[q][c] = src[row + M * c];
      }
    }
  }
  block_qr<RMAX, RPT>(a, R, sm);
  // V rows (unit lower trapezoidal) for all B rows of the block
  const int64_t ldv = (int64_t)gridDim.x * B;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int lr = tid + QR_THREADS * q;
    const int64_t row = (int64_t)p * B + lr;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      if (c < R) {
        const double v = (lr > c) ? a[q][c] : ((lr == c) ? 1.0 : 0.0);
        V[row + ldv * c] = v;
      }
    }
  }
  // leaf R (no sign fix) into the stack, T into Tbuf
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) stack[(int64_t)p * R + tid + ldstack * c] = (c >= tid) ? a[0][c] : 0.0;
  }
  for (int e = tid; e < R * R; e += QR_THREADS) {
    const int k = e % R, c = e / R;
    Tbuf[(int64_t)p * R * R + e] = sm.T[k][c];
  }
}

// --------------------------------------------------------------------- top
// QR of the P*R x R stack.  Writes R0 (R x R column-major, diag >= 0) and
// Qtop (P*R x R column-major) = explicit Q of the stack times the sign fix.
template <int RMAX, int RPT>
__global__ __launch_bounds__(QR_THREADS) void zqr_top(
    int R, int64_t rows, const double* __restrict__ stack, double* __restrict__ R0,
    double* __restrict__ Qtop) {
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  const int tid = threadIdx.x;
  double a[RPT][RMAX];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = tid + QR_THREADS * q;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[q][c] = (row < rows && c < R) ? stack[row + rows * c] : 0.0;
  }
  block_qr<RMAX, RPT>(a, R, sm);
  block_qr_publish<RMAX, RPT>(a, R, sm, wy, true);
  block_qr_wy_product<RMAX>(sm, wy, R, nullptr, 0);
  for (int e = tid; e < R * R; e += QR_THREADS) {
    const int i = e % R, c = e / R;
    R0[e] = wy.Rm[i][c];
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = tid + QR_THREADS * q;
    double qq[RMAX];
    block_qr_q_row<RMAX, RPT>(a, q, R, sm, wy, qq);
    if (row < rows) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c)
        if (c < R) Qtop[row + rows * c] = qq[c];
    }
  }
}

// ------------------------------------------------------------------ form Q0
// One workgroup per 256-row chunk.  Chunk rows lie inside one leaf p.
template <int RMAX>
__global__ __launch_bounds__(QR_THREADS) void form_q0(
    int R, int64_t M, int leaf_rows, const double* __restrict__ V, int64_t ldv,
    const double* __restrict__ Tbuf, const double* __restrict__ Qtop, int64_t ldq,
    double* __restrict__ Q0) {
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  __shared__ double sQt[RMAX * RMAX];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * QR_THREADS;
  const int p = (int)(row0 / leaf_rows);
  const int64_t leaf0 = (int64_t)p * leaf_rows;
  // V1 of the leaf, T of the leaf, Qtop block p (row-major in LDS)
  for (int e = tid; e < RMAX * RMAX; e += QR_THREADS) {
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
  double q[RMAX];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = (lr < R && c < R) ? sQt[lr * RMAX + c] : 0.0;
#pragma unroll
  for (int m = 0; m < RMAX; ++m) {
    if (m < R) {
      const double v = V[row + ldv * m];
#pragma unroll
      for (int c = 0; c < RMAX; ++c) q[c] = fma(-v, wy.M[m][c], q[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c)
    if (c < R) Q0[row + M * c] = q[c];
}

// ------------------------------------------------------------- factor QR
// QR of the I x R float64 factor `A` (column-major) by one workgroup.
// Writes Rn (R x R col-major, diag >= 0) and the explicit Q in the requested
// forms (any pointer may be null).
template <int RMAX, int RPT>
__global__ __launch_bounds__(QR_THREADS) void factor_qr(
    int I, int R, const double* __restrict__ A, double* __restrict__ Rn, double* __restrict__ q64,
    float* __restrict__ q32) {
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  const int tid = threadIdx.x;
  double a[RPT][RMAX];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = tid + QR_THREADS * q;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[q][c] = (row < I && c < R) ? A[row + (int64_t)I * c] : 0.0;
  }
  block_qr<RMAX, RPT>(a, R, sm);
  block_qr_publish<RMAX, RPT>(a, R, sm, wy, true);
  block_qr_wy_product<RMAX>(sm, wy, R, nullptr, 0);
  for (int e = tid; e < R * R; e += QR_THREADS) {
    const int i = e % R, c = e / R;
    Rn[e] = wy.Rm[i][c];
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = tid + QR_THREADS * q;
    double qq[RMAX];
    block_qr_q_row<RMAX, RPT>(a, q, R, sm, wy, qq);
    if (row < I) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        if (c < R) {
          if (q64) q64[row + (int64_t)I * c] = qq[c];
          if (q32) q32[row + (int64_t)I * c] = (float)qq[c];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
int qr_rmax(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : (R <= 32 ? 32 : 0)); }
int qr_rpt(int rmax) { return rmax == 8 ? 8 : (rmax == 16 ? 4 : 2); }
int64_t qr_leaf_rows(int R) { const int rm = qr_rmax(R); return rm ? (int64_t)QR_THREADS * qr_rpt(rm) : 0; }

#define CPQR_QR_DISPATCH(R, BODY)                   \
  do {                                              \
    const int rm__ = qr_rmax(R);                    \
    if (rm__ == 8) { constexpr int RM = 8, RP = 8; BODY; }        \
    else if (rm__ == 16) { constexpr int RM = 16, RP = 4; BODY; } \
    else if (rm__ == 32) { constexpr int RM = 32, RP = 2; BODY; } \
    else return hipErrorInvalidValue;               \
  } while (0)

hipError_t launch_tsqr(const TsqrArgs& t, hipStream_t st) {
  CPQR_QR_DISPATCH(t.R, {
    hipLaunchKernelGGL((zqr_leaf<RM, RP>), dim3(t.P), dim3(QR_THREADS), 0, st, t.N, t.n, t.R, t.rf,
                       t.src, t.M, t.V, t.T, t.stack, (int64_t)t.P * t.R);
    hipLaunchKernelGGL((zqr_top<RM, RP>), dim3(1), dim3(QR_THREADS), 0, st, t.R, (int64_t)t.P * t.R,
                       t.stack, t.R0, t.Qtop);
    const unsigned chunks = (unsigned)((t.M + QR_THREADS - 1) / QR_THREADS);
    hipLaunchKernelGGL((form_q0<RM>), dim3(chunks), dim3(QR_THREADS), 0, st, t.R, t.M,
                       (int)qr_leaf_rows(t.R), t.V, (int64_t)t.P * qr_leaf_rows(t.R), t.T, t.Qtop,
                       (int64_t)t.P * t.R, t.Q0);
  });
  return hipGetLastError();
}

hipError_t launch_factor_qr(int I, int R, const double* A, double* Rn, double* q64, float* q32,
                            hipStream_t st) {
  CPQR_QR_DISPATCH(R, {
    hipLaunchKernelGGL((factor_qr<RM, RP>), dim3(1), dim3(QR_THREADS), 0, st, I, R, A, Rn, q64, q32);
  });
  return hipGetLastError();
}

}  // namespace cpqr
