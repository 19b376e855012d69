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
  // Element c for a wave-uniform c, as a binary tree of uniform branches
  // whose leaves read a fixed register (get_u).  get() with a variable index
  // into two halves compiles to a select of the whole vectors, a move per
  // element; the tree avoids those moves, which pays where a thread holds one
  // row, and costs registers where it holds several.  The empty asm
  // statements keep the branches from being merged into selects.
  template <int LO, int HI>
  __device__ __forceinline__ double get_tree(int c) const {
    if constexpr (HI - LO == 1) {
      return h[LO / HW][LO % HW];
    } else {
      constexpr int MID = (LO + HI) / 2;
      double x;
      if (c < MID) {
        __asm__ volatile("");
        x = get_tree<LO, MID>(c);
      } else {
        __asm__ volatile("");
        x = get_tree<MID, HI>(c);
      }
      return x;
    }
  }
  __device__ __forceinline__ double get_u(int c) const {
    if constexpr (NH == 1) return h[0][c];
    else return get_tree<0, RMAX>(c);
  }
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
  double Mt[RMAX][RMAX + 2];   // (T V1^T B)^T: row c holds column c (16-byte aligned rows)
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

// T (upper triangular) of the compact WY form from the U entries collected
// during the factorisation: T[k][k] = tau_k and
// T[k][j] = -tau_j sum_{m=k}^{j-1} T[k][m] U[m][j] for j > k.  Lane k owns
// row k in registers; the loops are unrolled so that the U reads (the same
// address for every lane) are issued ahead of the arithmetic, and the term
// of the newest entry T[k][j-1] is added last to keep the dependent chain
// at one multiply-add per column.
template <int RMAX>
__device__ __forceinline__ void block_qr_build_t(int R, QrSmem<RMAX>& sm) {
  const int tid = threadIdx.x;
  if (tid < RMAX) {
    const int k = tid;
    double t[RMAX];
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      double u[RMAX];
#pragma unroll
      for (int m = 0; m < j; ++m) u[m] = sm.U[m][j];
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m + 1 < j; ++m) acc = fma(t[m], u[m], acc);
      if (j > 0) acc = fma(t[j - 1], u[j - 1], acc);
      // entries left of the diagonal are zero; columns j >= R are padding
      // (their U entries are never written, so they are selected away)
      t[j] = (j < k || j >= R) ? 0.0 : ((j == k) ? sm.tau[j] : -sm.tau[j] * acc);
    }
#pragma unroll
    for (int j = 0; j < RMAX; ++j) sm.T[k][j] = t[j];
  }
  __syncthreads();
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
    // every LDS operand of this step is read before any is used, so that the
    // reads are in flight together: the wave partials, the pivot row and the
    // reflector scales of the previous columns (written before the barrier)
    double tot = 0.0, pc = 0.0, scl = 0.0;
    const double x0 = sm.piv[buf][j];
    if (lane < RMAX) {
      double rv[QrCfg<RMAX>::NW];
#pragma unroll
      for (int w = 0; w < QrCfg<RMAX>::NW; ++w) rv[w] = sm.red[buf][w][lane];
      pc = sm.piv[buf][lane];
      scl = sm.scale[lane];
#pragma unroll
      for (int w = 0; w < QrCfg<RMAX>::NW; ++w) tot += rv[w];
    }
    const double st = lane_read(tot, j);
    double tau, beta, scale;
    qr_reflector_scalars(x0, st, &tau, &beta, &scale);
    if (lane < RMAX) {
      // c > j: w_c = a_j[c] + scale * sum_{i>j} x_i a_i[c]  (v^T a_c with v_j = 1)
      // m < j: u_m = (V^T v_j)_m = scale_m (x_m[j] + scale * sum_{i>j} x_i x_m[i])
      const double wu = fma(scale, tot, pc);
      sm.w[wave][lane] = (lane > j) ? wu : 0.0;
      if (wave == 0) sm.U[lane][j] = (lane < j) ? wu * scl : 0.0;
    }
    if (wave == 0 && lane == 0) {
      sm.tau[j] = tau;
      sm.beta[j] = beta;
      sm.scale[j] = scale;
    }
    // the wave reads back its own copy of w: one wave's LDS operations
    // complete in order, so no wait is needed between the write and the reads
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
      const int jc = jn < RMAX ? jn : 0;
      const double ajn = (RPT == 1) ? a[p].get_u(jc) : a[p].get(jc);
      const double an = (jn < RMAX) ? fma(-coef[p], wn, ajn) : 0.0;
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
  block_qr_build_t<RMAX>(R, sm);
}

// ------------------------------------------------------------ staircase QR
// Householder QR of Z_n with its rows in staircase order.  Section 3.2 notes
// the triangular structure of Q0 and Section 5 names exploiting it as a way
// to cut the cost of Q0, its main bottleneck.  Column c of Z_n is the product,
// row by row, of the columns c of the upper triangular R factors of the other
// modes, so it vanishes at every row one of whose K digits (indices into the
// other modes) exceeds c.  With the rows ordered by their largest digit, the
// nonzeros of column c are the first (c+1)^K rows (its profile), and the
// Householder reflectors keep that profile.
//
// Layout: slice 0 (row tid) holds all RMAX columns; the narrow slices
// q = 0..NS-1 hold rows NT (q+1) + tid and only the RT columns [CS, CS+RT),
// because the first CS columns vanish beyond row CS^K <= NT.  A narrow slice
// takes part in a column step only once its first row lies in the column's
// profile, so early columns run on slice 0 alone.  Requires R <= CS + RT
// and R <= NT; otherwise the storage and reflector conventions of block_qr
// hold (a narrow row keeps x of reflector c in its column c - CS).
template <int RMAX, int NS, int RT, int CS>
struct QrStair {
  QrRow<RMAX> a0;
  QrRow<RT> at[NS > 0 ? NS : 1];
};

// Rows in the profile of column c: min(M, (c+1)^K).
__device__ __forceinline__ int64_t stair_profile(int c, int K, int64_t M) {
  int64_t p = 1;
  for (int k = 0; k < K; ++k) p *= (int64_t)(c + 1);
  return p < M ? p : M;
}

template <int RMAX, int NS, int RT, int CS>
__device__ __forceinline__ void block_qr_stair(QrStair<RMAX, NS, RT, CS>& z, int R, int K, int64_t M,
                                               QrSmem<RMAX>& sm) {
  static_assert(CS >= 1 && CS + RT <= RMAX, "narrow columns must lie inside the block");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT = QrCfg<RMAX>::NT;
  constexpr int G = 64 / RMAX;
  constexpr int NSA = NS > 0 ? NS : 1;
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sm.piv[0][c] = z.a0.get(c);
  }
  // x of the current column below the pivot: slice 0 and the narrow slices
  // (which vanish in column 0 < CS)
  double xs0 = (tid > 0) ? z.a0.get(0) : 0.0;
  double xt[NSA];
#pragma unroll
  for (int q = 0; q < NSA; ++q) xt[q] = 0.0;
  double part[RMAX];
#pragma unroll
  for (int s = 0; s < RMAX; ++s) part[s] = xs0 * z.a0.get(s);
  for (int j = 0; j < R; ++j) {
    const int buf = j & 1;
    wave_transpose_reduce<RMAX>(part);
    if ((lane % G) == 0) sm.red[buf][wave][lane / G] = part[0];
    __syncthreads();
    // every LDS operand of this step is read before any is used, so that the
    // reads are in flight together: the wave partials, the pivot row and the
    // reflector scales of the previous columns (written before the barrier)
    double tot = 0.0, pc = 0.0, scl = 0.0;
    const double xp = sm.piv[buf][j];
    if (lane < RMAX) {
      double rv[QrCfg<RMAX>::NW];
#pragma unroll
      for (int w = 0; w < QrCfg<RMAX>::NW; ++w) rv[w] = sm.red[buf][w][lane];
      pc = sm.piv[buf][lane];
      scl = sm.scale[lane];
#pragma unroll
      for (int w = 0; w < QrCfg<RMAX>::NW; ++w) tot += rv[w];
    }
    const double st = lane_read(tot, j);
    double tau, beta, scale;
    qr_reflector_scalars(xp, st, &tau, &beta, &scale);
    if (lane < RMAX) {
      const double wu = fma(scale, tot, pc);
      sm.w[wave][lane] = (lane > j) ? wu : 0.0;
      if (wave == 0) sm.U[lane][j] = (lane < j) ? wu * scl : 0.0;
    }
    if (wave == 0 && lane == 0) {
      sm.tau[j] = tau;
      sm.beta[j] = beta;
      sm.scale[j] = scale;
    }
    // the wave reads w back from its own LDS copy as the columns are updated
    // (keeping all of w in registers as well would not fit beside the rows);
    // one wave's LDS operations complete in order
    const int jn = j + 1;
    // narrow slices inside the profile of column min(jn, R-1); the profile
    // of column j is contained in it, so every slice the reflector changes
    // is among them
    const int64_t prof = stair_profile(jn < R ? jn : R - 1, K, M);
    int na = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) na += ((int64_t)NT * (q + 1) < prof) ? 1 : 0;
    const double coef0 = (tid > j) ? tau * xs0 * scale : ((tid == j) ? tau : 0.0);
    double coef[NSA];
#pragma unroll
    for (int q = 0; q < NSA; ++q) coef[q] = tau * xt[q] * scale;
    const double wn = (jn < RMAX) ? sm.w[wave][jn < RMAX ? jn : 0] : 0.0;
    const double an0 = (jn < RMAX) ? fma(-coef0, wn, z.a0.get(jn < RMAX ? jn : 0)) : 0.0;
    const double xn0 = (tid > jn) ? an0 : 0.0;
    const int jt = (jn - CS < 0) ? 0 : ((jn - CS >= RT) ? RT - 1 : jn - CS);
    const bool jin = (jn >= CS) && (jn - CS < RT);
    // one branch-free body per count of active narrow slices
    static_for<0, NS + 1>([&](auto nac) {
      constexpr int NA = decltype(nac)::value;
      if (na != NA) return;
      double xnt[NA > 0 ? NA : 1];
      static_for<0, NA>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        xnt[q] = jin ? fma(-coef[q], wn, z.at[q].get(jt)) : 0.0;
      });
      static_for<0, RMAX>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const double ws = sm.w[wave][s];
        const double v = fma(-coef0, ws, z.a0.get(s));
        z.a0.set(s, v);
        double acc = xn0 * v;
        if constexpr (s >= CS && s - CS < RT) {
          static_for<0, NA>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const double vt = fma(-coef[q], ws, z.at[q].get(s - CS));
            z.at[q].set(s - CS, vt);
            acc = fma(xnt[q], vt, acc);
          });
        }
        part[s] = acc;
      });
      static_for<0, NSA>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q < NA) xt[q] = xnt[q];
        else xt[q] = 0.0;
      });
    });
    xs0 = xn0;
    if (tid == jn && jn < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) sm.piv[buf ^ 1][c] = z.a0.get(c);
    }
  }
  __syncthreads();
  block_qr_build_t<RMAX>(R, sm);
}

// Element (row, c) of the reflector matrix V (unit lower trapezoidal) for a
// row held by this thread in `r` (c is a column index of r).
template <int RMAX>
__device__ __forceinline__ double block_qr_v(const QrRow<RMAX>& r, int row, int c, const QrSmem<RMAX>& sm) {
  return (row > c) ? r.get(c) * sm.scale[c] : ((row == c) ? 1.0 : 0.0);
}

// Element (j, c) of the R factor (before the sign fix), from the thread that
// holds row j in `row0`.
template <int RMAX>
__device__ __forceinline__ double block_qr_r(const QrRow<RMAX>& row0, int j, int c,
                                             const QrSmem<RMAX>& sm) {
  return (c > j) ? row0.get(c) : ((c == j) ? sm.beta[j] : 0.0);
}

// After the factorisation: publish the first R rows of V and the R factor to
// LDS (row0 is the thread's row of slice 0, which holds rows 0..R-1),
// optionally fixing signs so that diag(R) >= 0 (sm.sgn holds the signs).
template <int RMAX>
__device__ __forceinline__ void block_qr_publish(const QrRow<RMAX>& row0, int R, QrSmem<RMAX>& sm,
                                                 QrWySmem<RMAX>& wy, bool fix_sign) {
  const int tid = threadIdx.x;
  if (tid < RMAX) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R);
      wy.V1[tid][c] = in ? block_qr_v<RMAX>(row0, tid, c, sm) : 0.0;
    }
    double sg = 1.0;
    if (fix_sign && tid < R && sm.beta[tid] < 0.0) sg = -1.0;
    sm.sgn[tid] = sg;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = (tid < R) && (c < R);
      wy.Rm[tid][c] = in ? sg * block_qr_r<RMAX>(row0, tid, c, sm) : 0.0;
    }
  }
  __syncthreads();
}

// wy.Mt = (T * (V1^T * B))^T where B (R x R) is row-major in LDS with leading
// dimension ldb, or B = I when B == nullptr.  The inner products run over
// the full (zero-padded) RMAX range, unrolled, so that their LDS reads are
// issued together rather than one loop trip at a time.  NTH is the
// workgroup's thread count.
template <int RMAX, int NTH = QrCfg<RMAX>::NT>
__device__ __forceinline__ void block_qr_wy_product(const QrSmem<RMAX>& sm, QrWySmem<RMAX>& wy, int R,
                                                    const double* B, int ldb) {
  const int tid = threadIdx.x;
  if (B != nullptr) {
    // W = V1^T B (V1 is zero above its unit diagonal and beyond R)
    for (int e = tid; e < RMAX * RMAX; e += NTH) {
      const int k = e / RMAX, c = e % RMAX;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < RMAX; ++i) acc = fma(wy.V1[i][k], (c < R) ? B[i * ldb + (c < R ? c : 0)] : 0.0, acc);
      wy.W[k][c] = acc;
    }
  } else {
    for (int e = tid; e < RMAX * RMAX; e += NTH) {
      const int k = e / RMAX, c = e % RMAX;
      wy.W[k][c] = wy.V1[c][k];
    }
  }
  __syncthreads();
  // M = T W (T is zero below its diagonal and beyond R)
  for (int e = tid; e < RMAX * RMAX; e += NTH) {
    const int k = e / RMAX, c = e % RMAX;
    double tk[RMAX], wc[RMAX];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) tk[m] = sm.T[k][m];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) wc[m] = wy.W[m][c];
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int m = 0; m < RMAX; m += 2) {
      a0 = fma(tk[m], wc[m], a0);
      a1 = fma(tk[m + 1], wc[m + 1], a1);
    }
    wy.Mt[c][k] = (k < R && c < R) ? a0 + a1 : 0.0;
  }
  __syncthreads();
}

// Row `row` of the explicit Q = (E - V M) * diag(sgn) with M = T V1^T, from
// the row's reflector entries v[m] = V[row][OFF + m] (zero outside
// [OFF, OFF + W)): store(c, value) for c < R.  Two columns per trip and two
// partial sums per column keep four independent multiply-add chains, and
// the two M entries of a trip are adjacent in LDS.
template <int RMAX, int W, int OFF, typename Store>
__device__ __forceinline__ void wy_q_row(const double (&v)[W], int64_t row, int R, const QrSmem<RMAX>& sm,
                                         const QrWySmem<RMAX>& wy, Store&& store) {
  static_assert(W % 2 == 0 && RMAX % 2 == 0, "pairs of rows and columns");
  // M = T V1^T is upper triangular (T upper, V1 unit lower triangular):
  // M[m][c] = 0 for m > c, so the blocks of reflectors past c + 1 contribute
  // exact zeros to columns c, c + 1 and are skipped (a uniform test per
  // block keeps every register index fixed)
  constexpr int MB = W < 8 ? W : 8;
  static_assert(W % MB == 0, "blocks of reflectors");
  for (int c = 0; c < R; c += 2) {
    // c + 1 <= RMAX - 1 (R <= RMAX, RMAX even); M is zero in columns >= R
    double a0 = (row == c) ? 1.0 : 0.0, a1 = (row == c + 1) ? 1.0 : 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int mb = 0; mb < W; mb += MB) {
      if (OFF + mb > c + 1) break;
      double m0[MB], m1[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        m0[m] = wy.Mt[c][OFF + mb + m];
        m1[m] = wy.Mt[c + 1][OFF + mb + m];
      }
#pragma unroll
      for (int m = 0; m < MB; m += 2) {
        a0 = fma(-v[mb + m], m0[m], a0);
        a1 = fma(-v[mb + m], m1[m], a1);
        b0 = fma(-v[mb + m + 1], m0[m + 1], b0);
        b1 = fma(-v[mb + m + 1], m1[m + 1], b1);
      }
    }
    store(c, (a0 + b0) * sm.sgn[c]);
    if (c + 1 < R) store(c + 1, (a1 + b1) * sm.sgn[c + 1]);
  }
}

// Row `row` (block-local) of the explicit Q for a row held in `r`.
template <int RMAX, typename Store>
__device__ __forceinline__ void block_qr_q_row(const QrRow<RMAX>& r, int row, int R, const QrSmem<RMAX>& sm,
                                               const QrWySmem<RMAX>& wy, Store&& store) {
  double v[RMAX];
#pragma unroll
  for (int m = 0; m < RMAX; ++m) v[m] = (m < R) ? block_qr_v<RMAX>(r, row, m, sm) : 0.0;
  wy_q_row<RMAX, RMAX, 0>(v, row, R, sm, wy, store);
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
