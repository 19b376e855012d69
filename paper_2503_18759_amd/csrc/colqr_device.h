// Column-distributed Householder QR of a block held in registers (the
// compact QRs of Section 2.4: the factor QR of every mode update and the QR
// Z_n = Q0 R0 of Algorithm 2), for one workgroup of NW waves (4: one per
// SIMD, 8: two per SIMD, for blocks whose rows do not fit four waves'
// registers).
//
// Layout: wave w owns the CPW = RMAX / NW consecutive columns
// [CPW w, CPW w + CPW) of the block, every row of them: lane l holds rows
// l + 64 p (p < RPL) of its columns in a[p][q].  A column step then needs no
// workgroup-wide reduction: every wave reads the current column x_j (below
// the pivot) from an LDS broadcast buffer written by the wave that owns it,
// forms the dot products of x_j with its own columns and ||x_j||^2 in
// registers, reduces those CPW + 1 values over its own 64 lanes, computes the
// reflector scalars redundantly and updates only its own columns.  The owner
// of column j+1 then publishes its columns (updated) into the other half of
// the double buffer, and one barrier per column separates the steps.
//
// Reflector convention, storage and T are those of block_qr (qr_device.h):
// x = column j from row j down; beta = -sign(x0) ||x||, v = x / (x0 - beta)
// with v_j = 1, tau = (beta - x0) / beta (tau = 0 when the part below the
// pivot is exactly zero); below the diagonal column j keeps x, R[j][j] = beta_j
// and scale_j = 1 / (x0 - beta) are kept in LDS, U[m][j] = v_m^T v_j (m < j)
// feeds block_qr_build_t.
//
// prof(j) bounds the rows of column j that can be nonzero (below it the
// column is exactly zero, and the reflector leaves those rows untouched):
// the row count for a dense block, or (j+1)^K for Z_n with its rows in
// staircase order.  It must be non-decreasing in j.  Row chunks of 64 at or
// beyond prof(j) are skipped in step j (STAIR below).
#pragma once

#include "common.h"
#include "qr_device.h"

namespace cpqr {

template <int RMAX, int NW>
struct ColCfg {
  static constexpr int NT = 64 * NW;
  static constexpr int CPW = RMAX / NW;                          // columns per wave
  // values reduced per column step: CPW dot products and ||x||^2, padded to
  // a power of two
  static constexpr int NV = CPW + 1 <= 2 ? 2 : (CPW + 1 <= 4 ? 4 : (CPW + 1 <= 8 ? 8 : 16));
  static_assert(CPW >= 1 && CPW * NW == RMAX, "RMAX must be a multiple of the wave count");
};

// Column q (a compile-time index) of this wave's register block into the
// broadcast buffer, rows of the first `nch` chunks.
template <int Q, int RMAX, int RPL, int NW>
__device__ __forceinline__ void col_publish(const double (&a)[RPL][(ColCfg<RMAX, NW>::CPW)], int nch,
                                            double* __restrict__ xb) {
  const int lane = threadIdx.x & 63;
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    if (p < nch) xb[lane + 64 * p] = a[p][Q];
  });
}

// STAIR: prof(j) may be below the block's rows, and each column step runs
// a body compiled for the number of active chunks rounded up to a power of
// two (one branch per step); otherwise every chunk is active in every step.
// The loops over chunks need no guard beyond that: rows outside prof(j) hold
// zeros in x_j, so their coefficients are zero and their products exact
// zeros.  The column loop is unrolled by CPW, so that the wave that owns
// column j (wave j / CPW) and the local column of j are known when the body
// is compiled: the owner updates only its columns after j, waves with
// earlier columns only form the entries of U, and the next column is
// published from a fixed register.  On return tau, beta, scale and U are in
// LDS; T (block_qr_build_t) is left to the caller.
template <int RMAX, int RPL, int NW, bool STAIR, typename Prof>
__device__ __forceinline__ void col_qr(double (&a)[RPL][(ColCfg<RMAX, NW>::CPW)], int R, Prof&& prof,
                                       double (*xb)[64 * RPL], QrSmem<RMAX>& sm) {
  constexpr int CPW = ColCfg<RMAX, NW>::CPW, NV = ColCfg<RMAX, NW>::NV;
  constexpr int G = 64 / NV;   // lanes per reduced value
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto chunks = [&](int j) __attribute__((always_inline)) { return STAIR ? (prof(j) + 63) >> 6 : RPL; };
  // column 0 (wave 0, local column 0) into buffer 0
  if (wave == 0) col_publish<0, RMAX, RPL, NW>(a, chunks(0), xb[0]);
  __syncthreads();
  for (int jb = 0; jb * CPW < R; ++jb) {
    static_for<0, CPW>([&](auto jjc) __attribute__((always_inline)) {
      constexpr int jj = decltype(jjc)::value;
      const int j = jb * CPW + jj;
      if (j >= R) return;
      const int buf = j & 1;
      auto step = [&](auto nchc) __attribute__((always_inline)) {
        constexpr int NCH = decltype(nchc)::value;   // active chunks
        const double x0 = xb[buf][j];
        // x_j below the pivot (rows > j; the pivot row is in chunk 0, j < 64)
        double x[NCH];
        static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          const double v = xb[buf][lane + 64 * p];
          x[p] = (p > 0 || lane > j) ? v : 0.0;
        });
        // dot products with this wave's columns and ||x||^2 (value CPW)
        double d[NV];
        static_for<0, NV>([&](auto vc) __attribute__((always_inline)) { d[decltype(vc)::value] = 0.0; });
        static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            d[q] = fma(x[p], a[p][q], d[q]);
          });
          d[CPW] = fma(x[p], x[p], d[CPW]);
          if constexpr (NCH > 4) __builtin_amdgcn_sched_barrier(0);
        });
        wave_transpose_reduce<NV>(d);
        const double st = lane_read(d[0], G * CPW);
        double tau, beta, scale;
        qr_reflector_scalars(x0, st, &tau, &beta, &scale);
        // w_c = v^T a_c = a[j][c] + scale sum_{i>j} x_i a[i][c] (wave-uniform)
        auto wcol = [&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          return fma(scale, lane_read(d[0], G * q), lane_read(a[0][q], j));
        };
        // a -= tau v w^T for columns q in [Q0, CPW) (v = x scale below the
        // pivot, v_j = 1)
        auto update = [&](auto q0c) __attribute__((always_inline)) {
          constexpr int Q0 = decltype(q0c)::value;
          double w[CPW];
          static_for<Q0, CPW>([&](auto qc) __attribute__((always_inline)) { w[decltype(qc)::value] = wcol(qc); });
          const double ts = tau * scale;
          static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
            constexpr int p = decltype(pc)::value;
            const double coef = (p > 0 || lane > j) ? ts * x[p] : ((lane == j) ? tau : 0.0);
            static_for<Q0, CPW>([&](auto qc) __attribute__((always_inline)) {
              constexpr int q = decltype(qc)::value;
              a[p][q] = fma(-coef, w[q], a[p][q]);
            });
          });
        };
        // U[c][j] = v_c^T v_j = scale_c w_c for finished columns c < j; the
        // scale_c factor is applied after the loop
        auto ustore = [&](auto q1c) __attribute__((always_inline)) {
          constexpr int Q1 = decltype(q1c)::value;
          double w[CPW > 0 ? CPW : 1];
          static_for<0, Q1>([&](auto qc) __attribute__((always_inline)) { w[decltype(qc)::value] = wcol(qc); });
          if (lane == 0) {
            static_for<0, Q1>([&](auto qc) __attribute__((always_inline)) {
              constexpr int q = decltype(qc)::value;
              sm.U[CPW * wave + q][j] = w[q];
            });
          }
        };
        if (wave > jb) {
          update(std::integral_constant<int, 0>{});
        } else if (wave == jb) {
          update(std::integral_constant<int, jj + 1>{});
          ustore(std::integral_constant<int, jj>{});
        } else {
          ustore(std::integral_constant<int, CPW>{});
        }
        if (tid == 0) {
          sm.tau[j] = tau;
          sm.beta[j] = beta;
          sm.scale[j] = scale;
        }
      };
      if constexpr (!STAIR) {
        step(std::integral_constant<int, RPL>{});
      } else {
        const int nch = chunks(j);
        if (nch <= 1) step(std::integral_constant<int, 1>{});
        else if (nch <= 2 || RPL <= 2) step(std::integral_constant<int, (RPL < 2 ? RPL : 2)>{});
        else if (nch <= 4 || RPL <= 4) step(std::integral_constant<int, (RPL < 4 ? RPL : 4)>{});
        else if (nch <= 8 || RPL <= 8) step(std::integral_constant<int, (RPL < 8 ? RPL : 8)>{});
        else step(std::integral_constant<int, RPL>{});
      }
      // the owner of column j + 1 publishes it (updated) for the next step
      const int jn = j + 1;
      if (jn < R) {
        if constexpr (jj + 1 < CPW) {
          if (wave == jb) col_publish<jj + 1, RMAX, RPL, NW>(a, chunks(jn), xb[buf ^ 1]);
        } else {
          if (wave == jb + 1) col_publish<0, RMAX, RPL, NW>(a, chunks(jn), xb[buf ^ 1]);
        }
      }
      __syncthreads();
    });
  }
  // U entries were stored without the scale of their earlier column
  for (int e = tid; e < RMAX * RMAX; e += ColCfg<RMAX, NW>::NT) {
    const int m = e / RMAX, jc = e % RMAX;
    if (m < jc && jc < R) sm.U[m][jc] *= sm.scale[m];
  }
  __syncthreads();
}


// col_qr for a dense block, two columns per step.  Columns j and j + 1 (j
// even) belong to the same wave (CPW is even).  Before the step's barrier
// that wave alone forms reflector j from its column j, applies it to column
// j + 1, forms reflector j + 1 (two reductions over its own lanes) and
// publishes both columns with their scalars and v_j^T v_{j+1}.  After the
// barrier every wave applies H_{j+1} H_j to its later columns in the compact
// WY form: with s1 = v_j^T a and s2 = v_{j+1}^T a (one reduction of 2 CPW
// values), a -= v_j (tau_j s1) + v_{j+1} tau_{j+1} (s2 - (v_j^T v_{j+1}) tau_j s1);
// waves with finished columns form their entries of U from the same dot
// products.  Half as many barriers, broadcasts and reductions as col_qr;
// the reflector convention, storage, tau, beta, scale and U on return are
// those of col_qr (the reflectors are the same up to rounding).  xp holds
// two double-buffered pairs of published columns.
template <int RMAX, int RPL, int NW>
__device__ __forceinline__ void col_qr_pair(double (&a)[RPL][(ColCfg<RMAX, NW>::CPW)], int R,
                                            double (*xp)[2][64 * RPL], QrSmem<RMAX>& sm) {
  constexpr int CPW = ColCfg<RMAX, NW>::CPW;
  static_assert(CPW % 2 == 0, "pairs of columns must lie in one wave");
  constexpr int NP = CPW / 2;
  constexpr int NV2 = 2 * CPW <= 2 ? 2 : (2 * CPW <= 4 ? 4 : (2 * CPW <= 8 ? 8 : 16));
  constexpr int G2 = 64 / NV2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the owner's work for pair (j, j + 1): local columns QA = 2 PP, QB = QA + 1
  auto prework = [&](auto ppc, int j, int buf) __attribute__((always_inline)) {
    constexpr int QA = 2 * decltype(ppc)::value, QB = QA + 1;
    const int j1 = j + 1;
    double d[2] = {0.0, 0.0};
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      const double xv = (p > 0 || lane > j) ? a[p][QA] : 0.0;
      d[0] = fma(xv, xv, d[0]);
      d[1] = fma(xv, a[p][QB], d[1]);
    });
    wave_transpose_reduce<2>(d);
    double tau1, beta1, scale1;
    qr_reflector_scalars(lane_read(a[0][QA], j), lane_read(d[0], 0), &tau1, &beta1, &scale1);
    // column j + 1 <- H_j column j + 1
    const double w1y = fma(scale1, lane_read(d[0], 32), lane_read(a[0][QB], j));
    const double ts1 = tau1 * scale1;
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      const double coef = (p > 0 || lane > j) ? ts1 * a[p][QA] : ((lane == j) ? tau1 : 0.0);
      a[p][QB] = fma(-coef, w1y, a[p][QB]);
    });
    double tau2 = 0.0, beta2 = 0.0, scale2 = 0.0, w12 = 0.0;
    if (j1 < R) {
      double e[2] = {0.0, 0.0};
      static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const bool below = p > 0 || lane > j1;
        const double yv = below ? a[p][QB] : 0.0;
        e[0] = fma(yv, yv, e[0]);
        e[1] = fma(below ? a[p][QA] : 0.0, yv, e[1]);
      });
      wave_transpose_reduce<2>(e);
      qr_reflector_scalars(lane_read(a[0][QB], j1), lane_read(e[0], 0), &tau2, &beta2, &scale2);
      // v_j^T v_{j+1} without the scale of column j (applied with the other U entries)
      w12 = fma(scale2, lane_read(e[0], 32), lane_read(a[0][QA], j1));
    }
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      xp[buf][0][lane + 64 * p] = a[p][QA];
      xp[buf][1][lane + 64 * p] = a[p][QB];
    });
    if (lane == 0) {
      sm.tau[j] = tau1;
      sm.beta[j] = beta1;
      sm.scale[j] = scale1;
      if (j1 < R) {
        sm.tau[j1] = tau2;
        sm.beta[j1] = beta2;
        sm.scale[j1] = scale2;
        sm.U[j][j1] = w12;
      }
    }
  };
  if (wave == 0) prework(std::integral_constant<int, 0>{}, 0, 0);
  __syncthreads();
  for (int jb = 0; jb * CPW < R; ++jb) {
    static_for<0, NP>([&](auto ppc) __attribute__((always_inline)) {
      constexpr int PP = decltype(ppc)::value;
      const int j = jb * CPW + 2 * PP;
      if (j >= R) return;
      const int j1 = j + 1;
      const int buf = (j >> 1) & 1;
      const bool two = j1 < R;
      double x[RPL], y[RPL];
      static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const double xv = xp[buf][0][lane + 64 * p], yv = xp[buf][1][lane + 64 * p];
        x[p] = (p > 0 || lane > j) ? xv : 0.0;
        y[p] = (p > 0 || lane > j1) ? yv : 0.0;
      });
      const double tau1 = sm.tau[j], scale1 = sm.scale[j];
      const double tau2 = two ? sm.tau[j1] : 0.0, scale2 = two ? sm.scale[j1] : 0.0;
      const double u12 = two ? scale1 * sm.U[j][j1] : 0.0;
      // d[2q] = x^T a_q (rows > j), d[2q + 1] = y^T a_q (rows > j + 1)
      double d[NV2];
      static_for<0, NV2>([&](auto vc) __attribute__((always_inline)) { d[decltype(vc)::value] = 0.0; });
      static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          d[2 * q] = fma(x[p], a[p][q], d[2 * q]);
          d[2 * q + 1] = fma(y[p], a[p][q], d[2 * q + 1]);
        });
      });
      wave_transpose_reduce<NV2>(d);
      auto s1 = [&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        return fma(scale1, lane_read(d[0], G2 * (2 * q)), lane_read(a[0][q], j));
      };
      auto s2 = [&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        return fma(scale2, lane_read(d[0], G2 * (2 * q + 1)), lane_read(a[0][q], j1));
      };
      // a -= v_j c1 + v_{j+1} c2 for local columns [Q0, CPW)
      auto update = [&](auto q0c) __attribute__((always_inline)) {
        constexpr int Q0 = decltype(q0c)::value;
        double c1[CPW], c2[CPW];
        static_for<Q0, CPW>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          c1[q] = tau1 * s1(qc);
          c2[q] = tau2 * fma(-u12, c1[q], s2(qc));
        });
        static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          const double v1 = (p == 0 && lane == j) ? 1.0 : scale1 * x[p];
          const double v2 = (p == 0 && lane == j1) ? 1.0 : scale2 * y[p];
          static_for<Q0, CPW>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            a[p][q] = fma(-v2, c2[q], fma(-v1, c1[q], a[p][q]));
          });
        });
      };
      // U[c][j] and U[c][j + 1] of finished local columns [0, Q1) (without
      // their scale_c, applied after the loop)
      auto ustore = [&](auto q1c) __attribute__((always_inline)) {
        constexpr int Q1 = decltype(q1c)::value;
        double w1[CPW], w2[CPW];
        static_for<0, Q1>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          w1[q] = s1(qc);
          w2[q] = s2(qc);
        });
        if (lane == 0) {
          static_for<0, Q1>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            sm.U[CPW * wave + q][j] = w1[q];
            if (two) sm.U[CPW * wave + q][j1] = w2[q];
          });
        }
      };
      if (wave > jb) {
        update(std::integral_constant<int, 0>{});
      } else if (wave == jb) {
        update(std::integral_constant<int, 2 * PP + 2>{});
        ustore(std::integral_constant<int, 2 * PP>{});
      } else {
        ustore(std::integral_constant<int, CPW>{});
      }
      // the owner of the next pair forms and publishes it
      const int jn = j + 2;
      if (jn < R) {
        if constexpr (PP + 1 < NP) {
          if (wave == jb) prework(std::integral_constant<int, PP + 1>{}, jn, buf ^ 1);
        } else {
          if (wave == jb + 1) prework(std::integral_constant<int, 0>{}, jn, buf ^ 1);
        }
      }
      __syncthreads();
    });
  }
  for (int e = tid; e < RMAX * RMAX; e += ColCfg<RMAX, NW>::NT) {
    const int m = e / RMAX, jc = e % RMAX;
    if (m < jc && jc < R) sm.U[m][jc] *= sm.scale[m];
  }
  __syncthreads();
}

// T of the compact WY form from U and tau (block_qr_build_t) by the lanes of
// wave 0 alone, without a workgroup barrier: the caller synchronises before
// T is read.  Lane k forms row k, T[k][j] = -tau_j sum_{k <= m < j} T[k][m]
// U[m][j] (T[k][k] = tau_k): once T[k][m] is known its terms go into the
// sums of every later column, one row of U at a time, so that the row of T
// and the running sums share one register array (the caller's registers
// stay live).  Each sum adds its terms in ascending m, as block_qr_build_t.
template <int RMAX>
__device__ __forceinline__ void block_qr_build_t_wave0(int R, QrSmem<RMAX>& sm) {
  const int k = threadIdx.x;
  if (k < RMAX) {
    double acc[RMAX];   // the sum of column j until T[k][j] is known, then T[k][j]
#pragma unroll
    for (int j = 0; j < RMAX; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      const double tj = (j < k || j >= R) ? 0.0 : ((j == k) ? sm.tau[j] : -sm.tau[j] * acc[j]);
      acc[j] = tj;
#pragma unroll
      for (int jj = j + 1; jj < RMAX; ++jj) acc[jj] = fma(tj, sm.U[j][jj], acc[jj]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < RMAX; ++j) sm.T[k][j] = acc[j];
  }
}

// ---------------------------------------------------------------------------
// The same factorisation for Z_n with its rows in staircase order, where
// column c is nonzero only on its profile, the first (c+1)^K rows.  Columns
// go to the waves round-robin (column c = NW q + w is local column q of wave
// w), so that local column q of every wave stays below (NW (q+1))^K rows and
// needs only L(q) of the RPL row chunks in registers: at rank 32 and K = 2
// that is 1 + 4 + 9 + 16 = 30 chunks for 4 local columns instead of 64.  The
// owner of column j is wave j mod NW, and it publishes all of its columns
// (their live chunks) into the broadcast buffer, packed: local column q at
// row offset 64 OFF(q); the readers take column j at local column j / NW.
// The column loop is not unrolled (the owner and local column of a step are
// runtime values), which keeps the kernel within the instruction cache: each
// step runs one of the bodies compiled per chunk count.
// PAIRS: the columns go to the waves two at a time (columns 2 (NW r + w) and
// 2 (NW r + w) + 1 are local columns 2 r and 2 r + 1 of wave w), for
// col_qr_stair_pair, which factors two columns per step.
template <int RMAX, int RPL, int NW, int K, bool PAIRS = false>
struct StairCfg {
  static constexpr int CPW = RMAX / NW;
  static constexpr int MR = 64 * RPL;
  static constexpr int L(int q) {
    long long c = PAIRS ? 2LL * NW * (q / 2 + 1) : (long long)NW * (q + 1), pw = 1;
    for (int k = 0; k < K; ++k) pw *= c;
    const long long ch = (pw + 63) / 64;
    return ch < RPL ? (int)ch : RPL;
  }
  // column index of local column q of wave w
  static __device__ __forceinline__ int col(int q, int w) {
    return PAIRS ? 2 * (NW * (q / 2) + w) + (q & 1) : NW * q + w;
  }
  static constexpr int OFF(int q) {
    int o = 0;
    for (int i = 0; i < q; ++i) o += L(i);
    return o;
  }
  static constexpr int TOT = OFF(CPW);
};

template <int RMAX, int RPL, int NW, int K, typename Prof>
__device__ __forceinline__ void col_qr_stair(double (&a)[(StairCfg<RMAX, RPL, NW, K>::TOT)], int R, Prof&& prof,
                                             double (*xb)[(StairCfg<RMAX, RPL, NW, K>::TOT) * 64],
                                             QrSmem<RMAX>& sm) {
  using SC = StairCfg<RMAX, RPL, NW, K>;
  constexpr int CPW = SC::CPW, MR = SC::MR;
  constexpr int NV = ColCfg<RMAX, NW>::NV, G = 64 / NV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto chunks = [&](int j) __attribute__((always_inline)) { return (prof(j) + 63) >> 6; };
  // every column of this wave into the buffer (live chunks only)
  auto publish = [&](double* __restrict__ dst) __attribute__((always_inline)) {
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      static_for<0, SC::L(q)>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        dst[64 * (SC::OFF(q) + p) + lane] = a[SC::OFF(q) + p];
      });
    });
  };
  if (wave == 0) publish(xb[0]);
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    {
      const int jb = j / NW, jj = j % NW;   // local column and owner wave of column j
      const int buf = j & 1;
      int off = 0;   // 64 OFF(jb): chunks of the local columns before jb
      static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        off += (q < jb) ? SC::L(q) : 0;
      });
      const double* __restrict__ xj = xb[buf] + 64 * off;
      const int nch = chunks(j);
      auto step = [&](auto nchc) __attribute__((always_inline)) {
        constexpr int NCH = decltype(nchc)::value;   // active chunks, rounded up
        const double x0 = xj[j];
        // chunks at or beyond nch of the buffer may hold an earlier column
        // (the bucket rounds nch up), so they read as zero
        double x[NCH];
        static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          const double v = xj[lane + 64 * p];
          x[p] = (p < nch && (p > 0 || lane > j)) ? v : 0.0;
        });
        double d[NV];
        static_for<0, NV>([&](auto vc) __attribute__((always_inline)) { d[decltype(vc)::value] = 0.0; });
        static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            if constexpr (p < SC::L(q)) d[q] = fma(x[p], a[SC::OFF(q) + p], d[q]);
          });
          d[CPW] = fma(x[p], x[p], d[CPW]);
        });
        wave_transpose_reduce<NV>(d);
        const double st = lane_read(d[0], G * CPW);
        double tau, beta, scale;
        qr_reflector_scalars(x0, st, &tau, &beta, &scale);
        const double ts = tau * scale;
        double coef[NCH];
        static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          coef[p] = (p > 0 || lane > j) ? ts * x[p] : ((lane == j) ? tau : 0.0);
        });
        static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          // w_c = v^T a_c for c = NW q + wave (wave-uniform)
          const double w = fma(scale, lane_read(d[0], G * q), lane_read(a[SC::OFF(q)], j));
          const bool after = (q > jb) || (q == jb && wave > jj);
          const bool before = (q < jb) || (q == jb && wave < jj);
          const double wu = after ? w : 0.0;
          static_for<0, (NCH < SC::L(q) ? NCH : SC::L(q))>([&](auto pc) __attribute__((always_inline)) {
            constexpr int p = decltype(pc)::value;
            a[SC::OFF(q) + p] = fma(-coef[p], wu, a[SC::OFF(q) + p]);
          });
          // U[c][j] = v_c^T v_j without the scale_c factor (applied below)
          if (lane == 0 && before) sm.U[NW * q + wave][j] = w;
        });
        if (tid == 0) {
          sm.tau[j] = tau;
          sm.beta[j] = beta;
          sm.scale[j] = scale;
        }
      };
      if (nch <= 1) step(std::integral_constant<int, 1>{});
      else if (nch <= 2 || RPL <= 2) step(std::integral_constant<int, (RPL < 2 ? RPL : 2)>{});
      else if (nch <= 4 || RPL <= 4) step(std::integral_constant<int, (RPL < 4 ? RPL : 4)>{});
      else if (nch <= 8 || RPL <= 8) step(std::integral_constant<int, (RPL < 8 ? RPL : 8)>{});
      else step(std::integral_constant<int, RPL>{});
      // the owner of column j + 1 publishes its columns for the next step
      if (j + 1 < R && wave == (jj + 1) % NW) publish(xb[buf ^ 1]);
      __syncthreads();
    }
  }
  for (int e = tid; e < RMAX * RMAX; e += 64 * NW) {
    const int m = e / RMAX, jc = e % RMAX;
    if (m < jc && jc < R) sm.U[m][jc] *= sm.scale[m];
  }
  __syncthreads();
}

// col_qr_stair with two columns per step (the scheme of col_qr_pair) and
// the paired column layout (StairCfg<..., true>): pair (j, j + 1), j even,
// is local pair j / (2 NW) of wave (j / 2) mod NW.  The owner forms both
// reflectors on the rows of column j + 1's profile and publishes the two
// columns; the other waves' steps run the body compiled for that chunk
// count.  Same outputs as col_qr_stair.
template <int RMAX, int RPL, int NW, int K, typename Prof>
__device__ __forceinline__ void col_qr_stair_pair(double (&a)[(StairCfg<RMAX, RPL, NW, K, true>::TOT)], int R,
                                                  Prof&& prof, double (*xp)[2][64 * RPL], QrSmem<RMAX>& sm) {
  using SC = StairCfg<RMAX, RPL, NW, K, true>;
  constexpr int CPW = SC::CPW;
  static_assert(CPW % 2 == 0, "pairs of columns must lie in one wave");
  constexpr int NP = CPW / 2;
  constexpr int NV2 = 2 * CPW <= 2 ? 2 : (2 * CPW <= 4 ? 4 : (2 * CPW <= 8 ? 8 : 16));
  constexpr int G2 = 64 / NV2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto chunks = [&](int j) __attribute__((always_inline)) { return (prof(j) + 63) >> 6; };
  // dispatch on the active chunk count of a step, rounded up to a power of two
  auto by_chunks = [&](int nch, auto&& body) __attribute__((always_inline)) {
    if (nch <= 1) body(std::integral_constant<int, 1>{});
    else if (nch <= 2 || RPL <= 2) body(std::integral_constant<int, (RPL < 2 ? RPL : 2)>{});
    else if (nch <= 4 || RPL <= 4) body(std::integral_constant<int, (RPL < 4 ? RPL : 4)>{});
    else if (nch <= 8 || RPL <= 8) body(std::integral_constant<int, (RPL < 8 ? RPL : 8)>{});
    else body(std::integral_constant<int, RPL>{});
  };
  // the owner's work for pair (j, j + 1) held in local pair LP
  auto prework = [&](auto lpc, int j, int buf) __attribute__((always_inline)) {
    constexpr int QA = 2 * decltype(lpc)::value, QB = QA + 1;
    constexpr int LA = SC::L(QA);   // chunks held for both columns of the pair
    const int j1 = j + 1;
    by_chunks(chunks(j1), [&](auto nchc) __attribute__((always_inline)) {
      constexpr int NC = decltype(nchc)::value < LA ? decltype(nchc)::value : LA;
      double d[2] = {0.0, 0.0};
      static_for<0, NC>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const double xv = (p > 0 || lane > j) ? a[SC::OFF(QA) + p] : 0.0;
        d[0] = fma(xv, xv, d[0]);
        d[1] = fma(xv, a[SC::OFF(QB) + p], d[1]);
      });
      wave_transpose_reduce<2>(d);
      double tau1, beta1, scale1;
      qr_reflector_scalars(lane_read(a[SC::OFF(QA)], j), lane_read(d[0], 0), &tau1, &beta1, &scale1);
      const double w1y = fma(scale1, lane_read(d[0], 32), lane_read(a[SC::OFF(QB)], j));
      const double ts1 = tau1 * scale1;
      static_for<0, NC>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const double coef = (p > 0 || lane > j) ? ts1 * a[SC::OFF(QA) + p] : ((lane == j) ? tau1 : 0.0);
        a[SC::OFF(QB) + p] = fma(-coef, w1y, a[SC::OFF(QB) + p]);
      });
      double tau2 = 0.0, beta2 = 0.0, scale2 = 0.0, w12 = 0.0;
      if (j1 < R) {
        double e[2] = {0.0, 0.0};
        static_for<0, NC>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          const bool below = p > 0 || lane > j1;
          const double yv = below ? a[SC::OFF(QB) + p] : 0.0;
          e[0] = fma(yv, yv, e[0]);
          e[1] = fma(below ? a[SC::OFF(QA) + p] : 0.0, yv, e[1]);
        });
        wave_transpose_reduce<2>(e);
        qr_reflector_scalars(lane_read(a[SC::OFF(QB)], j1), lane_read(e[0], 0), &tau2, &beta2, &scale2);
        w12 = fma(scale2, lane_read(e[0], 32), lane_read(a[SC::OFF(QA)], j1));
      }
      static_for<0, NC>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        xp[buf][0][lane + 64 * p] = a[SC::OFF(QA) + p];
        xp[buf][1][lane + 64 * p] = a[SC::OFF(QB) + p];
      });
      if (lane == 0) {
        sm.tau[j] = tau1;
        sm.beta[j] = beta1;
        sm.scale[j] = scale1;
        if (j1 < R) {
          sm.tau[j1] = tau2;
          sm.beta[j1] = beta2;
          sm.scale[j1] = scale2;
          sm.U[j][j1] = w12;
        }
      }
    });
  };
  auto prework_at = [&](int j, int buf) __attribute__((always_inline)) {
    const int lp = (j >> 1) / NW;
    static_for<0, NP>([&](auto lpc) __attribute__((always_inline)) {
      if (lp == decltype(lpc)::value) prework(lpc, j, buf);
    });
  };
  if (wave == 0) prework_at(0, 0);
  __syncthreads();
  for (int j = 0; j < R; j += 2) {
    const int j1 = j + 1;
    const int buf = (j >> 1) & 1;
    const bool two = j1 < R;
    by_chunks(chunks(two ? j1 : j), [&](auto nchc) __attribute__((always_inline)) {
      constexpr int NCH = decltype(nchc)::value;
      const int nch = chunks(two ? j1 : j);
      // chunks at or beyond nch of the buffer may hold an earlier pair (the
      // bucket rounds nch up), so they read as zero
      double x[NCH], y[NCH];
      static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const double xv = xp[buf][0][lane + 64 * p], yv = xp[buf][1][lane + 64 * p];
        x[p] = (p < nch && (p > 0 || lane > j)) ? xv : 0.0;
        y[p] = (p < nch && (p > 0 || lane > j1)) ? yv : 0.0;
      });
      const double tau1 = sm.tau[j], scale1 = sm.scale[j];
      const double tau2 = two ? sm.tau[j1] : 0.0, scale2 = two ? sm.scale[j1] : 0.0;
      const double u12 = two ? scale1 * sm.U[j][j1] : 0.0;
      double d[NV2];
      static_for<0, NV2>([&](auto vc) __attribute__((always_inline)) { d[decltype(vc)::value] = 0.0; });
      static_for<0, NCH>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          if constexpr (p < SC::L(q)) {
            d[2 * q] = fma(x[p], a[SC::OFF(q) + p], d[2 * q]);
            d[2 * q + 1] = fma(y[p], a[SC::OFF(q) + p], d[2 * q + 1]);
          }
        });
      });
      wave_transpose_reduce<NV2>(d);
      static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        const int c = SC::col(q, wave);
        const double s1 = fma(scale1, lane_read(d[0], G2 * (2 * q)), lane_read(a[SC::OFF(q)], j));
        const double s2 = fma(scale2, lane_read(d[0], G2 * (2 * q + 1)), lane_read(a[SC::OFF(q)], j1));
        const bool after = c > j1, before = c < j;
        const double c1 = after ? tau1 * s1 : 0.0;
        const double c2 = after ? tau2 * fma(-u12, c1, s2) : 0.0;
        static_for<0, (NCH < SC::L(q) ? NCH : SC::L(q))>([&](auto pc) __attribute__((always_inline)) {
          constexpr int p = decltype(pc)::value;
          const double v1 = (p == 0 && lane == j) ? 1.0 : scale1 * x[p];
          const double v2 = (p == 0 && lane == j1) ? 1.0 : scale2 * y[p];
          a[SC::OFF(q) + p] = fma(-v2, c2, fma(-v1, c1, a[SC::OFF(q) + p]));
        });
        // U[c][j], U[c][j + 1] without the scale_c factor (applied below)
        if (lane == 0 && before) {
          sm.U[c][j] = s1;
          if (two) sm.U[c][j1] = s2;
        }
      });
    });
    // the owner of the next pair forms and publishes it
    const int jn = j + 2;
    if (jn < R && wave == (jn >> 1) % NW) prework_at(jn, buf ^ 1);
    __syncthreads();
  }
  for (int e = tid; e < RMAX * RMAX; e += 64 * NW) {
    const int m = e / RMAX, jc = e % RMAX;
    if (m < jc && jc < R) sm.U[m][jc] *= sm.scale[m];
  }
  __syncthreads();
}

}  // namespace cpqr
