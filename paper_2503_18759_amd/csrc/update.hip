// Mode-update kernels of QR-based ALS (Algorithm 2: the product with Q0, the
// triangular solve and the factor QR; Algorithm 3: the same update with the
// extrapolated Q0) and the norm kernels of the fit (Section 4.1).
//
//  * apply_partial / apply_reduce:  [Vp | Vq] = Y_(n) [Q0 | Q0prev] in float64
//    (Y_(n) columns in the Kolda order of the remaining modes, i.e. column
//    l + L s of the leaf stored as [L, I_n, S]).  The K = R^(N-1) reduction is
//    split over workgroups and the partial products are summed in a second
//    pass in a fixed order.
//  * finish_update: one workgroup per mode update.  Vu = (1+beta) Vp - alpha beta Vq
//    (eq. 19 applied through V = Y_(n) Qhat0), <Vp,Vu> and ||Vu||^2 for the
//    fit, back substitution of Ahat R0^T = Vu, lambda = column norms,
//    A = Ahat / lambda, Householder QR of A -> Q_n, R_n; after the last update
//    of a sweep the fit and the extrapolation activation rule.
//    finish_col does the same for factors of at most 256 rows with the
//    factor QR in the column-distributed layout (colqr_device.h), and leaves
//    the explicit Q_n to form_qn.
//  * finish_tall / tall_factor_tail: the same update for modes beyond the
//    single-workgroup factor QR (the factor QR then goes through the TSQR).
//  * sumsq / residual: ||X||^2 and ||X - K||^2 with float64 accumulation.
#include "common.h"
#include "kernels.h"
#include "qr_device.h"
#include "colqr_device.h"

namespace cpqr {

static constexpr int AP_THREADS = 256;
static constexpr int AP_ROWS = 64;
static constexpr int AP_KT = 32;

// Largest digit of the Kolda column index k of Y_(n) (base R, K digits).
// Column c of Q0 is zero at every row whose largest digit exceeds c (the
// staircase of Z_n; Section 3.2), so a tile's leading columns below the
// smallest such digit are zero and need not be read.
__device__ __forceinline__ int kolda_max_digit(int k, int R, int K) {
  int m = 0;
  for (int t = 0; t < K; ++t) {
    const int d = k % R;
    m = d > m ? d : m;
    k /= R;
  }
  return m;
}

template <typename TY, int RMAX>
__global__ __launch_bounds__(AP_THREADS) __attribute__((amdgpu_waves_per_eu(1, 2))) void apply_partial(ApplyDev a0, const ApplyDev* __restrict__ batch) {
  const ApplyDev a = kernel_args(a0, batch, blockIdx.z);
  typedef __attribute__((address_space(1))) TY gTY;
  const gTY* __restrict__ Y = static_cast<const gTY*>((const gTY*)a.Y);
  const int64_t L = a.L, S = a.S, chunk = a.chunk;
  const int I = a.I, R = a.R;
  const gdouble* __restrict__ Q0 = (const gdouble*)a.Q0;
  const gdouble* __restrict__ Q0prev = (const gdouble*)a.Q0prev;
  gdouble* __restrict__ partial = (gdouble*)a.partial;
  if ((int)blockIdx.x * AP_ROWS >= I || (int)blockIdx.y >= a.nchunks) return;
  // k loop: Y tile (rows padded by two so that each thread's pair of rows is
  // one 16-byte read) and the Q0 / Q0prev tiles; epilogue (compact Q0): the
  // chunk's products and the two Md
  __shared__ union __attribute__((aligned(16))) ApLds {
    struct {
      double y[AP_KT][AP_ROWS + 2];
      double q[AP_KT][RMAX];
      double p[AP_KT][RMAX];
    } loop;
    struct {
      double pp[AP_ROWS][RMAX + 2];
      double pq[AP_ROWS][RMAX + 2];
      double mp[RMAX][RMAX];
      double mq[RMAX][RMAX];
    } epi;
  } lds;
  auto& sY = lds.loop.y;
  auto& sQ = lds.loop.q;
  auto& sP = lds.loop.p;
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * AP_ROWS;
  const int64_t M = L * S;
  const int64_t k0 = (int64_t)blockIdx.y * chunk;
  int64_t k1 = k0 + chunk;
  if (k1 > M) k1 = M;
  // digits of the Kolda index: M = R^K
  int K = 0;
  for (int64_t m = M; m > 1; m /= R) ++K;
  // Q0prev is read whenever it is given; its product is used by the finish
  // kernel only while the extrapolation is active (a select, so whatever the
  // product holds before then is never mixed in)
  const bool use_prev = (Q0prev != nullptr);
  // Register tile: rows 2 ti and 2 ti + 1, columns cg CW .. cg CW + CW - 1
  // of both Q0 and Q0prev.  A wave holds two column groups, i.e. the
  // contiguous columns [2 w CW, 2 (w + 1) CW).
  constexpr int CW = RMAX / 8;
  const int ti = tid & 31, cg = tid >> 5, w = tid >> 6, lane = tid & 63;
  constexpr int NY = AP_ROWS * AP_KT / AP_THREADS;   // Y elements per thread and tile
  constexpr int NQ = AP_KT * RMAX / AP_THREADS;      // Q0 (and Q0prev) elements per thread and tile
  double ap[2][CW], aq[2][CW];
#pragma unroll
  for (int m = 0; m < CW; ++m) ap[0][m] = ap[1][m] = aq[0][m] = aq[1][m] = 0.0;
  const int64_t LI = L * (int64_t)I;
  // The tiles of the chunk are software-pipelined: the global loads of the
  // next tile are issued into registers before the current tile is used.
  double ry[NY], rq[NQ], rp[NQ];
  int cnext = 0;   // staircase bound of the tile held in ry/rq/rp
  auto load_tile = [&](int64_t kt) __attribute__((always_inline)) {
    // smallest largest-digit over the tile's columns (wave-wide minimum)
    const int64_t kl = kt + (lane & (AP_KT - 1));
    int md = (kl < k1) ? kolda_max_digit((int)kl, R, K) : RMAX;
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) {
      const int o = __shfl_xor(md, m, 64);
      md = o < md ? o : md;
    }
    const int cmin = __builtin_amdgcn_readfirstlane(md);
    cnext = cmin;
#pragma unroll
    for (int t = 0; t < NY; ++t) {
      const int e = tid + AP_THREADS * t;
      int ii, kk;
      if (L == 1) { ii = e & 63; kk = e >> 6; }
      else        { kk = e % AP_KT; ii = e / AP_KT; }
      const int64_t k = kt + kk;
      const bool in = (i0 + ii < I && k < k1);
      // k < M = L S < 2^31 (the Kolda column index): 32-bit division
      const int s = (int)k / (int)L, l = (int)k - s * (int)L;
      const TY v = Y[in ? l + L * (int64_t)(i0 + ii) + LI * s : 0];
      ry[t] = in ? (double)v : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int e = tid + AP_THREADS * t;
      const int kk = e % AP_KT, c = e / AP_KT;
      const int64_t k = kt + kk;
      const bool in = (k < k1) && (c < R) && (c >= cmin);
      const int64_t idx = in ? k + M * c : 0;
      const double q = Q0[idx];
      const double pq = use_prev ? Q0prev[idx] : 0.0;
      rq[t] = in ? q : 0.0;
      rp[t] = (in && use_prev) ? pq : 0.0;
    }
  };
  if (k0 < k1) load_tile(k0);
  for (int64_t kt = k0; kt < k1; kt += AP_KT) {
#pragma unroll
    for (int t = 0; t < NY; ++t) {
      const int e = tid + AP_THREADS * t;
      int ii, kk;
      if (L == 1) { ii = e & 63; kk = e >> 6; }
      else        { kk = e % AP_KT; ii = e / AP_KT; }
      sY[kk][ii] = ry[t];
    }
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int e = tid + AP_THREADS * t;
      const int kk = e % AP_KT, c = e / AP_KT;
      sQ[kk][c] = rq[t];
      sP[kk][c] = rp[t];
    }
    const int ccur = cnext;
    __syncthreads();
    if (kt + AP_KT < k1) load_tile(kt + AP_KT);
    // every column of this wave below the tile's staircase bound: its
    // products are exact zeros and are skipped (wave-uniform branch)
    if (2 * (w + 1) * CW > ccur) {
#pragma unroll 4
      for (int kk = 0; kk < AP_KT; ++kk) {
        const double y0 = sY[kk][2 * ti], y1 = sY[kk][2 * ti + 1];
        double q[CW], p[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) {
          q[m] = sQ[kk][cg * CW + m];
          p[m] = sP[kk][cg * CW + m];
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
          ap[0][m] = fma(y0, q[m], ap[0][m]);
          ap[1][m] = fma(y1, q[m], ap[1][m]);
          aq[0][m] = fma(y0, p[m], aq[0][m]);
          aq[1][m] = fma(y1, p[m], aq[1][m]);
        }
      }
    }
    __syncthreads();
  }
  if (a.meta_p != nullptr) {
    // compact Q0 = (E - V T V1^T) D: this chunk's share of Y_(n) Q0 is
    // -(Y_(n) V)_chunk Md (the E D term is added once, in apply_reduce)
    const gdouble* __restrict__ mp = (const gdouble*)a.meta_p;
    const gdouble* __restrict__ mq = (const gdouble*)a.meta_q;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int m = 0; m < CW; ++m) {
        lds.epi.pp[2 * ti + r][cg * CW + m] = ap[r][m];
        lds.epi.pq[2 * ti + r][cg * CW + m] = aq[r][m];
      }
    for (int e = tid; e < RMAX * RMAX; e += AP_THREADS) {
      const int i = e % RMAX, c = e / RMAX;
      const bool in = i < R && c < R;
      const double x = mp[in ? i + R * c : 0];
      const double y = (mq != nullptr) ? mq[in ? i + R * c : 0] : 0.0;
      lds.epi.mp[i][c] = in ? x : 0.0;
      lds.epi.mq[i][c] = in ? y : 0.0;
    }
    __syncthreads();
    double bp[2][CW], bq[2][CW];
#pragma unroll
    for (int m = 0; m < CW; ++m) bp[0][m] = bp[1][m] = bq[0][m] = bq[1][m] = 0.0;
#pragma unroll 4
    for (int k = 0; k < RMAX; ++k) {
      const double p0 = lds.epi.pp[2 * ti][k], p1 = lds.epi.pp[2 * ti + 1][k];
      const double q0 = lds.epi.pq[2 * ti][k], q1 = lds.epi.pq[2 * ti + 1][k];
#pragma unroll
      for (int m = 0; m < CW; ++m) {
        const double x = lds.epi.mp[k][cg * CW + m], y = lds.epi.mq[k][cg * CW + m];
        bp[0][m] = fma(p0, x, bp[0][m]);
        bp[1][m] = fma(p1, x, bp[1][m]);
        bq[0][m] = fma(q0, y, bq[0][m]);
        bq[1][m] = fma(q1, y, bq[1][m]);
      }
    }
#pragma unroll
    for (int m = 0; m < CW; ++m) {
      ap[0][m] = -bp[0][m];
      ap[1][m] = -bp[1][m];
      aq[0][m] = -bq[0][m];
      aq[1][m] = -bq[1][m];
    }
  }
  gdouble* out = partial + (int64_t)blockIdx.y * 2 * I * R;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int row = i0 + 2 * ti + r;
    if (row >= I) continue;
#pragma unroll
    for (int m = 0; m < CW; ++m) {
      const int c = cg * CW + m;
      if (c < R) {
        out[row + (int64_t)I * c] = ap[r][m];
        out[(int64_t)I * R + row + (int64_t)I * c] = aq[r][m];
      }
    }
  }
}

// Waves per reduction workgroup: each wave sums a fixed, strided subset of
// the chunks for 64 consecutive outputs and the subsets are then added in
// wave order, so the result does not depend on scheduling.
static constexpr int AR_WAVES = 16;

__global__ __launch_bounds__(64 * AR_WAVES) void apply_reduce(ApplyDev a0, const ApplyDev* __restrict__ batch) {
  const ApplyDev a = kernel_args(a0, batch, blockIdx.y);
  const gdouble* __restrict__ partial = (const gdouble*)a.partial;
  const int nchunks = a.nchunks;
  const int64_t n = 2 * (int64_t)a.I * a.R;
  gdouble* __restrict__ V = (gdouble*)a.V;
  __shared__ double sp[AR_WAVES][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t ob = (int64_t)blockIdx.x * 64; ob < n; ob += (int64_t)gridDim.x * 64) {
    const int64_t o = ob + lane;
    double s = 0.0;
    if (o < n) {
      // chunks w, w + AR_WAVES, ... in increasing order, four loads in flight
      int c = w;
      for (; c + 3 * AR_WAVES < nchunks; c += 4 * AR_WAVES) {
        const double p0 = partial[(int64_t)c * n + o];
        const double p1 = partial[(int64_t)(c + AR_WAVES) * n + o];
        const double p2 = partial[(int64_t)(c + 2 * AR_WAVES) * n + o];
        const double p3 = partial[(int64_t)(c + 3 * AR_WAVES) * n + o];
        s = (((s + p0) + p1) + p2) + p3;
      }
      for (; c < nchunks; c += AR_WAVES) s += partial[(int64_t)c * n + o];
    }
    sp[w][lane] = s;
    __syncthreads();
    if (w == 0 && o < n) {
      double t = sp[0][lane];
#pragma unroll
      for (int q = 1; q < AR_WAVES; ++q) t += sp[q][lane];
      // compact Q0: add the E D term, D_c Y_(n)[i, piv_c]
      const int h = (int)(o / ((int64_t)a.I * a.R));
      const gdouble* __restrict__ meta = (const gdouble*)(h ? a.meta_q : a.meta_p);
      if (meta != nullptr) {
        const int64_t rem = o - (int64_t)h * a.I * a.R;
        const int i = (int)(rem % a.I), c = (int)(rem / a.I);
        const int R = a.R;
        const int64_t k = (int64_t)meta[R * R + R + c];
        const int64_t l = k % a.L, sidx = k / a.L;
        const int64_t yi = l + a.L * (int64_t)i + a.L * (int64_t)a.I * sidx;
        const double y = a.y_f64 ? (double)((const gdouble*)a.Y)[yi] : (double)((const gfloat*)a.Y)[yi];
        t += meta[R * R + c] * y;
      }
      V[o] = t;
    }
    __syncthreads();
  }
}

int apply_num_chunks(int64_t M, int I) {
  const int iblocks = (I + AP_ROWS - 1) / AP_ROWS;
  int64_t want = (512 + iblocks - 1) / iblocks;            // about two workgroups per CU
  int64_t maxc = (M + AP_KT - 1) / AP_KT;                   // at least one k-tile each
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  // chunk length must be a multiple of the k-tile
  int64_t chunk = (M + want - 1) / want;
  chunk = ((chunk + AP_KT - 1) / AP_KT) * AP_KT;
  return (int)((M + chunk - 1) / chunk);
}

ApplyDev apply_dev(const ApplyArgs& a) {
  const int64_t M = a.L * a.S;
  int64_t chunk = (M + a.nchunks - 1) / a.nchunks;
  chunk = ((chunk + AP_KT - 1) / AP_KT) * AP_KT;
  return ApplyDev{a.Y, a.L, a.S, chunk, a.I, a.R, a.nchunks, a.Q0, a.Q0prev, a.partial, a.V, a.state,
                  a.meta_p, a.meta_q, a.y_f64 ? 1 : 0};
}

static hipError_t apply_launch(int rm, bool y_f64, dim3 grid, dim3 rgrid, const ApplyDev& a,
                               const ApplyDev* batch, hipStream_t st) {
#define CPQR_APPLY(RM)                                                                            \
  if (y_f64)                                                                                      \
    hipLaunchKernelGGL((apply_partial<double, RM>), grid, dim3(AP_THREADS), 0, st, a, batch);     \
  else                                                                                            \
    hipLaunchKernelGGL((apply_partial<float, RM>), grid, dim3(AP_THREADS), 0, st, a, batch);
  if (rm == 8) { CPQR_APPLY(8) }
  else if (rm == 16) { CPQR_APPLY(16) }
  else if (rm == 32) { CPQR_APPLY(32) }
  else return hipErrorInvalidValue;
#undef CPQR_APPLY
  hipLaunchKernelGGL(apply_reduce, rgrid, dim3(64 * AR_WAVES), 0, st, a, batch);
  return hipGetLastError();
}

unsigned apply_iblocks(int I) { return (unsigned)((I + AP_ROWS - 1) / AP_ROWS); }

unsigned apply_reduce_blocks(int I, int R) {
  const int64_t n = 2 * (int64_t)I * R;
  int64_t blocks = (n + 63) / 64;
  if (blocks > 4096) blocks = 4096;
  return (unsigned)blocks;
}

hipError_t launch_apply(const ApplyArgs& a, hipStream_t st) {
  const ApplyDev d = apply_dev(a);
  const dim3 grid((a.I + AP_ROWS - 1) / AP_ROWS, a.nchunks);
  return apply_launch(qr_rmax(a.R), a.y_f64, grid, dim3(apply_reduce_blocks(a.I, a.R)), d, nullptr, st);
}

hipError_t launch_apply_batched(const ApplyBatch& b, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  return apply_launch(b.rmax, b.y_f64, dim3(b.iblocks, b.nchunks, (unsigned)b.count),
                      dim3(b.rblocks, (unsigned)b.count), ApplyDev{}, b.args, st);
}

// ------------------------------------------------------------------ finish
__device__ inline double beta_from_fit(double fit) {
  // Section 4.3: fit > 0.95 -> 1/20000; (0.90, 0.95] -> 1/2000;
  // (0.70, 0.90] -> 1/500; otherwise 1/250
  if (fit > 0.95) return 1.0 / 20000.0;
  if (fit > 0.90) return 1.0 / 2000.0;
  if (fit > 0.70) return 1.0 / 500.0;
  return 1.0 / 250.0;
}

// Thread-0 tail of a mode update: store <Vp,Vu> and ||Vu||^2 and, after the
// sweep's last update, the fit of Section 4.1 and the extrapolation
// activation rule (Section 4.3, or a fixed/scheduled beta).
__device__ __forceinline__ void finish_state_tail(const FinishArgs& f, DevState* st, const double (&sc)[2], int bad) {
  if (!isfinite(sc[0]) || !isfinite(sc[1])) bad |= FLAG_NONFINITE;
  if (bad) atomicOr(&st->flags, bad);
  st->vpvu = sc[0];
  st->vuvu = sc[1];
  if (f.last_in_sweep) {
    const double res2 = st->nx2 - 2.0 * sc[0] + sc[1];
    const double fit = 1.0 - sqrt(res2 > 0.0 ? res2 : 0.0) / sqrt(st->nx2);
    const int k0 = st->sweep;
    f.fit_hist[k0] = fit;
    if (!isfinite(fit)) atomicOr(&st->flags, FLAG_NONFINITE);
    if (f.extrap != 0 && f.beta_sched != nullptr) {
      // scheduled beta for the next sweep (k0 + 1 is its 0-based index)
      if (k0 + 1 < f.sched_len) {
        st->active = 1;
        st->beta = f.beta_sched[k0 + 1];
        st->beta_sweep = k0 + 1;
      }
    } else if (f.extrap != 0 && !st->active) {
      if (f.fixed_beta > 0.0) {
        if (k0 == 0) {
          st->active = 1;
          st->beta = f.fixed_beta;
          st->beta_sweep = 1;
        }
      } else if (k0 >= 1 && fabs(fit - f.fit_hist[k0 - 1]) < f.delta) {
        st->active = 1;
        st->beta = beta_from_fit(fit);
        st->beta_sweep = k0 + 1;
      }
    }
    st->fit = fit;
    st->sweep = k0 + 1;
  }
}

template <int RMAX, int RPT>
__global__ CPQR_QR_KERNEL(RMAX) void finish_update(FinishArgs f0, const FinishArgs* __restrict__ batch) {
  const FinishArgs f = kernel_args(f0, batch, blockIdx.x);
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  __shared__ double sR0[RMAX][RMAX + 1];
  constexpr int NT = QrCfg<RMAX>::NT, NW = QrCfg<RMAX>::NW;
  __shared__ double sred2[NW][2];
  __shared__ double sredR[NW][RMAX];
  const int tid = threadIdx.x;
  const int I = f.I, R = f.R;
  DevState* st = f.state;
  const gdouble* __restrict__ gV = (const gdouble*)f.V;
  gdouble* __restrict__ gA = (gdouble*)f.A;
  gdouble* __restrict__ gq64 = (gdouble*)f.q64;
  gfloat* __restrict__ gq32 = (gfloat*)f.q32;
  for (int e = tid; e < RMAX * RMAX; e += NT) {
    const int i = e / RMAX, c = e % RMAX;
    sR0[i][c] = (i < R && c < R) ? ((const gdouble*)f.R0)[i + R * c] : 0.0;
  }
  const bool active = (f.extrap != 0) && st->active;
  const double beta = active ? st->beta : 0.0;
  const double cp = 1.0 + beta, cq = -f.alpha * beta;
  __syncthreads();

  int bad = 0;
  // singular or nearly singular Z_n (dependent R factors)
  if (rank_deficient(R, [&](int c) { return sR0[c][c]; })) bad |= FLAG_RANKDEF;
  QrRow<RMAX> a[RPT];
  double sc[2] = {0.0, 0.0};
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int row = tid + NT * p;
    double vu[RMAX];
    // groups of eight columns: branch-free loads (index 0 outside the
    // matrix, selected away) so that a group's loads are in flight together
#pragma unroll
    for (int c0 = 0; c0 < RMAX; c0 += 8) {
      double lp[8], lq[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u;
        const int64_t e = (row < I && c < R) ? row + (int64_t)I * c : 0;
        lp[u] = gV[e];
        lq[u] = gV[(int64_t)I * R + e];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u;
        const bool in = row < I && c < R;
        const double vp = in ? lp[u] : 0.0, vq = in ? lq[u] : 0.0;
        vu[c] = active ? fma(cq, vq, cp * vp) : vp;
        sc[0] = fma(vp, vu[c], sc[0]);
        sc[1] = fma(vu[c], vu[c], sc[1]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // back substitution of R0 ahat = vu (row of Ahat R0^T = Vu)
    static_for<0, RMAX>([&](auto ic) {
      constexpr int c = RMAX - 1 - decltype(ic)::value;
      double s = vu[c];
      static_for<c + 1, RMAX>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        s = fma(-sR0[c][d], a[p].get(d), s);
      });
      a[p].set(c, (c < R && row < I && sR0[c][c] != 0.0) ? s / sR0[c][c] : 0.0);
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  block_allreduce<2, NW>(sc, sred2);
  // lambda = column norms of Ahat.  The wave partials of the squared norms
  // go to LDS; lane c of every wave then owns column c (its total, norm and
  // reciprocal), and each row takes the reciprocals with lane reads.
  {
    // two halves of at most 16 columns keep the reduction's registers low
    constexpr int H = RMAX > 16 ? 16 : RMAX;
    constexpr int G = 64 / H;
    const int lane = tid & 63, wave = tid >> 6;
    static_for<0, RMAX / H>([&](auto hc) {
      constexpr int h0 = decltype(hc)::value * H;
      double cn[H];
#pragma unroll
      for (int c = 0; c < H; ++c) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < RPT; ++p) s = fma(a[p].get(h0 + c), a[p].get(h0 + c), s);
        cn[c] = s;
      }
      wave_transpose_reduce<H>(cn);
      if ((lane % G) == 0) sredR[wave][h0 + lane / G] = cn[0];
    });
  }
  __syncthreads();
  const int lane = tid & 63;
  double inv_l = 0.0;
  {
    double tot = 0.0;
    if (lane < RMAX) {
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += sredR[w][lane];
    }
    const bool col = lane < R;
    const double lam = sqrt(tot);
    const double lmax = wave_max(col ? lam : 0.0);
    if (__any(col && !(lam > kRankRel * lmax))) bad |= FLAG_RANKDEF;
    if (__any(col && !isfinite(lam))) bad |= FLAG_NONFINITE;
    inv_l = (col && lam != 0.0) ? 1.0 / lam : 0.0;
    if (tid < R) ((gdouble*)f.lambda)[tid] = lam;
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c) {
    const double ic = lane_read(inv_l, c);
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int row = tid + NT * p;
      a[p].set(c, a[p].get(c) * ic);
      if (row < I && c < R) gA[row + (int64_t)I * c] = a[p].get(c);
    }
  }
  block_qr<RMAX, RPT>(a, R, sm);
  block_qr_publish<RMAX>(a[0], R, sm, wy, true);
  block_qr_wy_product<RMAX>(sm, wy, R, nullptr, 0);
  for (int e = tid; e < R * R; e += NT) {
    const int i = e % R, c = e / R;
    ((gdouble*)f.Rn)[e] = wy.Rm[i][c];
  }
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int row = tid + NT * p;
    if (row < I)
      block_qr_q_row<RMAX>(a[p], row, R, sm, wy, [&](int c, double val) {
        if (gq64) gq64[row + (int64_t)I * c] = val;
        if (gq32) gq32[row + (int64_t)I * c] = (float)val;
      });
  }
  if (tid == 0) {
    // a mode smaller than the rank has min(I, R) reflectors; the padded
    // rows of R_n (c >= I) are zero by construction
    if (rank_deficient(R < I ? R : I, [&](int c) { return wy.Rm[c][c]; })) bad |= FLAG_RANKDEF;
    finish_state_tail(f, st, sc, bad);
  }
}

// ------------------------------------------------ column-distributed layout
// finish_update for factors of at most 256 rows, the factor QR in the
// column-distributed layout of col_qr (colqr_device.h) with eight waves (two
// per SIMD): wave w owns columns [CPW w, CPW w + CPW) of every row, so the
// column norms (lambda) and every reduction of a Householder step stay
// inside one wave.  The arithmetic per entry is that of finish_update (same
// Vu, solve, lambda, reflector convention and T) except that the solve
// multiplies by the reciprocals of R0's diagonal; the reflectors go to
// form_qn for the explicit Q_n, off the next update's Z QR path, and so does
// T of the compact WY form.  Layout of f.qn: V rows (I x R column-major) at
// 0, V1 and U (RMAX x RMAX row-major) at QN_V1 and QN_U, the signs of
// diag(R) at QN_SGN and tau at QN_TAU.
static constexpr int QN_V1 = 256 * 32, QN_U = QN_V1 + 32 * 32, QN_SGN = QN_U + 32 * 32, QN_TAU = QN_SGN + 32;
// Eight waves, two per SIMD: each owns RMAX / 8 columns, and one wave's
// reduction, barrier and LDS waits overlap the other's work (measured at
// 256^3 rank 32: 46.4 us with four waves, 41.1 us with eight).
static constexpr int FC_NW = 8, FC_NT = 64 * FC_NW;

template <int RMAX, int RPL>
__global__ __launch_bounds__(FC_NT) __attribute__((amdgpu_waves_per_eu(FC_NW / 4, FC_NW / 4)))
void finish_col(FinishArgs f0, const FinishArgs* __restrict__ batch) {
  const FinishArgs f = kernel_args(f0, batch, blockIdx.x);
  using Cfg = ColCfg<RMAX, FC_NW>;
  constexpr int CPW = Cfg::CPW, NV = Cfg::NV, G = 64 / NV, NT = FC_NT;
  constexpr int MR = 64 * RPL;
  constexpr int LDR = RMAX + 2;   // 16-byte aligned rows of R0
  __shared__ QrSmem<RMAX> sm;
  __shared__ __attribute__((aligned(16))) double sR0[RMAX][LDR];
  __shared__ double rinv[RMAX];
  __shared__ double sA[MR][RMAX + 1];
  __shared__ double xb[2][MR];
  __shared__ double xp[2][2][MR];
  __shared__ double sred2[FC_NW][2];
  __shared__ double slam[RMAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = CPW * wave;
  const int I = f.I, R = f.R;
  DevState* st = f.state;
  const gdouble* __restrict__ gV = (const gdouble*)f.V;
  for (int e = tid; e < RMAX * RMAX; e += NT) {
    const int i = e / RMAX, c = e % RMAX;
    const double r0 = ((const gdouble*)f.R0)[(i < R && c < R) ? i + R * c : 0];
    sR0[i][c] = (i < R && c < R) ? r0 : 0.0;
    if (i == c) rinv[c] = (c < R && r0 != 0.0) ? 1.0 / r0 : 0.0;
  }
  const bool active = (f.extrap != 0) && st->active;
  const double beta = active ? st->beta : 0.0;
  const double cp = 1.0 + beta, cq = -f.alpha * beta;
  // Vu = (1 + beta) Vp - alpha beta Vq element by element (coalesced reads of
  // the column-major I x R halves, all issued before they are used),
  // <Vp,Vu> and ||Vu||^2
  double sc[2] = {0.0, 0.0};
  {
    constexpr int NE = MR * RMAX / NT;
    double vp[NE], vq[NE];
    // without extrapolation in this sweep Vq is not read at all
    const bool load_q = f.extrap != 0;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tid + NT * t;
      const int r = e % MR, c = e / MR;
      const int64_t g = (r < I && c < R) ? r + (int64_t)I * c : 0;
      vp[t] = gV[g];
      vq[t] = load_q ? gV[(int64_t)I * R + g] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tid + NT * t;
      const int r = e % MR, c = e / MR;
      const bool in = r < I && c < R;
      const double p = in ? vp[t] : 0.0, q = in ? vq[t] : 0.0;
      const double vu = active ? fma(cq, q, cp * p) : p;
      sc[0] = fma(p, vu, sc[0]);
      sc[1] = fma(vu, vu, sc[1]);
      sA[r][c] = vu;
    }
  }
  block_allreduce<2, FC_NW>(sc, sred2);   // its barriers also publish sR0, rinv and sA
  // back substitution of R0 ahat = vu, one row per thread, in place in sA
  static_assert(MR <= NT, "one row per thread");
  if (tid < MR) {
    double x[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) x[c] = sA[tid][c];
    const bool row_in = tid < I;
    static_for<0, RMAX>([&](auto ic) __attribute__((always_inline)) {
      constexpr int c = RMAX - 1 - decltype(ic)::value;
      double s = x[c];
      static_for<c + 1, RMAX>([&](auto dc) __attribute__((always_inline)) {
        constexpr int d = decltype(dc)::value;
        s = fma(-sR0[c][d], x[d], s);
      });
      x[c] = row_in ? s * rinv[c] : 0.0;
      __builtin_amdgcn_sched_barrier(0);
    });
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sA[tid][c] = x[c];
  }
  __syncthreads();
  // this wave's columns of every row; lambda = column norms (a reduction over
  // this wave's lanes only), A = Ahat / lambda
  double a[RPL][CPW];
  static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      a[p][q] = sA[lane + 64 * p][c0 + q];
    });
  });
  {
    double cn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cn[v] = 0.0;
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        cn[q] = fma(a[p][q], a[p][q], cn[q]);
      });
    });
    wave_transpose_reduce<NV>(cn);
    gdouble* __restrict__ gA = (gdouble*)f.A;
    static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const int c = c0 + q;
      const double lam = sqrt(lane_read(cn[0], G * q));
      const double inv = (c < R && lam != 0.0) ? 1.0 / lam : 0.0;
      if (lane == 0 && c < R) {
        slam[c] = lam;
        ((gdouble*)f.lambda)[c] = lam;
      }
      static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = decltype(pc)::value;
        const int row = lane + 64 * p;
        a[p][q] *= inv;
        if (row < I && c < R) gA[row + (int64_t)I * c] = a[p][q];
      });
    });
  }
  // Householder QR of A (rows beyond I are zero)
  if constexpr (CPW % 2 == 0)
    col_qr_pair<RMAX, RPL, FC_NW>(a, R, xp, sm);
  else
    col_qr<RMAX, RPL, FC_NW, false>(a, R, [&](int) { return I; }, xb, sm);
  // R_n = D R (D = sign(diag R)) and the reflectors for form_qn
  gdouble* __restrict__ qv = (gdouble*)f.qn;
  static_for<0, CPW>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const int c = c0 + q;
    const double sc_c = sm.scale[c < R ? c : 0];
    if (lane < RMAX) {
      const int j = lane;
      const double sg = (j < R && sm.beta[j] < 0.0) ? -1.0 : 1.0;
      const bool in = (j < R) && (c < R);
      const double rr = (c > j) ? a[0][q] : ((c == j) ? sm.beta[j] : 0.0);
      if (in) ((gdouble*)f.Rn)[j + R * c] = sg * rr;
      const double v1 = (j > c) ? a[0][q] * sc_c : ((j == c) ? 1.0 : 0.0);
      qv[QN_V1 + j * RMAX + c] = in ? v1 : 0.0;
      if (c == 0) qv[QN_SGN + j] = sg;
    }
    static_for<0, RPL>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p = decltype(pc)::value;
      const int row = lane + 64 * p;
      const double v = (row > c) ? a[p][q] * sc_c : ((row == c) ? 1.0 : 0.0);
      if (row < I && c < R) qv[row + (int64_t)I * c] = v;
    });
  });
  for (int e = tid; e < RMAX * RMAX; e += NT) qv[QN_U + e] = sm.U[e / RMAX][e % RMAX];
  if (tid < RMAX) qv[QN_TAU + tid] = (tid < R) ? sm.tau[tid] : 0.0;
  if (wave == 0) {
    // rank tests of R0, lambda and R_n (|R_n[c][c]| = |beta_c|; a mode
    // smaller than the rank has min(I, R) reflectors), one value per lane
    const bool in = lane < R;
    const double r0 = in ? sR0[lane][lane] : 0.0, lam = in ? slam[lane] : 0.0;
    const double bt = in ? sm.beta[lane] : 0.0;
    int bad = 0;
    if (wave_rank_deficient(R, r0)) bad |= FLAG_RANKDEF;
    if (wave_rank_deficient(R, lam)) bad |= FLAG_RANKDEF;
    if (__ballot(in && !isfinite(lam)) != 0) bad |= FLAG_NONFINITE;
    if (wave_rank_deficient(R < I ? R : I, bt)) bad |= FLAG_RANKDEF;
    if (lane == 0) finish_state_tail(f, st, sc, bad);
  }
}

// Explicit Q_n = (E - V M) diag(sgn), M = T V1^T, from the reflectors that
// finish_col leaves in f.qn (one row per thread, the WY product of
// block_qr_wy_product and the row arithmetic of wy_q_row).
template <int RMAX>
__global__ __launch_bounds__(256) void form_qn(FinishArgs f0, const FinishArgs* __restrict__ batch) {
  const FinishArgs f = kernel_args(f0, batch, blockIdx.x);
  __shared__ QrSmem<RMAX> sm;
  __shared__ QrWySmem<RMAX> wy;
  const int tid = threadIdx.x;
  const int I = f.I, R = f.R;
  const gdouble* __restrict__ qv = (const gdouble*)f.qn;
  gdouble* __restrict__ gq64 = (gdouble*)f.q64;
  gfloat* __restrict__ gq32 = (gfloat*)f.q32;
  for (int e = tid; e < RMAX * RMAX; e += 256) {
    const int k = e / RMAX, c = e % RMAX;
    wy.V1[k][c] = qv[QN_V1 + e];
    sm.U[k][c] = qv[QN_U + e];
  }
  if (tid < RMAX) {
    sm.sgn[tid] = qv[QN_SGN + tid];
    sm.tau[tid] = qv[QN_TAU + tid];
  }
  __syncthreads();
  block_qr_build_t<RMAX>(R, sm);
  block_qr_wy_product<RMAX, 256>(sm, wy, R, nullptr, 0);
  const int r = tid;
  if (r < I) {
    double v[RMAX];
#pragma unroll
    for (int m = 0; m < RMAX; ++m) v[m] = (m < R) ? qv[r + (int64_t)I * (m < R ? m : 0)] : 0.0;
    wy_q_row<RMAX, RMAX, 0>(v, r, R, sm, wy, [&](int c, double val) {
      if (gq64) gq64[r + (int64_t)I * c] = val;
      if (gq32) gq32[r + (int64_t)I * c] = (float)val;
    });
  }
}

// ------------------------------------------------------------ tall factors
// A mode with more rows than the single-workgroup factor QR holds in
// registers: this kernel streams the rows in chunks of its 256 threads for
// the solve Ahat R0^T = Vu, lambda, A = Ahat / lambda and the fit (the same
// arithmetic per row as finish_update), and leaves the factor QR of A to the
// two-level TSQR (an explicit source matrix) followed by tall_factor_tail.
static constexpr int FT_THREADS = 256;

template <int RMAX>
__global__ __launch_bounds__(FT_THREADS) void finish_tall(FinishArgs f) {
  constexpr int NT = FT_THREADS, NW = NT / 64;
  __shared__ double sR0[RMAX][RMAX + 1];
  __shared__ double sred2[NW][2];
  __shared__ double sredR[NW][RMAX];
  __shared__ double sinv[RMAX], slam[RMAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int I = f.I, R = f.R;
  DevState* st = f.state;
  const gdouble* __restrict__ gV = (const gdouble*)f.V;
  gdouble* __restrict__ gA = (gdouble*)f.A;
  for (int e = tid; e < RMAX * RMAX; e += NT) {
    const int i = e / RMAX, c = e % RMAX;
    sR0[i][c] = (i < R && c < R) ? ((const gdouble*)f.R0)[i + R * c] : 0.0;
  }
  const bool active = (f.extrap != 0) && st->active;
  const double beta = active ? st->beta : 0.0;
  const double cp = 1.0 + beta, cq = -f.alpha * beta;
  __syncthreads();
  int bad = 0;
  if (rank_deficient(R, [&](int c) { return sR0[c][c]; })) bad |= FLAG_RANKDEF;
  double sc[2] = {0.0, 0.0};
  double cn[RMAX];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) cn[c] = 0.0;
  for (int r0 = 0; r0 < I; r0 += NT) {
    // keeps the R0 reads (loop-invariant LDS loads) inside the row loop, so
    // that they are not all held in registers across it
    __asm__ volatile("" ::: "memory");
    const int row = r0 + tid;
    double vu[RMAX], ah[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const bool in = row < I && c < R;
      const int64_t e = in ? row + (int64_t)I * c : 0;
      const double vp = in ? gV[e] : 0.0, vq = in ? gV[(int64_t)I * R + e] : 0.0;
      vu[c] = active ? fma(cq, vq, cp * vp) : vp;
      sc[0] = fma(vp, vu[c], sc[0]);
      sc[1] = fma(vu[c], vu[c], sc[1]);
    }
    // back substitution of R0 ahat = vu (row of Ahat R0^T = Vu)
    static_for<0, RMAX>([&](auto ic) {
      constexpr int c = RMAX - 1 - decltype(ic)::value;
      double t = vu[c];
      static_for<c + 1, RMAX>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        t = fma(-sR0[c][d], ah[d], t);
      });
      ah[c] = (c < R && row < I && sR0[c][c] != 0.0) ? t / sR0[c][c] : 0.0;
      __builtin_amdgcn_sched_barrier(0);
    });
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      cn[c] = fma(ah[c], ah[c], cn[c]);
      if (row < I && c < R) gA[row + (int64_t)I * c] = ah[c];
    }
  }
  block_allreduce<2, NW>(sc, sred2);
  {
    constexpr int H = RMAX > 16 ? 16 : RMAX;
    constexpr int G = 64 / H;
    static_for<0, RMAX / H>([&](auto hc) {
      constexpr int h0 = decltype(hc)::value * H;
      double part[H];
#pragma unroll
      for (int c = 0; c < H; ++c) part[c] = cn[h0 + c];
      wave_transpose_reduce<H>(part);
      if ((lane % G) == 0) sredR[wave][h0 + lane / G] = part[0];
    });
  }
  __syncthreads();
  if (tid < RMAX) {
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sredR[w][tid];
    const double lam = sqrt(tot);
    slam[tid] = lam;
    sinv[tid] = (tid < R && lam != 0.0) ? 1.0 / lam : 0.0;
    if (tid < R) ((gdouble*)f.lambda)[tid] = lam;
  }
  __syncthreads();
  if (tid == 0) {
    if (rank_deficient(R, [&](int c) { return slam[c]; })) bad |= FLAG_RANKDEF;
    for (int c = 0; c < R; ++c)
      if (!isfinite(slam[c])) bad |= FLAG_NONFINITE;
  }
  // A = Ahat / lambda (the rows were written by this workgroup above; the
  // barriers since then order those stores before these loads)
  for (int c = 0; c < R; ++c) {
    const double ic = sinv[c];
    for (int i = tid; i < I; i += NT) gA[i + (int64_t)I * c] = gA[i + (int64_t)I * c] * ic;
  }
  if (tid == 0) finish_state_tail(f, st, sc, bad);
}

// After the TSQR of a tall factor: the float32 copy of Q_n for the TTMs (the
// TSQR wrote the float64 one) and the rank check of R_n's diagonal.
__global__ void tall_factor_tail(int64_t n, int R, const double* __restrict__ q64, float* __restrict__ q32,
                                 const double* __restrict__ Rn, DevState* st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q32 != nullptr && i < n) ((gfloat*)q32)[i] = (float)((const gdouble*)q64)[i];
  if (blockIdx.x == 0 && threadIdx.x == 0 && st != nullptr) {
    if (rank_deficient(R, [&](int c) { return Rn[c + (int64_t)R * c]; })) atomicOr(&st->flags, FLAG_RANKDEF);
  }
}

hipError_t launch_finish_tall(const FinishArgs& f, hipStream_t st) {
  const int rm = qr_rmax(f.R);
  if (rm == 8) hipLaunchKernelGGL(finish_tall<8>, dim3(1), dim3(FT_THREADS), 0, st, f);
  else if (rm == 16) hipLaunchKernelGGL(finish_tall<16>, dim3(1), dim3(FT_THREADS), 0, st, f);
  else if (rm == 32) hipLaunchKernelGGL(finish_tall<32>, dim3(1), dim3(FT_THREADS), 0, st, f);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_tall_factor_tail(int I, int R, const double* q64, float* q32, const double* Rn,
                                   DevState* state, hipStream_t st) {
  const int64_t n = (int64_t)I * R;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(tall_factor_tail, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, n, R, q64, q32, Rn,
                     state);
  return hipGetLastError();
}

static hipError_t finish_launch(int rm, int rp, unsigned blocks, const FinishArgs& f,
                                const FinishArgs* batch, hipStream_t st) {
#define CPQR_FIN(RM, RP) \
  hipLaunchKernelGGL((finish_update<RM, RP>), dim3(blocks), dim3(QrCfg<RM>::NT), 0, st, f, batch)
  if (rm == 8) { if (rp == 1) CPQR_FIN(8, 1); else CPQR_FIN(8, 2); }
  else if (rm == 16) { if (rp == 1) CPQR_FIN(16, 1); else CPQR_FIN(16, 2); }
  else if (rm == 32) { if (rp == 1) CPQR_FIN(32, 1); else CPQR_FIN(32, 2); }
  else return hipErrorInvalidValue;
#undef CPQR_FIN
  return hipGetLastError();
}

// Rows per lane of finish_col for a factor of I rows (0: beyond its 256 rows).
static int col_rpl(int I) { return I <= 64 ? 1 : (I <= 128 ? 2 : (I <= 256 ? 4 : 0)); }

static hipError_t finish_col_launch(int rm, int rpl, unsigned blocks, const FinishArgs& f,
                                    const FinishArgs* batch, hipStream_t st) {
#define CPQR_FC(RM, RP) \
  hipLaunchKernelGGL((finish_col<RM, RP>), dim3(blocks), dim3(FC_NT), 0, st, f, batch)
#define CPQR_FC_RPL(RM) \
  if (rpl == 1) CPQR_FC(RM, 1); else if (rpl == 2) CPQR_FC(RM, 2); else if (rpl == 4) CPQR_FC(RM, 4); \
  else return hipErrorInvalidValue;
  if (rm == 8) { CPQR_FC_RPL(8) }
  else if (rm == 16) { CPQR_FC_RPL(16) }
  else if (rm == 32) { CPQR_FC_RPL(32) }
  else return hipErrorInvalidValue;
#undef CPQR_FC_RPL
#undef CPQR_FC
  return hipGetLastError();
}

static hipError_t form_qn_launch(int rm, unsigned blocks, const FinishArgs& f, const FinishArgs* batch,
                                 hipStream_t st) {
  if (rm == 8) hipLaunchKernelGGL((form_qn<8>), dim3(blocks), dim3(256), 0, st, f, batch);
  else if (rm == 16) hipLaunchKernelGGL((form_qn<16>), dim3(blocks), dim3(256), 0, st, f, batch);
  else if (rm == 32) hipLaunchKernelGGL((form_qn<32>), dim3(blocks), dim3(256), 0, st, f, batch);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_finish_head(const FinishArgs& f, hipStream_t st, bool* tail) {
  *tail = false;
  if (f.I > CPQR_MAX_FACTOR_ROWS) return hipErrorInvalidValue;
  const int rm = qr_rmax(f.R), rpl = col_rpl(f.I);
  if (rpl > 0 && f.qn != nullptr) {
    // column-distributed layout: 512 threads, rows r < 256; Q_n in form_qn
    *tail = true;
    return finish_col_launch(rm, rpl, 1, f, nullptr, st);
  }
  return finish_launch(rm, factor_rpt(f.I), 1, f, nullptr, st);
}

hipError_t launch_finish_tail(const FinishArgs& f, hipStream_t st) {
  if (f.I > 256 || f.R > 32 || f.qn == nullptr) return hipErrorInvalidValue;
  return form_qn_launch(qr_rmax(f.R), 1, f, nullptr, st);
}

hipError_t launch_finish(const FinishArgs& f, hipStream_t st) {
  bool tail = false;
  hipError_t e = launch_finish_head(f, st, &tail);
  if (e != hipSuccess || !tail) return e;
  return launch_finish_tail(f, st);
}

hipError_t launch_finish_batched(int count, int rmax, int rpt, const FinishArgs* args, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return finish_launch(rmax, rpt, (unsigned)count, FinishArgs{}, args, st);
}

int finish_col_rpl(int I) { return col_rpl(I); }

hipError_t launch_finish_col_batched(int count, int rmax, int rpl, const FinishArgs* args, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return finish_col_launch(rmax, rpl, (unsigned)count, FinishArgs{}, args, st);
}

hipError_t launch_form_qn_batched(int count, int rmax, const FinishArgs* args, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return form_qn_launch(rmax, (unsigned)count, FinishArgs{}, args, st);
}

// ------------------------------------------------------------------- norms
static constexpr int NORM_BLOCKS = 1024;
static constexpr int NORM_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(NORM_THREADS) void sumsq_kernel(const T* __restrict__ x, int64_t n,
                                                             double* __restrict__ part) {
  __shared__ double red[NORM_THREADS / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * NORM_THREADS) {
    const double v = (double)x[i];
    s = fma(v, v, s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NORM_THREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

int sumsq_blocks(int64_t n) {
  int64_t b = (n + NORM_THREADS - 1) / NORM_THREADS;
  return (int)(b < NORM_BLOCKS ? (b < 1 ? 1 : b) : NORM_BLOCKS);
}

hipError_t launch_sumsq(const void* x, bool f64, int64_t n, double* part, hipStream_t st) {
  const int b = sumsq_blocks(n);
  if (f64) hipLaunchKernelGGL(sumsq_kernel<double>, dim3(b), dim3(NORM_THREADS), 0, st, (const double*)x, n, part);
  else     hipLaunchKernelGGL(sumsq_kernel<float>, dim3(b), dim3(NORM_THREADS), 0, st, (const float*)x, n, part);
  return hipGetLastError();
}

__global__ void state_init_kernel(DevState* s, const double* part, int nparts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nparts; ++i) t += part[i];
    s->nx2 = t;
    s->beta = 0.0;
    s->vpvu = 0.0;
    s->vuvu = 0.0;
    s->fit = 0.0;
    s->active = 0;
    s->beta_sweep = 0;
    s->sweep = 0;
    s->flags = isfinite(t) ? 0 : FLAG_NONFINITE;
  }
}

hipError_t launch_state_init(DevState* s, const double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, st, s, part, nparts);
  return hipGetLastError();
}

// Rank test of the initial factors' R factors (after the QRs of the
// "Initialize" step of Algorithms 2 and 3): mode n's diagonal has
// min(I_n, R) entries; a relative test (rank_deficient) flags dependent
// initial columns before the first sweep.
struct InitRank {
  const double* rf;   // N x R x R column-major R factors
  int N, R;
  int rows[CPQR_MAX_ORDER];   // min(I_n, R)
  DevState* st;
};

__global__ void init_rank_check(InitRank a) {
  const int n = threadIdx.x;
  if (n >= a.N) return;
  const gdouble* r = (const gdouble*)a.rf + (int64_t)n * a.R * a.R;
  if (rank_deficient(a.rows[n], [&](int c) { return r[c + (int64_t)a.R * c]; }))
    atomicOr(&a.st->flags, FLAG_RANKDEF);
}

hipError_t launch_init_rank_check(const double* rf, int N, int R, const int64_t* dims, DevState* st,
                                  hipStream_t s) {
  if (N < 1 || N > CPQR_MAX_ORDER) return hipErrorInvalidValue;
  InitRank a{};
  a.rf = rf;
  a.N = N;
  a.R = R;
  for (int k = 0; k < N; ++k) a.rows[k] = (int)(dims[k] < R ? dims[k] : R);
  a.st = st;
  hipLaunchKernelGGL(init_rank_check, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

struct FactorPtrs {
  const double* a[CPQR_MAX_ORDER];
  int64_t dims[CPQR_MAX_ORDER];
};

template <typename T>
__global__ __launch_bounds__(NORM_THREADS) void residual_kernel(const T* __restrict__ x, int N,
                                                                FactorPtrs fp, const double* __restrict__ lam,
                                                                int R, int64_t n, double* __restrict__ part) {
  __shared__ double red[NORM_THREADS / 64];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * NORM_THREADS) {
    int64_t idx[CPQR_MAX_ORDER];
    int64_t rem = e;
    for (int k = 0; k < N; ++k) {
      idx[k] = rem % fp.dims[k];
      rem /= fp.dims[k];
    }
    double kv = 0.0;
    for (int r = 0; r < R; ++r) {
      double prod = lam[r];
      for (int k = 0; k < N; ++k) prod *= fp.a[k][idx[k] + fp.dims[k] * r];
      kv += prod;
    }
    const double d = (double)x[e] - kv;
    s = fma(d, d, s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NORM_THREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// ||X - K||^2 by mode-1 fibres: a wave takes one fibre (i_2 .. i_N) at a
// time, forms w_r = s lambda_r prod_{k >= 2} A_k[i_k][r] in lanes r < R
// (shared through the wave's LDS row), and its lanes run along mode 1
// (contiguous in X) with K[i] = sum_r A_1[i][r] w_r from A_1 in LDS.
// float64 throughout, as residual_kernel; R <= 64 and I_1 R <= RF_A1.
static constexpr int RF_A1 = 8192;

template <typename T>
__global__ __launch_bounds__(NORM_THREADS) void residual_fiber_kernel(const T* __restrict__ x, int N,
                                                                      FactorPtrs fp, const double* __restrict__ lam,
                                                                      double lscale, int R, int64_t nfib,
                                                                      double* __restrict__ part) {
  __shared__ double a1s[RF_A1];
  __shared__ double wv[NORM_THREADS / 64][64];
  __shared__ double red[NORM_THREADS / 64];
  const int I1 = (int)fp.dims[0];
  for (int e = threadIdx.x; e < I1 * R; e += NORM_THREADS) {
    const int i = e / R, r = e % R;
    a1s[e] = fp.a[0][i + (int64_t)I1 * r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * (NORM_THREADS / 64);
  double s = 0.0;
  for (int64_t f = (int64_t)blockIdx.x * (NORM_THREADS / 64) + wave; f < nfib; f += nwaves) {
    if (lane < R) {
      double prod = lam[lane] * lscale;
      int64_t rem = f;
      for (int k = 1; k < N; ++k) {
        const int64_t ik = rem % fp.dims[k];
        rem /= fp.dims[k];
        prod *= fp.a[k][ik + fp.dims[k] * lane];
      }
      wv[wave][lane] = prod;
    }
    // one wave's LDS operations complete in order: the row is written
    // before any lane reads it
    const T* __restrict__ xf = x + f * I1;
    for (int i = lane; i < I1; i += 64) {
      double kv = 0.0;
      for (int r = 0; r < R; ++r) kv = fma(a1s[i * R + r], wv[wave][r], kv);
      const double d = (double)xf[i] - kv;
      s = fma(d, d, s);
    }
  }
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NORM_THREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// ||X - K||^2 with one mode-1 fibre (i_2 .. i_N) per thread, for short
// fibres (I_1 < 64, where a wave per fibre would leave lanes idle and pay
// the fibre's index arithmetic and factor loads for few entries): the thread
// forms w_r = s lambda_r prod_{k >= 2} A_k[i_k][r] in registers and runs
// along the fibre with K[i] = sum_r A_1[i][r] w_r, reading A_1 from LDS
// (every lane reads the same row: broadcast).  A_1 is held as I_1 rows of
// RM doubles, zero beyond R.  float64 throughout.
template <typename T, int RM>
__global__ __launch_bounds__(NORM_THREADS) void residual_thread_fiber_kernel(
    const T* __restrict__ x, int N, FactorPtrs fp, const double* __restrict__ lam, double lscale, int R,
    int64_t nfib, double* __restrict__ part) {
  extern __shared__ double a1t[];
  __shared__ double red[NORM_THREADS / 64];
  const int I1 = (int)fp.dims[0];
  for (int e = threadIdx.x; e < I1 * RM; e += NORM_THREADS) {
    const int i = e / RM, r = e % RM;
    a1t[e] = r < R ? fp.a[0][i + (int64_t)I1 * r] : 0.0;
  }
  __syncthreads();
  double s = 0.0;
  for (int64_t f = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; f < nfib;
       f += (int64_t)gridDim.x * NORM_THREADS) {
    double w[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) w[r] = r < R ? lam[r] * lscale : 0.0;
    int64_t rem = f;
    for (int k = 1; k < N; ++k) {
      const int64_t dk = fp.dims[k];
      const int64_t ik = rem % dk;
      rem /= dk;
      const double* __restrict__ ak = fp.a[k] + ik;
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (r < R) w[r] *= ak[dk * r];
    }
    const T* __restrict__ xf = x + f * I1;
    for (int i = 0; i < I1; ++i) {
      const double* __restrict__ row = a1t + i * RM;
      double kv = 0.0;
#pragma unroll
      for (int r = 0; r < RM; ++r) kv = fma(row[r], w[r], kv);
      const double d = (double)xf[i] - kv;
      s = fma(d, d, s);
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NORM_THREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

template <int RM>
void launch_residual_thread_fiber(const void* x, bool f64, int N, const FactorPtrs& fp, const double* lambda,
                                  double lscale, int R, int64_t nfib, int b, double* part, hipStream_t st) {
  const size_t lds = (size_t)fp.dims[0] * RM * sizeof(double);
  if (f64)
    hipLaunchKernelGGL((residual_thread_fiber_kernel<double, RM>), dim3(b), dim3(NORM_THREADS), lds, st,
                       (const double*)x, N, fp, lambda, lscale, R, nfib, part);
  else
    hipLaunchKernelGGL((residual_thread_fiber_kernel<float, RM>), dim3(b), dim3(NORM_THREADS), lds, st,
                       (const float*)x, N, fp, lambda, lscale, R, nfib, part);
}

hipError_t launch_residual(const void* x, bool f64, int N, const int64_t* dims_host,
                           double* const* factors, const double* lambda, int R, double* part,
                           hipStream_t st, double lambda_scale) {
  FactorPtrs fp;
  int64_t n = 1;
  for (int k = 0; k < N; ++k) {
    fp.a[k] = factors[k];
    fp.dims[k] = dims_host[k];
    n *= dims_host[k];
  }
  const int b = sumsq_blocks(n);
  if (R <= 64 && dims_host[0] < 64 && N >= 2) {
    const int64_t nfib = n / dims_host[0];
    if (R <= 8) launch_residual_thread_fiber<8>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    else if (R <= 16) launch_residual_thread_fiber<16>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    else if (R <= 24) launch_residual_thread_fiber<24>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    else if (R <= 32) launch_residual_thread_fiber<32>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    else if (R <= 48) launch_residual_thread_fiber<48>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    else launch_residual_thread_fiber<64>(x, f64, N, fp, lambda, lambda_scale, R, nfib, b, part, st);
    return hipGetLastError();
  }
  if (R <= 64 && dims_host[0] * R <= RF_A1) {
    const int64_t nfib = n / dims_host[0];
    if (f64)
      hipLaunchKernelGGL(residual_fiber_kernel<double>, dim3(b), dim3(NORM_THREADS), 0, st, (const double*)x, N, fp,
                         lambda, lambda_scale, R, nfib, part);
    else
      hipLaunchKernelGGL(residual_fiber_kernel<float>, dim3(b), dim3(NORM_THREADS), 0, st, (const float*)x, N, fp,
                         lambda, lambda_scale, R, nfib, part);
    return hipGetLastError();
  }
  if (lambda_scale != 1.0) return hipErrorInvalidValue;
  if (f64) hipLaunchKernelGGL(residual_kernel<double>, dim3(b), dim3(NORM_THREADS), 0, st, (const double*)x, N, fp, lambda, R, n, part);
  else     hipLaunchKernelGGL(residual_kernel<float>, dim3(b), dim3(NORM_THREADS), 0, st, (const float*)x, N, fp, lambda, R, n, part);
  return hipGetLastError();
}

// ---------------------------------------------------------------- copy list
// One launch copies up to COPY_LIST_MAX device buffers (the checkpoint of
// the learned extrapolation: factors, Q0 halves, live intermediates).  Work
// goes in chunks of COPY_CHUNK bytes; block b finds its buffer from the
// chunk prefix sums.  16-byte accesses where both addresses are 16-byte
// aligned, 4-byte ones otherwise and for the tail (sizes are multiples of 4).
static constexpr int COPY_THREADS = 256;
static constexpr int64_t COPY_CHUNK = 16384;

struct CopyListArgs {
  CopySeg seg[COPY_LIST_MAX];
  int64_t chunk0[COPY_LIST_MAX + 1];   // first chunk of each buffer; chunk0[n] = total
  int n;
};

__global__ __launch_bounds__(COPY_THREADS) void copy_list_kernel(CopyListArgs a) {
  const int64_t c = blockIdx.x;
  int s = 0;
  while (s + 1 < a.n && a.chunk0[s + 1] <= c) ++s;
  const CopySeg g = a.seg[s];
  const int64_t off = (c - a.chunk0[s]) * COPY_CHUNK;
  const int64_t rest = g.bytes - off;
  const int64_t len = rest < COPY_CHUNK ? rest : COPY_CHUNK;
  const char* __restrict__ src = static_cast<const char*>(g.src) + off;
  char* __restrict__ dst = static_cast<char*>(g.dst) + off;
  int64_t done = 0;
  if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
    const int64_t n16 = len / 16;
    const uint4* __restrict__ s4 = reinterpret_cast<const uint4*>(src);
    uint4* __restrict__ d4 = reinterpret_cast<uint4*>(dst);
    for (int64_t i = threadIdx.x; i < n16; i += COPY_THREADS) d4[i] = s4[i];
    done = n16 * 16;
  }
  const int64_t n4 = (len - done) / 4;
  const uint32_t* __restrict__ s1 = reinterpret_cast<const uint32_t*>(src + done);
  uint32_t* __restrict__ d1 = reinterpret_cast<uint32_t*>(dst + done);
  for (int64_t i = threadIdx.x; i < n4; i += COPY_THREADS) d1[i] = s1[i];
}

hipError_t launch_copy_list(const CopySeg* segs, int n, hipStream_t st) {
  int i = 0;
  while (i < n) {
    CopyListArgs a{};
    a.n = 0;
    int64_t chunks = 0;
    for (; i < n && a.n < COPY_LIST_MAX; ++i) {
      if (segs[i].bytes <= 0) continue;
      if (segs[i].bytes % 4 != 0) return hipErrorInvalidValue;
      a.seg[a.n] = segs[i];
      a.chunk0[a.n] = chunks;
      chunks += (segs[i].bytes + COPY_CHUNK - 1) / COPY_CHUNK;
      ++a.n;
    }
    a.chunk0[a.n] = chunks;
    if (chunks == 0) continue;
    hipLaunchKernelGGL(copy_list_kernel, dim3((unsigned)chunks), dim3(COPY_THREADS), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cpqr
