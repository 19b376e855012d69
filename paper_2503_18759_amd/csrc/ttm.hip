// Mode-m tensor-times-matrix (TTM) kernels for gfx950.
//
// Section 2.1 defines Y = X x_m B with Y(..., j, ...) = sum_i X(..., i, ...) B(j, i).
// The chain of the QR-based ALS uses B = Q_m^T, so with the tensor viewed as
// [L, I, S] around mode m (L = product of the dims before m, S = product of
// the dims after m, mode 1 fastest):
//
//     out[l + L r + L R s] = sum_i in[l + L i + L I s] * Q[i + I r].
//
// For a fixed s this is a skinny GEMM (L x I) * (I x R).  Each kernel streams
// the input once from HBM with 16-byte loads straight into MFMA operand
// registers and keeps Q in LDS, staged once per workgroup in MFMA lane order.
//
// Work decomposition.  The output is cut into tiles of 64 rows.  A workgroup
// (4 waves) takes 4/KS tiles per pass and gives each tile KS waves, which
// split the reduction over I into KS contiguous ranges of 32-wide k chunks
// (KS = 1, 2 or 4, chosen per shape so that tiles x KS fills the chip); the
// KS partial tiles are added through LDS.  The grid is persistent: a
// workgroup walks tile groups blockIdx.x, blockIdx.x + gridDim.x, ...
//
// Loads.  Inputs below 2 GiB are read through a buffer resource: a lane whose
// row lies past the end of the tensor or whose k lies past I gets the offset
// 0x80000000, which the hardware range check turns into a zero without a
// memory access, so ragged tiles need no branches.  The k loop is software
// pipelined over two register buffers (chunk q+1 is in flight while the MFMAs
// of chunk q issue).  Larger inputs use plain global loads.
//
//  * ttm_mc: L > 1 ("M-contiguous": rows l are adjacent in memory).  A tile
//    is 64 consecutive rows m = l + L s.  MFMA f32 16x16x4: lane
//    (i = lane%16, g = lane/16) feeds A[i][g]; with L % 4 == 0 each lane
//    loads a float4 of rows m0+4i..m0+4i+3 at column k and MFMA v uses
//    component v, so output row rho of MFMA v is m = m0 + 4 rho + v.
//    Otherwise each lane loads rows m0 + 16 v + i separately.
//  * ttm_kc: L == 1 ("K-contiguous": the contracted index is adjacent).  A
//    tile is 64 consecutive s.  The product is computed transposed,
//    C[r][s] = sum_k Q[k][r] in[k + I s], so the 16-byte loads run along k
//    and each lane stores four consecutive r of one s.
//  * ttm_bf16x3_*: same two layouts with each product computed as
//    x_hi q_hi + x_hi q_lo + x_lo q_hi on bf16 MFMA (16x16x32) with float32
//    accumulation; x is split in registers, Q is split once into LDS.
//  * ttm_generic<T>: a plain VALU kernel (float64 chain and shapes outside
//    the MFMA kernels' limits).
#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"

namespace cpqr {

static constexpr int TTM_THREADS = 256;
static constexpr int TTM_TILE = 64;
static constexpr uint32_t TTM_OOB = 0x80000000u;   // offset past any buffer we build

// Keeps the instruction scheduler from moving the prefetch loads of the next
// chunk down to their uses (which would serialise load and MFMA phases).
#define TTM_PHASE() __builtin_amdgcn_sched_barrier(0)
// Two waves per SIMD: 256 registers per lane for two chunk buffers, the
// accumulators and the staged Q operands.
#define TTM_KERNEL __global__ __launch_bounds__(TTM_THREADS) __attribute__((amdgpu_waves_per_eu(1, 2)))

// ------------------------------------------------------------------ loads
template <bool BUF>
struct TtmSrc;

// Buffer-resource source (tensor < 2 GiB): lane offset `lo` and wave-uniform
// offset `uo` in elements; an invalid lane reads zero.
template <>
struct TtmSrc<true> {
  __amdgpu_buffer_rsrc_t rsrc;
  __device__ __forceinline__ TtmSrc(const float* p, int64_t n) {
    rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * 4), 0x00020000);
  }
  __device__ __forceinline__ f32x4 ld4(int64_t lo, int64_t uo, bool ok) const {
    const uint32_t v = ok ? (uint32_t)lo * 4u : TTM_OOB;
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, v, (int)(uo * 4), 0));
  }
  __device__ __forceinline__ float ld1(int64_t lo, int64_t uo, bool ok) const {
    const uint32_t v = ok ? (uint32_t)lo * 4u : TTM_OOB;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, v, (int)(uo * 4), 0));
  }
};

// Global-pointer source (any size).
template <>
struct TtmSrc<false> {
  const float* p;
  __device__ __forceinline__ TtmSrc(const float* q, int64_t) : p(q) {}
  __device__ __forceinline__ f32x4 ld4(int64_t lo, int64_t uo, bool ok) const {
    return ok ? *reinterpret_cast<const f32x4*>(p + lo + uo) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  __device__ __forceinline__ float ld1(int64_t lo, int64_t uo, bool ok) const {
    return ok ? p[lo + uo] : 0.f;
  }
};

// Wave-uniform wave index (keeps tile bookkeeping in scalar registers).
__device__ __forceinline__ int ttm_wave() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Per-wave split of a tile-group pass: slot (which tile of the group) and
// part (which k range), with the k-chunk range [qb, qe).
struct TtmSplit {
  int tpw, slot, part, qb, qe;
  __device__ __forceinline__ TtmSplit(int ks, int TC) {
    const int wave = ttm_wave();
    tpw = 4 / ks;
    slot = wave / ks;
    part = wave - slot * ks;
    const int per = (TC + ks - 1) / ks;
    qb = part * per;
    qe = qb + per < TC ? qb + per : TC;
  }
};

// Adds the KS partial accumulators of each tile through LDS; on return the
// part-0 wave of each slot holds the sum.  `red` holds (KS-1) * tpw partial
// tiles of NREG floats per lane.  Every wave of the workgroup calls it.
template <int NREG>
__device__ __forceinline__ void ttm_reduce_parts(f32x4 (&acc)[NREG / 4], float* red, int ks,
                                                 const TtmSplit& sp) {
  const int lane = threadIdx.x & 63;
  if (sp.part > 0) {
    f32x4* dst = reinterpret_cast<f32x4*>(red) + ((sp.slot * (ks - 1) + sp.part - 1) * (NREG / 4)) * 64;
#pragma unroll
    for (int j = 0; j < NREG / 4; ++j) dst[j * 64 + lane] = acc[j];
  }
  __syncthreads();
  if (sp.part == 0) {
    for (int p = 1; p < ks; ++p) {
      const f32x4* src = reinterpret_cast<const f32x4*>(red) + ((sp.slot * (ks - 1) + p - 1) * (NREG / 4)) * 64;
#pragma unroll
      for (int j = 0; j < NREG / 4; ++j) acc[j] += src[j * 64 + lane];
    }
  }
  __syncthreads();
}


// Pipelined tile loop shared by the four MFMA kernels.  The policy P supplies
// the register buffer of one k chunk (Buf), the per-tile lane bookkeeping
// (Tile) and tile(), load(), mma(), store() and stage().  The first chunk of
// the first tile is requested before Q is staged, so the two overlap; when a
// wave owns an even number of chunks per tile, the first chunk of its next
// tile is requested while the last chunk of the current one is multiplied.
template <class P>
__device__ __forceinline__ void ttm_drive(const P& p, int64_t ntiles, int TC, int ks, float* red) {
  const TtmSplit sp(ks, TC);
  const int nq = sp.qe > sp.qb ? sp.qe - sp.qb : 0;
  const bool even = (nq & 1) == 0;
  int64_t grp = blockIdx.x;
  if (grp * sp.tpw >= ntiles) return;   // whole workgroup: no tile of this problem
  typename P::Buf bufA, bufB;
  typename P::Tile cur = p.tile(grp * sp.tpw + sp.slot);
  if (nq > 0) p.load(bufA, cur, sp.qb);
  p.stage();
  __syncthreads();
  for (; grp * sp.tpw < ntiles; grp += gridDim.x) {
    const int64_t ngrp = grp + gridDim.x;
    const bool more = ngrp * sp.tpw < ntiles;
    const typename P::Tile nxt = p.tile(ngrp * sp.tpw + sp.slot);
    f32x4 acc[P::NACC];
#pragma unroll
    for (int j = 0; j < P::NACC; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int q = 0;
    if (even) {
      // pairs whose follow-up loads stay in this tile, then a peeled last
      // pair that requests the next tile's first chunk (or chunk TC, past I:
      // every lane reads zero without a memory access)
      for (; q + 3 < nq; q += 2) {
        p.load(bufB, cur, sp.qb + q + 1);
        TTM_PHASE();
        p.mma(acc, bufA, sp.qb + q);
        TTM_PHASE();
        p.load(bufA, cur, sp.qb + q + 2);
        TTM_PHASE();
        p.mma(acc, bufB, sp.qb + q + 1);
        TTM_PHASE();
      }
      if (nq > 0) {
        p.load(bufB, cur, sp.qb + q + 1);
        TTM_PHASE();
        p.mma(acc, bufA, sp.qb + q);
        TTM_PHASE();
        p.load(bufA, nxt, more ? sp.qb : TC);
        TTM_PHASE();
        p.mma(acc, bufB, sp.qb + q + 1);
        TTM_PHASE();
      }
    } else {
      for (; q + 2 < nq; q += 2) {
        p.load(bufB, cur, sp.qb + q + 1);
        TTM_PHASE();
        p.mma(acc, bufA, sp.qb + q);
        TTM_PHASE();
        p.load(bufA, cur, sp.qb + q + 2);
        TTM_PHASE();
        p.mma(acc, bufB, sp.qb + q + 1);
        TTM_PHASE();
      }
      p.mma(acc, bufA, sp.qb + q);
    }
    if (ks > 1) ttm_reduce_parts<P::NACC * 4>(acc, red, ks, sp);
    if (sp.part == 0) p.store(acc, cur);
    cur = nxt;
    if (!even && more) p.load(bufA, cur, sp.qb);
  }
}

// Coalesced Q staging: visits Q as float4 runs of 4 consecutive k of one
// column (needs I % 4 == 0 and a 16-byte aligned Q), padded to 32 TC rows and
// 16 NB columns with zeros, and hands each run to put(k0, c, value).
template <int NB, class Put>
__device__ __forceinline__ void stage_q_runs(const float* __restrict__ Q, int I, int R, int TC, Put put) {
  const int runs_per_col = 8 * TC;                 // 32 TC / 4
  const int total = runs_per_col * 16 * NB;
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * TTM_THREADS) {
    f32x4 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + j * TTM_THREADS;
      const int c = e / runs_per_col, k0 = 4 * (e - c * runs_per_col);
      v[j] = (e < total && c < R && k0 < I) ? *reinterpret_cast<const gf32x4*>((const gfloat*)Q + k0 + (int64_t)I * c)
                                            : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + j * TTM_THREADS;
      const int c = e / runs_per_col, k0 = 4 * (e - c * runs_per_col);
      if (e < total) put(k0, c, v[j]);
    }
  }
}

__device__ __forceinline__ bool ttm_q_vec(const float* Q, int I) {
  return (I % 4) == 0 && (((uintptr_t)Q) & 15) == 0;
}

// ------------------------------------------------------------------ f32 MFMA
// LDS layout of Q for ttm_mc: for k-step t (4 k's), column block nb, lane:
// value Q[4t + lane/16][16 nb + lane%16]; four consecutive t are packed in a
// float4:  sq[(((t/4) * NB + nb) * 64 + lane) * 4 + t%4].
template <int NB>
__device__ void stage_q_mc(float* sq, const float* __restrict__ Q, int I, int R, int T4) {
  // T4 * NB elements per thread, gathered in batches of 16 independent loads
  const int n = T4 * NB;
  for (int b0 = 0; b0 < n; b0 += 16) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = (b0 + j) * TTM_THREADS + threadIdx.x;
      const int tt = e & 3;
      const int lane = (e >> 2) & 63;
      const int rest = e >> 8;               // (t4 * NB + nb)
      const int nb = rest % NB;
      const int t4 = rest / NB;
      const int k = (t4 * 4 + tt) * 4 + (lane >> 4);
      const int c = nb * 16 + (lane & 15);
      v[j] = (b0 + j < n && k < I && c < R) ? ((const gfloat*)Q)[k + (int64_t)I * c] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (b0 + j < n) sq[(b0 + j) * TTM_THREADS + threadIdx.x] = v[j];
  }
}

// Rows of an mc tile held by this lane: with VEC one float4 of rows
// m0 + 4i .. m0 + 4i + 3, else rows m0 + 16 v + i (v = 0..3).
template <bool VEC>
struct McRows {
  int64_t off[4];   // element offset of (row, k = 0)
  bool ok[4];
  __device__ __forceinline__ McRows(int64_t m0, int64_t M, int64_t L, int64_t LI, int li) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = VEC ? m0 + 4 * li : m0 + 16 * v + li;
      ok[v] = m < M;
      const int64_t s = m / L, l = m - s * L;
      off[v] = l + LI * s;
      if (VEC) break;
    }
  }
};

template <bool VEC, bool BUF>
__device__ __forceinline__ void mc_f32_load(f32x4 (&a)[8], const TtmSrc<BUF>& src,
                                            const McRows<VEC>& rows, int64_t L, int I, int q,
                                            int g) {
#pragma unroll
  for (int tt = 0; tt < 8; ++tt) {
    const int kb = 32 * q + 4 * tt;             // uniform part of k
    const bool kok = g < I - kb;
    if (VEC) {
      a[tt] = src.ld4(rows.off[0] + L * g, L * kb, rows.ok[0] && kok);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) a[tt][v] = src.ld1(rows.off[v] + L * g, L * kb, rows.ok[v] && kok);
    }
  }
}

template <int NB>
__device__ __forceinline__ void mc_f32_mma(f32x4 (&acc)[4 * NB], const f32x4 (&a)[8],
                                           const f32x4* sqv, int q, int lane) {
  f32x4 b[2][NB];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[hh][nb] = sqv[((2 * q + hh) * NB + nb) * 64 + lane];
#pragma unroll
  for (int tt = 0; tt < 8; ++tt)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[v * NB + nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[tt][v], b[tt >> 2][nb][tt & 3],
                                                                acc[v * NB + nb], 0, 0, 0);
}

// Store of an mc tile from the MFMA accumulator layout: lane holds rows
// rho = 4 g + jj of MFMA v, column 16 nb + li; with VEC row rho of MFMA v is
// m = m0 + 4 rho + v (four consecutive rows per (nb, jj): one 16-byte store).
template <int NB, bool VEC>
__device__ __forceinline__ void mc_store(const f32x4 (&acc)[4 * NB], float* __restrict__ out,
                                         int64_t m0, int64_t M, int64_t L, int R, int li, int g) {
  gfloat* __restrict__ gout = (gfloat*)out;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int c = 16 * nb + li;
    if (c >= R) continue;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      if (VEC) {
        const int64_t m = m0 + 16 * g + 4 * jj;
        if (m < M) {
          const int64_t s = m / L, l = m - s * L;
          f32x4 val = {acc[0 * NB + nb][jj], acc[1 * NB + nb][jj], acc[2 * NB + nb][jj], acc[3 * NB + nb][jj]};
          *reinterpret_cast<gf32x4*>(gout + l + L * (int64_t)c + L * (int64_t)R * s) = val;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = m0 + 16 * v + 4 * g + jj;
          if (m < M) {
            const int64_t s = m / L, l = m - s * L;
            gout[l + L * (int64_t)c + L * (int64_t)R * s] = acc[v * NB + nb][jj];
          }
        }
      }
    }
  }
}

template <int NB, bool VEC, bool BUF>
struct TtmMcF32 {
  static constexpr int NACC = 4 * NB;
  struct Buf { f32x4 a[8]; };
  struct Tile { McRows<VEC> rows; int64_t m0; };
  float* smem; const float* Q; float* out; TtmSrc<BUF> src;
  int64_t L, M, LI; int I, R, TC, lane, li, g;
  __device__ __forceinline__ TtmMcF32(float* sm, const float* in, const float* q, float* o, int64_t L_,
                                      int I_, int64_t S, int R_)
      : smem(sm), Q(q), out(o), src(in, L_ * S * I_), L(L_), M(L_ * S), LI(L_ * (int64_t)I_), I(I_),
        R(R_), TC((I_ + 31) / 32) {
    lane = threadIdx.x & 63; li = lane & 15; g = lane >> 4;
  }
  __device__ __forceinline__ Tile tile(int64_t t) const {
    const int64_t m0 = t * TTM_TILE;
    return Tile{McRows<VEC>(m0, M, L, LI, li), m0};
  }
  __device__ __forceinline__ void load(Buf& b, const Tile& t, int q) const {
    mc_f32_load<VEC, BUF>(b.a, src, t.rows, L, I, q, g);
  }
  __device__ __forceinline__ void mma(f32x4 (&acc)[NACC], const Buf& b, int q) const {
    mc_f32_mma<NB>(acc, b.a, reinterpret_cast<const f32x4*>(smem), q, lane);
  }
  __device__ __forceinline__ void store(const f32x4 (&acc)[NACC], const Tile& t) const {
    mc_store<NB, VEC>(acc, out, t.m0, M, L, R, li, g);
  }
  __device__ __forceinline__ void stage() const {
    if (ttm_q_vec(Q, I)) {
      // k = 16 t4 + 4 tt + g: a run k0..k0+3 shares (t4, tt) and spreads over g
      float* sq = smem;
      stage_q_runs<NB>(Q, I, R, TC, [sq](int k0, int c, f32x4 v) {
        const int m = k0 >> 2, t4 = m >> 2, tt = m & 3, nb = c >> 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) sq[(((t4 * NB + nb) * 64 + 16 * j + (c & 15)) << 2) + tt] = v[j];
      });
    } else {
      stage_q_mc<NB>(smem, Q, I, R, 2 * TC);
    }
  }
};

template <int NB, bool VEC, bool BUF>
TTM_KERNEL void ttm_mc_f32(TtmArgs a0, const TtmArgs* __restrict__ batch, int ks) {
  extern __shared__ float smem[];
  const TtmArgs a = kernel_args(a0, batch, blockIdx.y);
  const TtmMcF32<NB, VEC, BUF> p(smem, a.in, a.Q, a.out, a.L, a.I, a.S, a.R);
  ttm_drive(p, (a.L * a.S + TTM_TILE - 1) / TTM_TILE, p.TC, ks, smem + (size_t)p.TC * 32 * 16 * NB);
}

// LDS layout of Q for ttm_kc: k-step t covers 32 k; MFMA index v = 4h + cc
// maps to k = 32 t + 16 h + 4 (lane/16) + cc; lane%16 selects r in block nb.
// sq[((t * NB + nb) * 64 + lane) * 8 + v] = Q[k][16 nb + lane%16].
template <int NB>
__device__ void stage_q_kc(float* sq, const float* __restrict__ Q, int I, int R, int T) {
  // 2 T NB elements per thread, gathered in batches of 16 independent loads
  const int n = 2 * T * NB;
  for (int b0 = 0; b0 < n; b0 += 16) {
    float x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = (b0 + j) * TTM_THREADS + threadIdx.x;
      const int v = e & 7;
      const int lane = (e >> 3) & 63;
      const int rest = e >> 9;
      const int nb = rest % NB;
      const int t = rest / NB;
      const int k = 32 * t + 16 * (v >> 2) + 4 * (lane >> 4) + (v & 3);
      const int c = nb * 16 + (lane & 15);
      x[j] = (b0 + j < n && k < I && c < R) ? ((const gfloat*)Q)[k + (int64_t)I * c] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (b0 + j < n) sq[(b0 + j) * TTM_THREADS + threadIdx.x] = x[j];
  }
}

// Columns s of a kc tile held by this lane: s = s0 + 16 b + col (b = 0..3).
struct KcCols {
  int64_t off[4];   // element offset of (s, k = 4 g)
  bool ok[4];
  __device__ __forceinline__ KcCols(int64_t s0, int64_t S, int I, int col, int g) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t s = s0 + 16 * b + col;
      ok[b] = s < S;
      off[b] = s * (int64_t)I + 4 * g;
    }
  }
};

// Loads the 32 k of chunk t: x[b][h][cc] = in[s_b, 32 t + 16 h + 4 g + cc].
template <bool VEC, bool BUF>
__device__ __forceinline__ void kc_load(f32x4 (&x)[4][2], const TtmSrc<BUF>& src,
                                        const KcCols& cols, int I, int t, int g) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = 32 * t + 16 * h;
      if (VEC) {
        x[b][h] = src.ld4(cols.off[b], kb, cols.ok[b] && 4 * g < I - kb);
      } else {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc)
          x[b][h][cc] = src.ld1(cols.off[b] + cc, kb, cols.ok[b] && 4 * g + cc < I - kb);
      }
    }
}

template <int NB>
__device__ __forceinline__ void kc_f32_mma(f32x4 (&acc)[4 * NB], const f32x4 (&x)[4][2],
                                           const f32x4* sqv, int t, int lane) {
  f32x4 qa[NB][2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    qa[nb][0] = sqv[((t * NB + nb) * 64 + lane) * 2 + 0];
    qa[nb][1] = sqv[((t * NB + nb) * 64 + lane) * 2 + 1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[b * NB + nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[nb][h][cc], x[b][h][cc],
                                                                  acc[b * NB + nb], 0, 0, 0);
}

// Store of a kc tile: lane holds C[r = 16 nb + 4 g + jj][s = s0 + 16 b + col].
template <int NB>
__device__ __forceinline__ void kc_store(const f32x4 (&acc)[4 * NB], float* __restrict__ out,
                                         int64_t s0, int64_t S, int R, int col, int g) {
  gfloat* __restrict__ gout = (gfloat*)out;
  const bool vec_store = (R % 4) == 0 && (((uintptr_t)out) & 15) == 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t s = s0 + 16 * b + col;
    if (s >= S) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int r0 = 16 * nb + 4 * g;
      if (r0 >= R) continue;
      if (vec_store) {
        *reinterpret_cast<gf32x4*>(gout + r0 + (int64_t)R * s) = acc[b * NB + nb];
      } else {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (r0 + jj < R) gout[r0 + jj + (int64_t)R * s] = acc[b * NB + nb][jj];
      }
    }
  }
}

template <int NB, bool VEC, bool BUF>
struct TtmKcF32 {
  static constexpr int NACC = 4 * NB;
  struct Buf { f32x4 x[4][2]; };
  struct Tile { KcCols cols; int64_t s0; };
  float* smem; const float* Q; float* out; TtmSrc<BUF> src;
  int64_t S; int I, R, TC, lane, col, g;
  __device__ __forceinline__ TtmKcF32(float* sm, const float* in, const float* q, float* o, int I_,
                                      int64_t S_, int R_)
      : smem(sm), Q(q), out(o), src(in, S_ * I_), S(S_), I(I_), R(R_), TC((I_ + 31) / 32) {
    lane = threadIdx.x & 63; col = lane & 15; g = lane >> 4;
  }
  __device__ __forceinline__ Tile tile(int64_t t) const {
    const int64_t s0 = t * TTM_TILE;
    return Tile{KcCols(s0, S, I, col, g), s0};
  }
  __device__ __forceinline__ void load(Buf& b, const Tile& t, int q) const {
    kc_load<VEC, BUF>(b.x, src, t.cols, I, q, g);
  }
  __device__ __forceinline__ void mma(f32x4 (&acc)[NACC], const Buf& b, int q) const {
    kc_f32_mma<NB>(acc, b.x, reinterpret_cast<const f32x4*>(smem), q, lane);
  }
  __device__ __forceinline__ void store(const f32x4 (&acc)[NACC], const Tile& t) const {
    kc_store<NB>(acc, out, t.s0, S, R, col, g);
  }
  __device__ __forceinline__ void stage() const {
    if (ttm_q_vec(Q, I)) {
      // k = 32 t + 16 h + 4 (lane/16) + cc: a run k0..k0+3 is one float4 slot
      f32x4* sq4 = reinterpret_cast<f32x4*>(smem);
      stage_q_runs<NB>(Q, I, R, TC, [sq4](int k0, int c, f32x4 v) {
        const int m = k0 >> 2, t = m >> 3, h = (m >> 2) & 1, lg = m & 3, nb = c >> 4;
        sq4[((t * NB + nb) * 64 + 16 * lg + (c & 15)) * 2 + h] = v;
      });
    } else {
      stage_q_kc<NB>(smem, Q, I, R, TC);
    }
  }
};

template <int NB, bool VEC, bool BUF>
TTM_KERNEL void ttm_kc_f32(TtmArgs a0, const TtmArgs* __restrict__ batch, int ks) {
  extern __shared__ float smem[];
  const TtmArgs a = kernel_args(a0, batch, blockIdx.y);
  const TtmKcF32<NB, VEC, BUF> p(smem, a.in, a.Q, a.out, a.I, a.S, a.R);
  ttm_drive(p, (a.S + TTM_TILE - 1) / TTM_TILE, p.TC, ks, smem + (size_t)p.TC * 32 * 16 * NB);
}

// ------------------------------------------------------------- bf16x3 MFMA
// Q split into bf16 hi/lo in LDS in MFMA lane order.  For the mc layout the
// B operand of MFMA 16x16x32 holds Q[k][r] with r = 16 nb + lane%16 and
// k = 32 t + 8 (lane/16) + e (e = 0..7); for the kc layout the A operand
// holds Q[k][r] with k = 32 t + 16 (e/4) + 4 (lane/16) + e%4.
template <int NB, bool KC>
__device__ void stage_q_bf16(bf16x8* sq, const float* __restrict__ Q, int I, int R, int T) {
  // one item = 8 k of one (t, nb, lane); four items per batch
  const int total = T * NB * 64;
  const bool vq = ttm_q_vec(Q, I);
  for (int e0 = threadIdx.x; e0 < total; e0 += 4 * TTM_THREADS) {
    float x[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * TTM_THREADS;
      const int lane = e & 63;
      const int rest = e >> 6;
      const int nb = rest % NB;
      const int t = rest / NB;
      const int c = nb * 16 + (lane & 15);
      const bool ok = e < total && c < R;
      if (vq) {
        // two runs of 4 consecutive k: KC: 32t + 4g and 32t + 16 + 4g; else 32t + 8g and +4
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k0 = KC ? 32 * t + 16 * h + 4 * (lane >> 4) : 32 * t + 8 * (lane >> 4) + 4 * h;
          const f32x4 v = (ok && k0 < I) ? *reinterpret_cast<const gf32x4*>((const gfloat*)Q + k0 + (int64_t)I * c)
                                         : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int j = 0; j < 4; ++j) x[u][4 * h + j] = v[j];
        }
      } else {
#pragma unroll
        for (int ee = 0; ee < 8; ++ee) {
          const int k = KC ? (32 * t + 16 * (ee >> 2) + 4 * (lane >> 4) + (ee & 3))
                           : (32 * t + 8 * (lane >> 4) + ee);
          x[u][ee] = (ok && k < I) ? ((const gfloat*)Q)[k + (int64_t)I * c] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * TTM_THREADS;
      if (e >= total) continue;
      bf16x8 hi, lo;
#pragma unroll
      for (int ee = 0; ee < 8; ++ee) {
        __bf16 h, l;
        split_bf16(x[u][ee], h, l);
        hi[ee] = h;
        lo[ee] = l;
      }
      sq[2 * e] = hi;
      sq[2 * e + 1] = lo;
    }
  }
}

// A operand of the mc bf16 product: rows of the lane (as McRows), 8
// consecutive k = 32 t + 8 g + e.
template <bool VEC, bool BUF>
__device__ __forceinline__ void mc_bf16_load(f32x4 (&a)[8], const TtmSrc<BUF>& src,
                                             const McRows<VEC>& rows, int64_t L, int I, int t,
                                             int g) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int kb = 32 * t + e;
    const bool kok = 8 * g < I - kb;
    if (VEC) {
      a[e] = src.ld4(rows.off[0] + L * (8 * g), L * kb, rows.ok[0] && kok);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) a[e][v] = src.ld1(rows.off[v] + L * (8 * g), L * kb, rows.ok[v] && kok);
    }
  }
}

template <int NB>
__device__ __forceinline__ void mc_bf16_mma(f32x4 (&acc)[4 * NB], const f32x4 (&a)[8],
                                            const bf16x8* sq, int t, int lane) {
  bf16x8 qh[NB], ql[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    qh[nb] = sq[2 * ((t * NB + nb) * 64 + lane)];
    ql[nb] = sq[2 * ((t * NB + nb) * 64 + lane) + 1];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bf16x8 xh, xl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h, l;
      split_bf16(a[e][v], h, l);
      xh[e] = h;
      xl[e] = l;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      f32x4& c = acc[v * NB + nb];
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, qh[nb], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ql[nb], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, qh[nb], c, 0, 0, 0);
    }
  }
}

template <int NB, bool VEC, bool BUF>
struct TtmMcBf16 {
  static constexpr int NACC = 4 * NB;
  struct Buf { f32x4 a[8]; };
  struct Tile { McRows<VEC> rows; int64_t m0; };
  float* smem; const float* Q; float* out; TtmSrc<BUF> src;
  int64_t L, M, LI; int I, R, TC, lane, li, g;
  __device__ __forceinline__ TtmMcBf16(float* sm, const float* in, const float* q, float* o, int64_t L_,
                                       int I_, int64_t S, int R_)
      : smem(sm), Q(q), out(o), src(in, L_ * S * I_), L(L_), M(L_ * S), LI(L_ * (int64_t)I_), I(I_),
        R(R_), TC((I_ + 31) / 32) {
    lane = threadIdx.x & 63; li = lane & 15; g = lane >> 4;
  }
  __device__ __forceinline__ Tile tile(int64_t t) const {
    const int64_t m0 = t * TTM_TILE;
    return Tile{McRows<VEC>(m0, M, L, LI, li), m0};
  }
  __device__ __forceinline__ void load(Buf& b, const Tile& t, int q) const {
    mc_bf16_load<VEC, BUF>(b.a, src, t.rows, L, I, q, g);
  }
  __device__ __forceinline__ void mma(f32x4 (&acc)[NACC], const Buf& b, int q) const {
    mc_bf16_mma<NB>(acc, b.a, reinterpret_cast<const bf16x8*>(smem), q, lane);
  }
  // the bf16 A operand puts rows in the same places as the f32 one
  __device__ __forceinline__ void store(const f32x4 (&acc)[NACC], const Tile& t) const {
    mc_store<NB, VEC>(acc, out, t.m0, M, L, R, li, g);
  }
  __device__ __forceinline__ void stage() const {
    stage_q_bf16<NB, false>(reinterpret_cast<bf16x8*>(smem), Q, I, R, TC);
  }
};

template <int NB, bool VEC, bool BUF>
TTM_KERNEL void ttm_mc_bf16x3(TtmArgs a0, const TtmArgs* __restrict__ batch, int ks) {
  extern __shared__ float smem[];
  const TtmArgs a = kernel_args(a0, batch, blockIdx.y);
  const TtmMcBf16<NB, VEC, BUF> p(smem, a.in, a.Q, a.out, a.L, a.I, a.S, a.R);
  ttm_drive(p, (a.L * a.S + TTM_TILE - 1) / TTM_TILE, p.TC, ks, smem + (size_t)p.TC * 32 * 16 * NB);
}

template <int NB>
__device__ __forceinline__ void kc_bf16_mma(f32x4 (&acc)[4 * NB], const f32x4 (&x)[4][2],
                                            const bf16x8* sq, int t, int lane) {
  bf16x8 qh[NB], ql[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    qh[nb] = sq[2 * ((t * NB + nb) * 64 + lane)];
    ql[nb] = sq[2 * ((t * NB + nb) * 64 + lane) + 1];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    bf16x8 xh, xl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h, l;
      split_bf16(x[b][e >> 2][e & 3], h, l);
      xh[e] = h;
      xl[e] = l;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      f32x4& c = acc[b * NB + nb];
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ql[nb], xh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[nb], xl, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[nb], xh, c, 0, 0, 0);
    }
  }
}

template <int NB, bool VEC, bool BUF>
struct TtmKcBf16 {
  static constexpr int NACC = 4 * NB;
  struct Buf { f32x4 x[4][2]; };
  struct Tile { KcCols cols; int64_t s0; };
  float* smem; const float* Q; float* out; TtmSrc<BUF> src;
  int64_t S; int I, R, TC, lane, col, g;
  __device__ __forceinline__ TtmKcBf16(float* sm, const float* in, const float* q, float* o, int I_,
                                       int64_t S_, int R_)
      : smem(sm), Q(q), out(o), src(in, S_ * I_), S(S_), I(I_), R(R_), TC((I_ + 31) / 32) {
    lane = threadIdx.x & 63; col = lane & 15; g = lane >> 4;
  }
  __device__ __forceinline__ Tile tile(int64_t t) const {
    const int64_t s0 = t * TTM_TILE;
    return Tile{KcCols(s0, S, I, col, g), s0};
  }
  __device__ __forceinline__ void load(Buf& b, const Tile& t, int q) const {
    kc_load<VEC, BUF>(b.x, src, t.cols, I, q, g);
  }
  __device__ __forceinline__ void mma(f32x4 (&acc)[NACC], const Buf& b, int q) const {
    kc_bf16_mma<NB>(acc, b.x, reinterpret_cast<const bf16x8*>(smem), q, lane);
  }
  __device__ __forceinline__ void store(const f32x4 (&acc)[NACC], const Tile& t) const {
    kc_store<NB>(acc, out, t.s0, S, R, col, g);
  }
  __device__ __forceinline__ void stage() const {
    stage_q_bf16<NB, true>(reinterpret_cast<bf16x8*>(smem), Q, I, R, TC);
  }
};

template <int NB, bool VEC, bool BUF>
TTM_KERNEL void ttm_kc_bf16x3(TtmArgs a0, const TtmArgs* __restrict__ batch, int ks) {
  extern __shared__ float smem[];
  const TtmArgs a = kernel_args(a0, batch, blockIdx.y);
  const TtmKcBf16<NB, VEC, BUF> p(smem, a.in, a.Q, a.out, a.I, a.S, a.R);
  ttm_drive(p, (a.S + TTM_TILE - 1) / TTM_TILE, p.TC, ks, smem + (size_t)p.TC * 32 * 16 * NB);
}

// ------------------------------------------------------------ generic VALU
template <typename T>
__global__ __launch_bounds__(TTM_THREADS) void ttm_generic(
    const T* __restrict__ in, const T* __restrict__ Q, T* __restrict__ out,
    int64_t L, int I, int64_t S, int R) {
  // one thread per output element, rows m fastest across threads
  const int64_t M = L * S;
  const int64_t total = M * R;
  for (int64_t o = (int64_t)blockIdx.x * TTM_THREADS + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * TTM_THREADS) {
    const int64_t m = o % M;
    const int r = (int)(o / M);
    const int64_t s = m / L, l = m - s * L;
    const T* src = in + l + L * (int64_t)I * s;
    const T* q = Q + (int64_t)I * r;
    T acc = 0;
    for (int i = 0; i < I; ++i) acc += src[L * (int64_t)i] * q[i];
    out[l + L * (int64_t)r + L * (int64_t)R * s] = acc;
  }
}

// ---------------------------------------------------------------- launchers
static constexpr int TTM_WG_PER_CU = 2;          // persistent grid: workgroups per CU
static constexpr int64_t TTM_BUF_LIMIT = (int64_t)1 << 31;   // bytes addressable by a buffer offset

static int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// LDS of one gfx950 workgroup (160 KiB per CU, all of it available to one
// workgroup).  Q_m staged whole bounds the contracted mode size: up to 160 KiB
// the MFMA kernels run (one workgroup per CU above 80 KiB); K splits and the
// batched path keep within 64 KiB.
static constexpr size_t TTM_LDS_WG_MAX = 160 * 1024;
static size_t ttm_q_lds(int I, int NB) { return (size_t)((I + 31) / 32) * 32 * 16 * NB * 4; }
static size_t ttm_red_lds(int ks, int NB) {
  return ks > 1 ? (size_t)(ks - 1) * (4 / ks) * 64 * 16 * NB * 4 : 0;
}

// K split: the smallest KS whose tiles x KS reaches one wave per SIMD, as
// long as every part keeps at least two chunks and the LDS fits (measured on
// the 256^3 rank-32 shapes: one wave per SIMD with the whole K range beats
// two waves with half of it; tile-starved shapes gain from the split).
static int ttm_pick_ks(int64_t tiles, int I, int NB) {
  const int TC = (I + 31) / 32;
  const int64_t want = (int64_t)device_cu_count() * 4;
  int ks = 1;
  while (ks < 4 && tiles * ks < want && TC >= 4 * ks &&
         ttm_q_lds(I, NB) + ttm_red_lds(2 * ks, NB) <= 64 * 1024)
    ks *= 2;
  return ks;
}

// A full two-per-CU grid leaves no CU room for another kernel's workgroup
// (registers), so the Z QR that runs beside a TTM would wait for the whole
// TTM; the grid keeps TTM_RESERVE slots free for it.
static constexpr int TTM_RESERVE = 4;

static dim3 ttm_grid(int64_t tiles, int ks, int wpc) {
  const int tpw = 4 / ks;
  int64_t wgs = (tiles + tpw - 1) / tpw;
  const int w = wpc > 0 ? wpc : TTM_WG_PER_CU;
  const int64_t cap = (int64_t)device_cu_count() * w - (w >= 2 ? TTM_RESERVE : 0);
  if (wgs > cap) wgs = cap;
  return dim3((unsigned)(wgs > 0 ? wgs : 1));
}

// Launches through hipExtLaunchKernel when timing events are given, so that
// the events carry the kernel's own start and end times.
#define TTM_LAUNCH(KERNEL, ...)                                                          \
  do {                                                                                   \
    if (ev0) hipExtLaunchKernelGGL(KERNEL, grid, blk, lds, st, ev0, ev1, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(KERNEL, grid, blk, lds, st, __VA_ARGS__);                     \
  } while (0)

template <int NB, bool BUF>
static void launch_f32_kernel(bool kc, bool vec, bool bf16x3, dim3 grid, size_t lds, hipStream_t st,
                              const TtmArgs& a, const TtmArgs* batch, int ks, hipEvent_t ev0,
                              hipEvent_t ev1) {
  const dim3 blk(TTM_THREADS);
  if (kc) {
    if (bf16x3) {
      if (vec) TTM_LAUNCH((ttm_kc_bf16x3<NB, true, BUF>), a, batch, ks);
      else     TTM_LAUNCH((ttm_kc_bf16x3<NB, false, BUF>), a, batch, ks);
    } else {
      if (vec) TTM_LAUNCH((ttm_kc_f32<NB, true, BUF>), a, batch, ks);
      else     TTM_LAUNCH((ttm_kc_f32<NB, false, BUF>), a, batch, ks);
    }
  } else {
    if (bf16x3) {
      if (vec) TTM_LAUNCH((ttm_mc_bf16x3<NB, true, BUF>), a, batch, ks);
      else     TTM_LAUNCH((ttm_mc_bf16x3<NB, false, BUF>), a, batch, ks);
    } else {
      if (vec) TTM_LAUNCH((ttm_mc_f32<NB, true, BUF>), a, batch, ks);
      else     TTM_LAUNCH((ttm_mc_f32<NB, false, BUF>), a, batch, ks);
    }
  }
}

static hipError_t launch_f32_any(int NB, bool buf, bool kc, bool vec, bool bf16x3, dim3 grid, size_t lds,
                                 hipStream_t st, const TtmArgs& a, const TtmArgs* batch, int ks,
                                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
#define CPQR_TTM_NB(V)                                                                              \
  case V:                                                                                          \
    if (buf) launch_f32_kernel<V, true>(kc, vec, bf16x3, grid, lds, st, a, batch, ks, ev0, ev1);   \
    else     launch_f32_kernel<V, false>(kc, vec, bf16x3, grid, lds, st, a, batch, ks, ev0, ev1);  \
    break;
  switch (NB) {
    CPQR_TTM_NB(1)
    CPQR_TTM_NB(2)
    CPQR_TTM_NB(3)
    CPQR_TTM_NB(4)
    default: return hipErrorInvalidValue;
  }
#undef CPQR_TTM_NB
  return hipGetLastError();
}

static bool ttm_vec_ok(const TtmArgs& a) {
  if (a.L == 1) return (a.I % 4) == 0 && (((uintptr_t)a.in) & 15) == 0;
  return (a.L % 4) == 0 && (((uintptr_t)a.in) & 15) == 0 && (((uintptr_t)a.out) & 15) == 0;
}

bool ttm_vec_legal(const TtmArgs& a) { return ttm_vec_ok(a); }
bool ttm_buf_legal(const TtmArgs& a) { return a.L * (int64_t)a.I * a.S * 4 < TTM_BUF_LIMIT - 64; }

bool ttm_batch_shape(int64_t rows, int I, int R, int* ks, unsigned* wgs, size_t* lds, int wpc) {
  const int NB = (R + 15) / 16;
  const int64_t tiles = (rows + TTM_TILE - 1) / TTM_TILE;
  if (*ks <= 0) *ks = ttm_pick_ks(tiles, I, NB);
  if (*ks != 1 && *ks != 2 && *ks != 4) return false;
  *lds = ttm_q_lds(I, NB) + ttm_red_lds(*ks, NB);
  if (*lds > 64 * 1024 || (I + 31) / 32 < *ks) return false;
  *wgs = ttm_grid(tiles, *ks, wpc).x;
  return true;
}

hipError_t launch_ttm_f32_batched(const TtmBatch& b, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  return launch_f32_any(b.nb, b.buf, b.kc, b.vec, b.bf16x3, dim3(b.wgs, (unsigned)b.count), b.lds, st,
                        TtmArgs{}, b.args, b.ks);
}

bool ttm_mfma_supported(int I, int R) {
  if (R < 1 || R > 64 || I < 1) return false;
  const int NB = (R + 15) / 16;
  // Q staged in LDS: I (padded to 32) x 16 NB floats (or bf16 hi + lo pairs)
  return ttm_q_lds(I, NB) <= TTM_LDS_WG_MAX;
}

unsigned ttm_ks_options(int64_t L, int I, int64_t S, int R) {
  if (!ttm_mfma_supported(I, R) || L * S == 0) return 0;
  const int64_t rows = L == 1 ? S : L * S;
  unsigned m = 0;
  for (int b = 0; b < 3; ++b) {
    int ks = 1 << b;
    unsigned wgs;
    size_t lds;
    // every part of a split K range keeps at least two chunks of 32
    if ((I + 31) / 32 >= 2 * ks && ttm_batch_shape(rows, I, R, &ks, &wgs, &lds)) m |= 1u << b;
  }
  return m;
}

hipError_t launch_ttm_f32(const float* in, const float* Q, float* out, int64_t L, int I, int64_t S,
                          int R, bool bf16x3, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int ks_req,
                          int wpc) {
  if (L * S == 0) return hipSuccess;
  if (!ttm_mfma_supported(I, R)) {
    if (bf16x3) return hipErrorInvalidValue;
    const int64_t total = L * S * R;
    int64_t blocks = (total + TTM_THREADS - 1) / TTM_THREADS;
    if (blocks > 65536) blocks = 65536;
    const dim3 grid((unsigned)blocks), blk(TTM_THREADS);
    const size_t lds = 0;
    TTM_LAUNCH(ttm_generic<float>, in, Q, out, L, I, S, R);
    return hipGetLastError();
  }
  const TtmArgs a{in, Q, out, L, S, I, R};
  const int NB = (R + 15) / 16;
  const int64_t rows = L == 1 ? S : L * S;
  const int64_t tiles = (rows + TTM_TILE - 1) / TTM_TILE;
  int ks = ttm_pick_ks(tiles, I, NB);
  if (ks_req == 1 || ks_req == 2 || ks_req == 4) {
    int k = ks_req;
    unsigned wgs;
    size_t lds;
    if (ttm_batch_shape(rows, I, R, &k, &wgs, &lds)) ks = ks_req;
  }
  const bool buf = ttm_buf_legal(a);
  return launch_f32_any(NB, buf, L == 1, ttm_vec_ok(a), bf16x3, ttm_grid(tiles, ks, wpc),
                        ttm_q_lds(I, NB) + ttm_red_lds(ks, NB), st, a, nullptr, ks, ev0, ev1);
}

hipError_t launch_ttm_f64(const double* in, const double* Q, double* out, int64_t L, int I, int64_t S,
                          int R, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t total = L * S * R;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + TTM_THREADS - 1) / TTM_THREADS;
  if (blocks > 65536) blocks = 65536;
  const dim3 grid((unsigned)blocks), blk(TTM_THREADS);
  const size_t lds = 0;
  TTM_LAUNCH(ttm_generic<double>, in, Q, out, L, I, S, R);
  return hipGetLastError();
}

}  // namespace cpqr
