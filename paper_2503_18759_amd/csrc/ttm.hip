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
// The grid is persistent: every wave owns one 64-row output tile at a time and
// runs the whole reduction over I for it in registers (no cross-wave
// reduction, no barrier after the staging), with the loads of the next chunk
// of k issued before the MFMAs of the current one, and stores its tile
// directly from the accumulator layout with 16-byte stores.
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
#include "common.h"
#include "kernels.h"

namespace cpqr {

static constexpr int TTM_THREADS = 256;
static constexpr int TTM_TILE = 64;

// ------------------------------------------------------------------ f32 MFMA
// LDS layout of Q for ttm_mc: for k-step t (4 k's), column block nb, lane:
// value Q[4t + lane/16][16 nb + lane%16]; four consecutive t are packed in a
// float4:  sq[(((t/4) * NB + nb) * 64 + lane) * 4 + t%4].
template <int NB>
__device__ void stage_q_mc(float* sq, const float* __restrict__ Q, int I, int R, int T4) {
  const int total = T4 * NB * 64 * 4;
  for (int e = threadIdx.x; e < total; e += TTM_THREADS) {
    const int tt = e & 3;
    const int lane = (e >> 2) & 63;
    const int rest = e >> 8;               // (t4 * NB + nb)
    const int nb = rest % NB;
    const int t4 = rest / NB;
    const int k = (t4 * 4 + tt) * 4 + (lane >> 4);
    const int c = nb * 16 + (lane & 15);
    sq[e] = (k < I && c < R) ? Q[k + (int64_t)I * c] : 0.0f;
  }
}

// One wave owns a tile of 64 rows m at a time (persistent over tiles); the
// K loop runs over chunks of 32 k (8 MFMA k-steps) and is software pipelined
// one chunk ahead, so 8 float4 loads per lane are in flight while the MFMAs
// of the previous chunk issue.
template <bool VEC>
__device__ __forceinline__ void mc_f32_load(f32x4 (&a)[8], const float* __restrict__ in,
                                            const int64_t (&base)[4], const bool (&valid)[4],
                                            int64_t L, int I, int q, int g) {
#pragma unroll
  for (int tt = 0; tt < 8; ++tt) {
    const int k = 32 * q + 4 * tt + g;
    if (VEC) {
      a[tt] = (valid[0] && k < I) ? *reinterpret_cast<const f32x4*>(in + base[0] + L * (int64_t)k)
                                  : f32x4{0.f, 0.f, 0.f, 0.f};
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) a[tt][v] = (valid[v] && k < I) ? in[base[v] + L * (int64_t)k] : 0.f;
    }
  }
}

template <int NB, bool VEC>
__global__ __launch_bounds__(TTM_THREADS) void ttm_mc_f32(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int64_t L, int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int TC = (I + 31) / 32;            // chunks of 32 k (8 MFMA k-steps)
  stage_q_mc<NB>(smem, Q, I, R, 2 * TC);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t M = L * S;
  const int64_t LI = L * (int64_t)I;
  const int64_t ntiles = (M + TTM_TILE - 1) / TTM_TILE;
  const f32x4* sqv = reinterpret_cast<const f32x4*>(smem);
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t m0 = tile * TTM_TILE;
    int64_t base[4];
    bool valid[4];
    if (VEC) {
      const int64_t m = m0 + 4 * li;
      valid[0] = m < M;
      const int64_t s = m / L, l = m - s * L;
      base[0] = l + LI * s;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + 16 * v + li;
        valid[v] = m < M;
        const int64_t s = m / L, l = m - s * L;
        base[v] = l + LI * s;
      }
    }
    f32x4 acc[4][NB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[v][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 cur[8], nxt[8];
    mc_f32_load<VEC>(cur, in, base, valid, L, I, 0, g);
    for (int q = 0; q < TC; ++q) {
      if (q + 1 < TC) mc_f32_load<VEC>(nxt, in, base, valid, L, I, q + 1, g);
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
            acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[tt][v], b[tt >> 2][nb][tt & 3],
                                                              acc[v][nb], 0, 0, 0);
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) cur[tt] = nxt[tt];
    }
    // lane holds rows rho = 4 g + jj of MFMA v, column 16 nb + li
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = 16 * nb + li;
      if (c >= R) continue;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (VEC) {
          const int64_t m = m0 + 16 * g + 4 * jj;     // rows m..m+3 (v = 0..3)
          if (m < M) {
            const int64_t s = m / L, l = m - s * L;
            f32x4 val = {acc[0][nb][jj], acc[1][nb][jj], acc[2][nb][jj], acc[3][nb][jj]};
            *reinterpret_cast<f32x4*>(out + l + L * (int64_t)c + L * (int64_t)R * s) = val;
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + 16 * v + 4 * g + jj;
            if (m < M) {
              const int64_t s = m / L, l = m - s * L;
              out[l + L * (int64_t)c + L * (int64_t)R * s] = acc[v][nb][jj];
            }
          }
        }
      }
    }
  }
}

// LDS layout of Q for ttm_kc: k-step t covers 32 k; MFMA index v = 4h + cc
// maps to k = 32 t + 16 h + 4 (lane/16) + cc; lane%16 selects r in block nb.
// sq[((t * NB + nb) * 64 + lane) * 8 + v] = Q[k][16 nb + lane%16].
template <int NB>
__device__ void stage_q_kc(float* sq, const float* __restrict__ Q, int I, int R, int T) {
  const int total = T * NB * 64 * 8;
  for (int e = threadIdx.x; e < total; e += TTM_THREADS) {
    const int v = e & 7;
    const int lane = (e >> 3) & 63;
    const int rest = e >> 9;
    const int nb = rest % NB;
    const int t = rest / NB;
    const int k = 32 * t + 16 * (v >> 2) + 4 * (lane >> 4) + (v & 3);
    const int c = nb * 16 + (lane & 15);
    sq[e] = (k < I && c < R) ? Q[k + (int64_t)I * c] : 0.0f;
  }
}

template <int NB, bool VEC>
__device__ __forceinline__ void kc_f32_load(f32x4 (&x)[4][2], const float* __restrict__ in,
                                            const int64_t (&base)[4], const bool (&valid)[4],
                                            int I, int t, int g) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 32 * t + 16 * h + 4 * g;
      if (VEC) {
        x[b][h] = (valid[b] && k < I) ? *reinterpret_cast<const f32x4*>(in + base[b] + k)
                                      : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) x[b][h][cc] = (valid[b] && k + cc < I) ? in[base[b] + k + cc] : 0.f;
      }
    }
}

template <int NB, bool VEC>
__global__ __launch_bounds__(TTM_THREADS) void ttm_kc_f32(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int T = (I + 31) / 32;
  stage_q_kc<NB>(smem, Q, I, R, T);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const int64_t ntiles = (S + TTM_TILE - 1) / TTM_TILE;
  const f32x4* sqv = reinterpret_cast<const f32x4*>(smem);
  const bool vec_store = (R % 4) == 0 && (((uintptr_t)out) & 15) == 0;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t s0 = tile * TTM_TILE;
    int64_t base[4];
    bool valid[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t s = s0 + 16 * b + col;
      valid[b] = s < S;
      base[b] = s * (int64_t)I;
    }
    f32x4 acc[4][NB];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[b][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 cur[4][2], nxt[4][2];
    kc_f32_load<NB, VEC>(cur, in, base, valid, I, 0, g);
    for (int t = 0; t < T; ++t) {
      if (t + 1 < T) kc_f32_load<NB, VEC>(nxt, in, base, valid, I, t + 1, g);
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
              acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[nb][h][cc], cur[b][h][cc], acc[b][nb], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cur[b][0] = nxt[b][0];
        cur[b][1] = nxt[b][1];
      }
    }
    // lane holds C[r = 16 nb + 4 g + jj][s = s0 + 16 b + col]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t s = s0 + 16 * b + col;
      if (s >= S) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int r0 = 16 * nb + 4 * g;
        if (r0 >= R) continue;
        if (vec_store) {
          *reinterpret_cast<f32x4*>(out + r0 + (int64_t)R * s) = acc[b][nb];
        } else {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            if (r0 + jj < R) out[r0 + jj + (int64_t)R * s] = acc[b][nb][jj];
        }
      }
    }
  }
}

// ------------------------------------------------------------- bf16x3 MFMA
// Q split into bf16 hi/lo in LDS in MFMA lane order.  For the mc layout the
// B operand of MFMA 16x16x32 holds Q[k][r] with r = 16 nb + lane%16 and
// k = 32 t + 8 (lane/16) + e (e = 0..7); for the kc layout the A operand
// holds Q[k][r] with k = 32 t + 16 (e/4) + 4 (lane/16) + e%4.
template <int NB, bool KC>
__device__ void stage_q_bf16(bf16x8* sq, const float* __restrict__ Q, int I, int R, int T) {
  const int total = T * NB * 64;
  for (int e = threadIdx.x; e < total; e += TTM_THREADS) {
    const int lane = e & 63;
    const int rest = e >> 6;
    const int nb = rest % NB;
    const int t = rest / NB;
    const int c = nb * 16 + (lane & 15);
    bf16x8 hi, lo;
#pragma unroll
    for (int ee = 0; ee < 8; ++ee) {
      const int k = KC ? (32 * t + 16 * (ee >> 2) + 4 * (lane >> 4) + (ee & 3))
                       : (32 * t + 8 * (lane >> 4) + ee);
      const float x = (k < I && c < R) ? Q[k + (int64_t)I * c] : 0.0f;
      __bf16 h, l;
      split_bf16(x, h, l);
      hi[ee] = h;
      lo[ee] = l;
    }
    sq[2 * e] = hi;
    sq[2 * e + 1] = lo;
  }
}

template <bool VEC>
__device__ __forceinline__ void mc_bf16_load(f32x4 (&a)[8], const float* __restrict__ in,
                                             const int64_t (&base)[4], const bool (&valid)[4],
                                             int64_t L, int I, int t, int g) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 32 * t + 8 * g + e;
    if (VEC) {
      a[e] = (valid[0] && k < I) ? *reinterpret_cast<const f32x4*>(in + base[0] + L * (int64_t)k)
                                 : f32x4{0.f, 0.f, 0.f, 0.f};
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) a[e][v] = (valid[v] && k < I) ? in[base[v] + L * (int64_t)k] : 0.f;
    }
  }
}

template <int NB, bool VEC>
__global__ __launch_bounds__(TTM_THREADS) void ttm_mc_bf16x3(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int64_t L, int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int T = (I + 31) / 32;
  bf16x8* sq = reinterpret_cast<bf16x8*>(smem);
  stage_q_bf16<NB, false>(sq, Q, I, R, T);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t M = L * S;
  const int64_t LI = L * (int64_t)I;
  const int64_t ntiles = (M + TTM_TILE - 1) / TTM_TILE;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t m0 = tile * TTM_TILE;
    int64_t base[4];
    bool valid[4];
    if (VEC) {
      const int64_t m = m0 + 4 * li;
      valid[0] = m < M;
      const int64_t s = m / L, l = m - s * L;
      base[0] = l + LI * s;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + 16 * v + li;
        valid[v] = m < M;
        const int64_t s = m / L, l = m - s * L;
        base[v] = l + LI * s;
      }
    }
    f32x4 acc[4][NB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[v][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // A operand: rows (4 per lane), 8 consecutive k = 32 t + 8 g + e
    f32x4 cur[8], nxt[8];
    mc_bf16_load<VEC>(cur, in, base, valid, L, I, 0, g);
    for (int t = 0; t < T; ++t) {
      if (t + 1 < T) mc_bf16_load<VEC>(nxt, in, base, valid, L, I, t + 1, g);
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
          split_bf16(cur[e][v], h, l);
          xh[e] = h;
          xl[e] = l;
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, qh[nb], acc[v][nb], 0, 0, 0);
          acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ql[nb], acc[v][nb], 0, 0, 0);
          acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, qh[nb], acc[v][nb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) cur[e] = nxt[e];
    }
    // lane holds rows rho = 4 g + jj of MFMA v, column 16 nb + li; with VEC
    // row rho of MFMA v is m = m0 + 4 rho + v, else m = m0 + 16 v + rho
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
            f32x4 val = {acc[0][nb][jj], acc[1][nb][jj], acc[2][nb][jj], acc[3][nb][jj]};
            *reinterpret_cast<f32x4*>(out + l + L * (int64_t)c + L * (int64_t)R * s) = val;
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + 16 * v + 4 * g + jj;
            if (m < M) {
              const int64_t s = m / L, l = m - s * L;
              out[l + L * (int64_t)c + L * (int64_t)R * s] = acc[v][nb][jj];
            }
          }
        }
      }
    }
  }
}

template <bool VEC>
__device__ __forceinline__ void kc_bf16_load(f32x4 (&x)[4][2], const float* __restrict__ in,
                                             const int64_t (&base)[4], const bool (&valid)[4],
                                             int I, int t, int g) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 32 * t + 16 * h + 4 * g;
      if (VEC) {
        x[b][h] = (valid[b] && k < I) ? *reinterpret_cast<const f32x4*>(in + base[b] + k)
                                      : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) x[b][h][cc] = (valid[b] && k + cc < I) ? in[base[b] + k + cc] : 0.f;
      }
    }
}

template <int NB, bool VEC>
__global__ __launch_bounds__(TTM_THREADS) void ttm_kc_bf16x3(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int T = (I + 31) / 32;
  bf16x8* sq = reinterpret_cast<bf16x8*>(smem);
  stage_q_bf16<NB, true>(sq, Q, I, R, T);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const int64_t ntiles = (S + TTM_TILE - 1) / TTM_TILE;
  const bool vec_store = (R % 4) == 0 && (((uintptr_t)out) & 15) == 0;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t s0 = tile * TTM_TILE;
    int64_t base[4];
    bool valid[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t s = s0 + 16 * b + col;
      valid[b] = s < S;
      base[b] = s * (int64_t)I;
    }
    f32x4 acc[4][NB];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[b][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 cur[4][2], nxt[4][2];
    kc_bf16_load<VEC>(cur, in, base, valid, I, 0, g);
    for (int t = 0; t < T; ++t) {
      if (t + 1 < T) kc_bf16_load<VEC>(nxt, in, base, valid, I, t + 1, g);
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
          split_bf16(cur[b][e >> 2][e & 3], h, l);
          xh[e] = h;
          xl[e] = l;
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ql[nb], xh, acc[b][nb], 0, 0, 0);
          acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[nb], xl, acc[b][nb], 0, 0, 0);
          acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[nb], xh, acc[b][nb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cur[b][0] = nxt[b][0];
        cur[b][1] = nxt[b][1];
      }
    }
    // lane holds C[r = 16 nb + 4 g + jj][s = s0 + 16 b + col]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t s = s0 + 16 * b + col;
      if (s >= S) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int r0 = 16 * nb + 4 * g;
        if (r0 >= R) continue;
        if (vec_store) {
          *reinterpret_cast<f32x4*>(out + r0 + (int64_t)R * s) = acc[b][nb];
        } else {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            if (r0 + jj < R) out[r0 + jj + (int64_t)R * s] = acc[b][nb][jj];
        }
      }
    }
  }
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
// Persistent grid: four 64-row tiles per workgroup pass (one per wave),
// at most TTM_WG_PER_CU workgroups per compute unit.
static constexpr int TTM_WG_PER_CU = 2;

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

static dim3 ttm_grid(int64_t rows) {
  const int64_t tiles = (rows + TTM_TILE - 1) / TTM_TILE;
  int64_t wgs = (tiles + 3) / 4;
  const int64_t cap = (int64_t)device_cu_count() * TTM_WG_PER_CU;
  if (wgs > cap) wgs = cap;
  return dim3((unsigned)(wgs > 0 ? wgs : 1));
}

template <int NB>
static hipError_t launch_f32_nb(const float* in, const float* Q, float* out, int64_t L, int I,
                                int64_t S, int R, bool bf16x3, hipStream_t st) {
  // Q staged in LDS: I padded to 32, 16 NB columns, 4 bytes per entry
  // (float, or a bf16 hi/lo pair)
  const size_t lds = (size_t)((I + 31) / 32) * 32 * 16 * NB * 4;
  if (L == 1) {
    const dim3 grid = ttm_grid(S);
    const bool vec = (I % 4) == 0 && (((uintptr_t)in) & 15) == 0;
    if (bf16x3) {
      if (vec) hipLaunchKernelGGL((ttm_kc_bf16x3<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
      else     hipLaunchKernelGGL((ttm_kc_bf16x3<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
    } else {
      if (vec) hipLaunchKernelGGL((ttm_kc_f32<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
      else     hipLaunchKernelGGL((ttm_kc_f32<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
    }
  } else {
    const dim3 grid = ttm_grid(L * S);
    const bool vec = (L % 4) == 0 && (((uintptr_t)in) & 15) == 0 && (((uintptr_t)out) & 15) == 0;
    if (bf16x3) {
      if (vec) hipLaunchKernelGGL((ttm_mc_bf16x3<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, L, I, S, R);
      else     hipLaunchKernelGGL((ttm_mc_bf16x3<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, L, I, S, R);
    } else {
      if (vec) hipLaunchKernelGGL((ttm_mc_f32<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, L, I, S, R);
      else     hipLaunchKernelGGL((ttm_mc_f32<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, L, I, S, R);
    }
  }
  return hipGetLastError();
}

bool ttm_mfma_supported(int I, int R) {
  if (R < 1 || R > 64 || I < 1) return false;
  const int NB = (R + 15) / 16;
  // Q staged in LDS: I (padded to 32) x 16 NB floats (or bf16 hi + lo pairs)
  const size_t q_bytes = (size_t)((I + 31) / 32) * 32 * 16 * NB * 4;
  return q_bytes <= 64 * 1024;
}

hipError_t launch_ttm_f32(const float* in, const float* Q, float* out, int64_t L, int I, int64_t S,
                          int R, bool bf16x3, hipStream_t st) {
  if (L * S == 0) return hipSuccess;
  if (!ttm_mfma_supported(I, R)) {
    if (bf16x3) return hipErrorInvalidValue;
    const int64_t total = L * S * R;
    int64_t blocks = (total + TTM_THREADS - 1) / TTM_THREADS;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ttm_generic<float>, dim3((unsigned)blocks), dim3(TTM_THREADS), 0, st, in, Q, out, L, I, S, R);
    return hipGetLastError();
  }
  switch ((R + 15) / 16) {
    case 1: return launch_f32_nb<1>(in, Q, out, L, I, S, R, bf16x3, st);
    case 2: return launch_f32_nb<2>(in, Q, out, L, I, S, R, bf16x3, st);
    case 3: return launch_f32_nb<3>(in, Q, out, L, I, S, R, bf16x3, st);
    default: return launch_f32_nb<4>(in, Q, out, L, I, S, R, bf16x3, st);
  }
}

hipError_t launch_ttm_f64(const double* in, const double* Q, double* out, int64_t L, int I, int64_t S,
                          int R, hipStream_t st) {
  const int64_t total = L * S * R;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + TTM_THREADS - 1) / TTM_THREADS;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(ttm_generic<double>, dim3((unsigned)blocks), dim3(TTM_THREADS), 0, st, in, Q, out, L, I, S, R);
  return hipGetLastError();
}

}  // namespace cpqr
