// Mode-m tensor-times-matrix (TTM) kernels for gfx950.
//
// Section 2.1 defines Y = X x_m B with Y(..., j, ...) = sum_i X(..., i, ...) B(j, i).
// The chain of the QR-based ALS uses B = Q_m^T, so with the tensor viewed as
// [L, I, S] around mode m (L = product of the dims before m, S = product of
// the dims after m, mode 1 fastest):
//
//     out[l + L r + L R s] = sum_i in[l + L i + L I s] * Q[i + I r].
//
// For a fixed s this is a skinny GEMM (L x I) * (I x R).  The kernels stream
// the input once from HBM with 16-byte loads straight into MFMA operand
// registers, keep Q in LDS pre-arranged in MFMA lane order, split the
// reduction over I across the four waves of a workgroup and combine the four
// partial tiles through LDS before a coalesced store.
//
//  * ttm_mc: L > 1 ("M-contiguous": rows l are adjacent in memory).  A
//    workgroup owns 64 consecutive rows m = l + L s.  MFMA f32 16x16x4:
//    lane (i = lane%16, g = lane/16) feeds A[i][g]; with L % 4 == 0 each lane
//    loads a float4 of rows m0+4i..m0+4i+3 at column k and MFMA v uses
//    component v, so output row rho of MFMA v is m = m0 + 4 rho + v.
//    Otherwise each lane loads rows m0 + 16 v + i separately.
//  * ttm_kc: L == 1 ("K-contiguous": the contracted index is adjacent).  A
//    workgroup owns 64 consecutive s.  The product is computed transposed,
//    C[r][s] = sum_k Q[k][r] in[k + I s], so the 16-byte loads run along k
//    and the output (r fastest) is stored contiguously.
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

template <int NB, bool VEC>
__global__ __launch_bounds__(TTM_THREADS) void ttm_mc_f32(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int64_t L, int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int T4 = (I + 15) / 16;            // chunks of 16 k (4 MFMA k-steps)
  stage_q_mc<NB>(smem, Q, I, R, T4);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t M = L * S;
  const int64_t m0 = (int64_t)blockIdx.x * TTM_TILE;
  const int64_t LI = L * (int64_t)I;

  // per-lane row bases
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

  const f32x4* sqv = reinterpret_cast<const f32x4*>(smem);
  for (int q = wave; q < T4; q += 4) {
    // four k-steps: k = 16 q + 4 tt + g
    f32x4 a[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const int k = 16 * q + 4 * tt + g;
      if (VEC) {
        if (valid[0] && k < I)
          a[tt] = *reinterpret_cast<const f32x4*>(in + base[0] + L * (int64_t)k);
        else
          a[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          a[tt][v] = (valid[v] && k < I) ? in[base[v] + L * (int64_t)k] : 0.f;
      }
    }
    f32x4 b[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[nb] = sqv[(q * NB + nb) * 64 + lane];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[tt][v], b[nb][tt], acc[v][nb], 0, 0, 0);
  }

  // combine the four waves' partial tiles: red[w][lane][slot], slot = (v*NB+nb)*4+jj
  __syncthreads();
  constexpr int SLOTS = 16 * NB;
  float* red = smem;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        red[(wave * 64 + lane) * SLOTS + (v * NB + nb) * 4 + jj] = acc[v][nb][jj];
  __syncthreads();
  const int outs = TTM_TILE * R;
  for (int o = threadIdx.x; o < outs; o += TTM_THREADS) {
    const int ml = o & 63, c = o >> 6;
    const int64_t m = m0 + ml;
    if (m >= M) continue;
    int gg, jj, v;
    if (VEC) { gg = ml >> 4; jj = (ml >> 2) & 3; v = ml & 3; }
    else     { v = ml >> 4; gg = (ml & 15) >> 2; jj = ml & 3; }
    const int ln = (c & 15) + 16 * gg;
    const int slot = (v * NB + (c >> 4)) * 4 + jj;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red[(w * 64 + ln) * SLOTS + slot];
    const int64_t s = m / L, l = m - s * L;
    out[l + L * (int64_t)c + L * (int64_t)R * s] = sum;
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
__global__ __launch_bounds__(TTM_THREADS) void ttm_kc_f32(
    const float* __restrict__ in, const float* __restrict__ Q, float* __restrict__ out,
    int I, int64_t S, int R) {
  extern __shared__ float smem[];
  const int T = (I + 31) / 32;
  stage_q_kc<NB>(smem, Q, I, R, T);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * TTM_TILE;

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

  const f32x4* sqv = reinterpret_cast<const f32x4*>(smem);
  for (int t = wave; t < T; t += 4) {
    f32x4 x[4][2];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 32 * t + 16 * h + 4 * g;
        if (VEC) {
          if (valid[b] && k < I)
            x[b][h] = *reinterpret_cast<const f32x4*>(in + base[b] + k);
          else
            x[b][h] = f32x4{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
          for (int cc = 0; cc < 4; ++cc)
            x[b][h][cc] = (valid[b] && k + cc < I) ? in[base[b] + k + cc] : 0.f;
        }
      }
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
            acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[nb][h][cc], x[b][h][cc], acc[b][nb], 0, 0, 0);
  }

  __syncthreads();
  constexpr int SLOTS = 16 * NB;
  float* red = smem;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        red[(wave * 64 + lane) * SLOTS + (b * NB + nb) * 4 + jj] = acc[b][nb][jj];
  __syncthreads();
  const int outs = TTM_TILE * R;
  for (int o = threadIdx.x; o < outs; o += TTM_THREADS) {
    const int sl = o / R, r = o - sl * R;
    const int64_t s = s0 + sl;
    if (s >= S) continue;
    const int b = sl >> 4, cl = sl & 15;
    const int nb = r >> 4, gg = (r & 15) >> 2, jj = r & 3;
    const int ln = cl + 16 * gg;
    const int slot = (b * NB + nb) * 4 + jj;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red[(w * 64 + ln) * SLOTS + slot];
    out[(int64_t)R * s0 + o] = sum;
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
  const int64_t m0 = (int64_t)blockIdx.x * TTM_TILE;
  const int64_t LI = L * (int64_t)I;
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

  for (int t = wave; t < T; t += 4) {
    // A operand: rows (4 per lane), 8 consecutive k = 32 t + 8 g + e
    f32x4 a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * t + 8 * g + e;
      if (VEC) {
        if (valid[0] && k < I)
          a[e] = *reinterpret_cast<const f32x4*>(in + base[0] + L * (int64_t)k);
        else
          a[e] = f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          a[e][v] = (valid[v] && k < I) ? in[base[v] + L * (int64_t)k] : 0.f;
      }
    }
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
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, qh[nb], acc[v][nb], 0, 0, 0);
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ql[nb], acc[v][nb], 0, 0, 0);
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, qh[nb], acc[v][nb], 0, 0, 0);
      }
    }
  }

  __syncthreads();
  constexpr int SLOTS = 16 * NB;
  float* red = smem;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        red[(wave * 64 + lane) * SLOTS + (v * NB + nb) * 4 + jj] = acc[v][nb][jj];
  __syncthreads();
  const int outs = TTM_TILE * R;
  for (int o = threadIdx.x; o < outs; o += TTM_THREADS) {
    const int ml = o & 63, c = o >> 6;
    const int64_t m = m0 + ml;
    if (m >= M) continue;
    int gg, jj, v;
    if (VEC) { gg = ml >> 4; jj = (ml >> 2) & 3; v = ml & 3; }
    else     { v = ml >> 4; gg = (ml & 15) >> 2; jj = ml & 3; }
    const int ln = (c & 15) + 16 * gg;
    const int slot = (v * NB + (c >> 4)) * 4 + jj;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red[(w * 64 + ln) * SLOTS + slot];
    const int64_t s = m / L, l = m - s * L;
    out[l + L * (int64_t)c + L * (int64_t)R * s] = sum;
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
  const int64_t s0 = (int64_t)blockIdx.x * TTM_TILE;
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

  for (int t = wave; t < T; t += 4) {
    bf16x8 qh[NB], ql[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      qh[nb] = sq[2 * ((t * NB + nb) * 64 + lane)];
      ql[nb] = sq[2 * ((t * NB + nb) * 64 + lane) + 1];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f32x4 x[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 32 * t + 16 * h + 4 * g;
        if (VEC) {
          if (valid[b] && k < I)
            x[h] = *reinterpret_cast<const f32x4*>(in + base[b] + k);
          else
            x[h] = f32x4{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
          for (int cc = 0; cc < 4; ++cc)
            x[h][cc] = (valid[b] && k + cc < I) ? in[base[b] + k + cc] : 0.f;
        }
      }
      bf16x8 xh, xl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 h, l;
        split_bf16(x[e >> 2][e & 3], h, l);
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
  }

  __syncthreads();
  constexpr int SLOTS = 16 * NB;
  float* red = smem;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        red[(wave * 64 + lane) * SLOTS + (b * NB + nb) * 4 + jj] = acc[b][nb][jj];
  __syncthreads();
  const int outs = TTM_TILE * R;
  for (int o = threadIdx.x; o < outs; o += TTM_THREADS) {
    const int sl = o / R, r = o - sl * R;
    const int64_t s = s0 + sl;
    if (s >= S) continue;
    const int b = sl >> 4, cl = sl & 15;
    const int nb = r >> 4, gg = (r & 15) >> 2, jj = r & 3;
    const int ln = cl + 16 * gg;
    const int slot = (b * NB + nb) * 4 + jj;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red[(w * 64 + ln) * SLOTS + slot];
    out[(int64_t)R * s0 + o] = sum;
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
template <int NB>
static hipError_t launch_f32_nb(const float* in, const float* Q, float* out, int64_t L, int I,
                                int64_t S, int R, bool bf16x3, hipStream_t st) {
  if (L == 1) {
    const int T = (I + 31) / 32;
    size_t lds_q = bf16x3 ? (size_t)T * NB * 64 * 2 * sizeof(bf16x8) : (size_t)T * NB * 64 * 8 * 4;
    size_t lds_r = (size_t)4 * 64 * 16 * NB * 4;
    size_t lds = lds_q > lds_r ? lds_q : lds_r;
    dim3 grid((unsigned)((S + TTM_TILE - 1) / TTM_TILE));
    const bool vec = (I % 4) == 0 && (((uintptr_t)in) & 15) == 0;
    if (bf16x3) {
      if (vec) hipLaunchKernelGGL((ttm_kc_bf16x3<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
      else     hipLaunchKernelGGL((ttm_kc_bf16x3<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
    } else {
      if (vec) hipLaunchKernelGGL((ttm_kc_f32<NB, true>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
      else     hipLaunchKernelGGL((ttm_kc_f32<NB, false>), grid, dim3(TTM_THREADS), lds, st, in, Q, out, I, S, R);
    }
  } else {
    size_t lds_q;
    if (bf16x3) {
      const int T = (I + 31) / 32;
      lds_q = (size_t)T * NB * 64 * 2 * sizeof(bf16x8);
    } else {
      const int T4 = (I + 15) / 16;
      lds_q = (size_t)T4 * NB * 64 * 4 * 4;
    }
    size_t lds_r = (size_t)4 * 64 * 16 * NB * 4;
    size_t lds = lds_q > lds_r ? lds_q : lds_r;
    const int64_t M = L * S;
    dim3 grid((unsigned)((M + TTM_TILE - 1) / TTM_TILE));
    const bool vec = (L % 4) == 0 && (((uintptr_t)in) & 15) == 0;
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
