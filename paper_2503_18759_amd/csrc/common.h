// Shared device helpers for the gfx950 CP-ALS-QR kernels: vector types, MFMA
// operand types, wave-level reductions and error checking.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define CPQR_WAVE 64

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace cpqr {

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).  Used
// where register arrays are indexed by the loop variable, so that every index
// is a constant and the arrays stay in registers.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// Wave-level "transpose" reduction of V doubles (V a power of two, <= 32).
//
// On entry lane L holds a[0..V).  On exit a[0] of lane L holds the sum over
// all 64 lanes of value index  L / (64 / V).  Each halving step pairs lanes
// that differ in one lane-index bit: the lane with the bit set keeps the
// upper half of its values, the other the lower half, and both add the
// partner's copy of the half they keep.  Steps over bits 5 and 4 use the
// gfx950 cross-row swap instructions (v_permlane32_swap / v_permlane16_swap);
// the remaining bits use DPP lane permutations within rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void swap32_add(double& x, double& y) {
  // lanes 0-31 end with x(L) + x(L+32); lanes 32-63 with y(L-32) + y(L)
  unsigned xl = __double2loint(x), xh = __double2hiint(x);
  unsigned yl = __double2loint(y), yh = __double2hiint(y);
  auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
  auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
  double a = __hiloint2double((int)hi[0], (int)lo[0]);
  double b = __hiloint2double((int)hi[1], (int)lo[1]);
  x = a + b;
}

__device__ __forceinline__ void swap16_add(double& x, double& y) {
  // rows (16 lanes) 0 and 2 end with x summed over rows {0,1} / {2,3};
  // rows 1 and 3 with y summed likewise
  unsigned xl = __double2loint(x), xh = __double2hiint(x);
  unsigned yl = __double2loint(y), yh = __double2hiint(y);
  auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
  auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
  double a = __hiloint2double((int)hi[0], (int)lo[0]);
  double b = __hiloint2double((int)hi[1], (int)lo[1]);
  x = a + b;
}

// Value of `v` in the lane selected by the DPP control CTRL (row-local).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Device global memory (address space 1).  Accesses through these types
// compile to global rather than flat loads and stores; flat accesses also
// count against the LDS wait counter, so an LDS wait would stall on
// outstanding global stores.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) f32x4 gf32x4;
typedef __attribute__((address_space(1))) double gdouble;

// Kernel arguments that come either by value or from a per-problem device
// array (batched launches): the array entry is read by every lane and then
// passed through readfirstlane word by word, so that the compiler keeps every
// field in scalar registers (uniform pointers for buffer resources and
// scalar loop bounds) instead of treating the struct as per-lane data.
template <typename T>
__device__ __forceinline__ T kernel_args(const T& by_value, const T* batch, unsigned index) {
  static_assert(sizeof(T) % 4 == 0, "argument structs are made of 32-bit words");
  T v = batch ? batch[index] : by_value;
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}

// Value of `v` in lane `l` (wave-uniform), read into scalar registers.
__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, CPQR_WAVE);
}

template <int V>
__device__ __forceinline__ void wave_transpose_reduce(double (&a)[V]) {
  static_assert(V >= 1 && V <= 32 && (V & (V - 1)) == 0, "V must be a power of two <= 32");
  const int lane = threadIdx.x & 63;
  // bit 5: lanes 32-63 keep the upper half
  if constexpr (V >= 2) {
    static_for<0, V / 2>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      swap32_add(a[q], a[q + V / 2]);
    });
  } else {
    a[0] += shfl_xor_d(a[0], 32);
  }
  // bit 4
  if constexpr (V >= 4) {
    static_for<0, V / 4>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      swap16_add(a[q], a[q + V / 4]);
    });
  } else {
    a[0] += shfl_xor_d(a[0], 16);
  }
  // bits 3..0 within each row of 16 lanes, by DPP: the partner of lane i is
  // 15-i (row mirror), then 7-i within each half row (half mirror), then the
  // quad permutations i^2 and i^1.  Each partner differs from the lane in the
  // bit that decides which half is kept, which is all the reduction needs.
  static_for<0, 4>([&](auto bc) {
    constexpr int bit = 3 - decltype(bc)::value;
    constexpr int m = 1 << bit;
    constexpr int ctrl = (bit == 3) ? 0x140 : (bit == 2) ? 0x141 : (bit == 1) ? 0x4E : 0xB1;
    constexpr int half = V >> (6 - bit);   // values kept per lane after this step
    if constexpr (half >= 1) {
      const bool upper = (lane & m) != 0;
      static_for<0, half>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double keep = upper ? a[q + half] : a[q];
        const double send = upper ? a[q] : a[q + half];
        a[q] = keep + dpp_d<ctrl>(send);
      });
    } else {
      a[0] += dpp_d<ctrl>(a[0]);
    }
  });
}

// Copy of a wave-uniform integer held in a vector register, so that
// comparisons against it are lane-wise selects (v_cndmask) rather than
// scalar branches; used for masked access to register arrays.
__device__ __forceinline__ int to_vgpr(int x) {
  int v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

// Plain all-lanes sum of one double over the wave.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, CPQR_WAVE);
  return v;
}

// Relative rank test of a triangular factor's diagonal (or of a set of column
// norms) d(0..n-1): rank-deficient when some entry is at most kRankRel times
// the largest magnitude (zero included) or is not a number.  Dependent
// columns (duplicate initial columns, say) leave rounding-level diagonals,
// about 1e-16 of the largest, which a test for exact zeros misses; a ratio
// of 1e-13 is a condition number beyond what float64 resolves.
constexpr double kRankRel = 1e-13;

template <typename Get>
__device__ __forceinline__ bool rank_deficient(int n, Get&& d) {
  double mx = 0.0;
  for (int c = 0; c < n; ++c) mx = fmax(mx, fabs(d(c)));
  bool bad = false;
  for (int c = 0; c < n; ++c) bad = bad || !(fabs(d(c)) > kRankRel * mx);
  return bad;
}

// Largest value of `v` over the lanes of the wave.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, CPQR_WAVE));
  return v;
}

// rank_deficient evaluated by one wave: lane c < n passes d(c) in v (other
// lanes' v is ignored); the same answer on every lane.
__device__ __forceinline__ bool wave_rank_deficient(int n, double v) {
  const int lane = threadIdx.x & 63;
  const double a = (lane < n) ? fabs(v) : 0.0;
  const double mx = wave_max(a);
  const bool bad = (lane < n) && !(a > kRankRel * mx);
  return __ballot(bad) != 0;
}

// Round-to-nearest-even split of a float into bf16 hi + bf16 lo.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

}  // namespace cpqr
