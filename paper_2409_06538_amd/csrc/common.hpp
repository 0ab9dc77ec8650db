// Device helpers shared by the TNMC kernels: Philox4x64-10 draws, bit-packed rows, block
// reductions and power-of-two rescaling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tnmc.h"

namespace tnmc {

constexpr int WAVE = 64;

__host__ __device__ constexpr int words_per_row(int L) { return (L + 63) / 64; }

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64 -> 128-bit
// multiplications with the published multipliers, key bumped by the published Weyl constants.
struct Philox4 {
  uint64_t w[4];
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                  uint64_t c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// 53 random bits -> [0, 1).
__device__ __forceinline__ double u53(uint64_t w) {
  return static_cast<double>(w >> 11) * 0x1.0p-53;
}

// Draw i of the stream keyed (k0, k1) with counter words (c1, c2, c3).
__device__ __forceinline__ double philox_uniform(uint64_t k0, uint64_t k1, uint64_t i, uint64_t c1,
                                                 uint64_t c2, uint64_t c3) {
  const Philox4 b = philox4x64_10(i >> 2, c1, c2, c3, k0, k1);
  return u53(b.w[i & 3]);
}

enum : uint64_t { STREAM_COUPLINGS = 0, STREAM_PROPOSAL = 1, STREAM_ACCEPT = 2 };

// Cross-lane moves within a row of 16 lanes (DPP).  Controls: quad_perm [1,0,3,2] = 0xB1,
// quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141, row_mirror = 0x140.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>(int(b & 0xffffffffll));
  const int hi = dpp_i<CTRL>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return dpp_i<CTRL>(v);
}

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float readlane_v(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_v(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ int readlane_v(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of a group gets the
// group's sum.  All lanes of a group must be active.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if (G >= 2) v += dpp<0xB1>(v);
  if (G >= 4) v += dpp<0x4E>(v);
  if (G >= 8) v += dpp<0x141>(v);
  if (G >= 16) v += dpp<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16);
  if (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Workgroup barrier that orders LDS accesses only: global loads and stores stay in flight across
// it (their consumers wait for them through the registers they fill).  For kernels whose threads
// exchange data through LDS alone.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// lds_sync() that also returns the OR of `pred` over the workgroup (NW wavefronts).  `flags`
// holds 2 NW ints of LDS; `par` alternates between calls, so that a wavefront running ahead to
// the next call cannot overwrite flags that a slower one still reads.
template <int NW>
__device__ __forceinline__ bool lds_sync_or(bool pred, int* flags, int& par) {
  const bool any = __ballot(pred) != 0ull;
  if ((threadIdx.x & 63) == 0) flags[par * NW + (threadIdx.x >> 6)] = any ? 1 : 0;
  lds_sync();
  int r = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) r |= flags[par * NW + i];
  par ^= 1;
  return r != 0;
}

// Unsigned maximum over aligned groups of G lanes (G = 16 or 32); every lane of a group gets it.
template <int G>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t v) {
  auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  v = mx(v, uint32_t(dpp<0xB1>(int(v))));
  v = mx(v, uint32_t(dpp<0x4E>(int(v))));
  v = mx(v, uint32_t(dpp<0x141>(int(v))));
  v = mx(v, uint32_t(dpp<0x140>(int(v))));
  if (G >= 32) v = mx(v, uint32_t(__shfl_xor(int(v), 16)));
  return v;
}

// Sum / max over a whole wavefront (all 64 lanes active); every lane gets the result.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v = group_sum<16>(v);
  return (readlane_v(v, 0) + readlane_v(v, 16)) + (readlane_v(v, 32) + readlane_v(v, 48));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  v = fmax(v, dpp<0xB1>(v));
  v = fmax(v, dpp<0x4E>(v));
  v = fmax(v, dpp<0x141>(v));
  v = fmax(v, dpp<0x140>(v));
  return fmax(fmax(readlane_v(v, 0), readlane_v(v, 16)), fmax(readlane_v(v, 32), readlane_v(v, 48)));
}

// Arg-max over a whole wavefront (ties -> smaller index); every lane gets (value, index).
template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
#define TNMC_ARGMAX_STEP(CTRL)                                       \
  {                                                                  \
    const T ov = dpp<CTRL>(v);                                       \
    const int oi = dpp<CTRL>(i);                                     \
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }           \
  }
  TNMC_ARGMAX_STEP(0xB1)
  TNMC_ARGMAX_STEP(0x4E)
  TNMC_ARGMAX_STEP(0x141)
  TNMC_ARGMAX_STEP(0x140)
#undef TNMC_ARGMAX_STEP
  T bv = readlane_v(v, 0);
  int bi = readlane_v(i, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const T ov = readlane_v(v, 16 * r);
    const int oi = readlane_v(i, 16 * r);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  v = bv;
  i = bi;
}

// Unsigned maximum over a whole wavefront; every lane gets the result.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  v = mx(v, uint32_t(dpp<0xB1>(int(v))));
  v = mx(v, uint32_t(dpp<0x4E>(int(v))));
  v = mx(v, uint32_t(dpp<0x141>(int(v))));
  v = mx(v, uint32_t(dpp<0x140>(int(v))));
  return mx(mx(uint32_t(readlane_i(int(v), 0)), uint32_t(readlane_i(int(v), 16))),
            mx(uint32_t(readlane_i(int(v), 32)), uint32_t(readlane_i(int(v), 48))));
}

// Block-wide sum for NT threads (NT a multiple of 64); `red` holds NT/64 entries of LDS.
// Contains the barriers it needs; every thread returns the total.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) s += red[i];
  return s;
}

template <int NT, typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
  v = wave_max(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < NT / WAVE; ++i) s = fmax(s, red[i]);
  return s;
}

// Global-memory pointers.  A pointer read from memory (the realization table) is generic, and the
// compiler then emits FLAT loads and stores, which count against the LDS wait counter as well: an
// LDS wait would also wait for every outstanding global load or store, so a prefetch issued early
// would stall the next LDS access.  Casting to the global address space gives global_load /
// global_store, which count against the vector-memory counter only.
template <typename T>
using gmem = T __attribute__((address_space(1)));
template <typename T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
  return (gmem<T>*)p;
}

// Environment storage types.  bfloat16 is the upper half of an IEEE binary32; narrowing rounds to
// nearest, ties to even (NaN stays NaN).  Arithmetic always runs in the wider compute type.
struct bf16_t {
  uint16_t bits;
};

// element loads and stores through global pointers (bfloat16 moves its 16 bits)
template <typename E>
__device__ __forceinline__ E gld(const gmem<E>* p, size_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ bf16_t gld<bf16_t>(const gmem<bf16_t>* p, size_t i) {
  return bf16_t{p[i].bits};
}
template <typename E>
__device__ __forceinline__ void gst(gmem<E>* p, size_t i, E v) {
  p[i] = v;
}
template <>
__device__ __forceinline__ void gst<bf16_t>(gmem<bf16_t>* p, size_t i, bf16_t v) {
  p[i].bits = v.bits;
}

__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(bf16_t v) { return __uint_as_float(uint32_t(v.bits) << 16); }

template <typename E>
struct Narrow;
template <>
struct Narrow<double> {
  __device__ __forceinline__ static double from(double v) { return v; }
};
template <>
struct Narrow<float> {
  __device__ __forceinline__ static float from(float v) { return v; }
};
template <>
struct Narrow<bf16_t> {
  __device__ __forceinline__ static bf16_t from(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t{uint16_t((u >> 16) | 0x40u)};
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t{uint16_t(u >> 16)};
  }
};
template <typename E, typename T>
__device__ __forceinline__ E narrow(T v) {
  return Narrow<E>::from(v);
}

// Reciprocal: the hardware estimate (FP32: about 1 ulp; FP64: refined by two Newton steps to
// a few ulp), for scale factors where a correctly rounded quotient is not needed.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  return r * (2.0 - x * r);
}

// Exponent e with 2^(e-1) <= |x| < 2^e (0 for x == 0 or non-finite); scaling by 2^-e is exact.
template <typename T>
__device__ __forceinline__ int pow2_exponent(T x) {
  if (!(x > T(0)) || !isfinite(x)) return 0;
  int e;
  (void)frexp(x, &e);
  return e;
}

}  // namespace tnmc
