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

// Sum over a whole wavefront (all 64 lanes end with the total).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
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

// Exponent e with 2^(e-1) <= |x| < 2^e (0 for x == 0 or non-finite); scaling by 2^-e is exact.
template <typename T>
__device__ __forceinline__ int pow2_exponent(T x) {
  if (!(x > T(0)) || !isfinite(x)) return 0;
  int e;
  (void)frexp(x, &e);
  return e;
}

}  // namespace tnmc
