// Couplings (Sec. III A), exact energies (Eq. (10)), the independence Metropolis chain (Eq. (3)
// with g(s'|s) = q(s'); Appendix A) and the observables of Sec. III C.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace tnmc {

// ---------------------------------------------------------------------------------------------
// Couplings: bond k antiferromagnetic iff u_k < p, u_k = draw k of the stream (seed, 0); the
// L(L-1) horizontal bonds (k = r(L-1) + c) precede the vertical bonds (k = L(L-1) + rL + c).
// One thread writes one 64-bit word of Jh or Jv.
__global__ void couplings_kernel(const DevReal* reals, const uint64_t* seeds, double p, int Lmax) {
  const int ri = blockIdx.y;
  const DevReal R = reals[ri];
  const int L = R.L, W = words_per_row(L);
  const int words = (2 * L - 1) * W;   // L rows of Jh then L-1 rows of Jv
  const uint64_t seed = seeds[ri];
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < words; o += gridDim.x * blockDim.x) {
    const int row = o / W, w = o % W;
    const bool horiz = row < L;
    const int r = horiz ? row : row - L;
    const int ncol = horiz ? L - 1 : L;
    uint64_t bits = 0;
    uint64_t cached = ~0ull;
    Philox4 blk{};
    for (int b = 0; b < 64; ++b) {
      const int c = w * 64 + b;
      if (c >= ncol) break;
      const uint64_t k = horiz ? uint64_t(r) * (L - 1) + c
                               : uint64_t(L) * (L - 1) + uint64_t(r) * L + c;
      if ((k >> 2) != cached) {
        blk = philox4x64_10(k >> 2, 0, 0, 0, seed, STREAM_COUPLINGS);
        cached = k >> 2;
      }
      const int q = int(k & 3);
      const uint64_t wd = q == 0 ? blk.w[0] : q == 1 ? blk.w[1] : q == 2 ? blk.w[2] : blk.w[3];
      if (u53(wd) < p) bits |= (1ull << b);
    }
    uint64_t* dst = horiz ? const_cast<uint64_t*>(R.Jh) + size_t(r) * W
                          : const_cast<uint64_t*>(R.Jv) + size_t(r) * W;
    dst[w] = bits;
  }
}

hipError_t couplings_launch(const DevReal* d_reals, int n, const uint64_t* d_seeds, double p,
                            int Lmax, hipStream_t stream) {
  const int W = words_per_row(Lmax);
  const int words = (2 * Lmax - 1) * W;
  dim3 grid((words + 255) / 256, n);
  hipLaunchKernelGGL(couplings_kernel, grid, dim3(256), 0, stream, d_reals, d_seeds, p, Lmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Energy E = 2U - N_B from bit-packed spins, U = number of unsatisfied bonds, i.e. bonds with
// bit(J) xor bit(s_i) xor bit(s_j) = 1.  One wavefront per configuration.
__device__ __forceinline__ int unsat_rows(const uint64_t* s, const uint64_t* jh, const uint64_t* jv,
                                          int L, int Wmax, int lane) {
  const int W = words_per_row(L);
  int u = 0;
  for (int o = lane; o < L * W; o += WAVE) {
    const int r = o / W, w = o % W;
    const uint64_t cw = s[size_t(r) * Wmax + w];
    const uint64_t nxt = (w + 1 < W) ? s[size_t(r) * Wmax + w + 1] : 0ull;
    const uint64_t right = (cw >> 1) | (nxt << 63);
    const int nb_h = (L - 1) - 64 * w;
    const uint64_t mh = nb_h >= 64 ? ~0ull : (nb_h > 0 ? ((1ull << nb_h) - 1) : 0ull);
    u += __popcll((cw ^ right ^ jh[size_t(r) * W + w]) & mh);
    if (r + 1 < L) {
      const int nb_v = L - 64 * w;
      const uint64_t mv = nb_v >= 64 ? ~0ull : ((1ull << nb_v) - 1);
      u += __popcll((cw ^ s[size_t(r + 1) * Wmax + w] ^ jv[size_t(r) * W + w]) & mv);
    }
  }
  return u;
}

__global__ void energy_kernel(const DevReal* reals, int n, int K, int Lmax, const uint64_t* spins,
                              int32_t* E) {
  const int lane = threadIdx.x % WAVE;
  const long cfg = long(blockIdx.x) * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (cfg >= long(n) * K) return;
  const int ri = int(cfg / K);
  const DevReal R = reals[ri];
  const int Wmax = words_per_row(Lmax);
  const uint64_t* s = spins + size_t(cfg) * Lmax * Wmax;
  int u = unsat_rows(s, R.Jh, R.Jv, R.L, Wmax, lane);
  u = wave_sum(u);
  if (lane == 0) E[cfg] = 2 * u - 2 * R.L * (R.L - 1);
}

hipError_t energy_launch(const DevReal* d_reals, int n, int K, int Lmax, const uint64_t* d_spins,
                         int32_t* d_E, hipStream_t stream) {
  const long cfgs = long(n) * K;
  const int per = 4;   // configurations per workgroup of 256 threads
  hipLaunchKernelGGL(energy_kernel, dim3(unsigned((cfgs + per - 1) / per)), dim3(per * WAVE), 0,
                     stream, d_reals, n, K, Lmax, d_spins, d_E);
  return hipGetLastError();
}

// Field part of the energy, -sum h s over the sites of a realization with fields: one wavefront
// per configuration (realization slot, proposal), lanes over the columns of each row.
__global__ void field_energy_kernel(const DevReal* reals, int K, int Lmax, const uint64_t* spins,
                                    int32_t* E) {
  const DevReal R = reals[blockIdx.y];
  if (R.field == nullptr) return;
  const int lane = threadIdx.x % WAVE;
  const int k = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (k >= K) return;
  const int L = R.L, Wmax = words_per_row(Lmax);
  const size_t cfg = size_t(R.slot) * K + k;
  const uint64_t* s = spins + cfg * Lmax * Wmax;
  int acc = 0;
  for (int r = 0; r < L; ++r)
    for (int c = lane; c < L; c += WAVE) {
      const int h = R.field[size_t(r) * L + c];
      const bool neg = (s[size_t(r) * Wmax + (c >> 6)] >> (c & 63)) & 1ull;
      acc += neg ? h : -h;   // -h s
    }
  acc = wave_sum(acc);
  if (lane == 0) E[cfg] += acc;
}

hipError_t field_energy_launch(const DevReal* d_reals, int n, int K, int Lmax,
                               const uint64_t* d_spins, int32_t* d_E, hipStream_t stream) {
  const int per = 4;   // configurations per workgroup of 256 threads
  hipLaunchKernelGGL(field_energy_kernel, dim3(unsigned((K + per - 1) / per), n), dim3(per * WAVE),
                     0, stream, d_reals, K, Lmax, d_spins, d_E);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Periodic lattices by a frozen line pair (Sec. IV).  Block site (a, b) is torus site
// (R(a), C(b)) = ((r0 + 1 + a) mod L, (c0 + 1 + b) mod L); block bonds are the torus bonds between
// block sites, and a block site's field is the sum of J s_f over its frozen neighbours f.
__device__ __forceinline__ int tbit(const uint64_t* row, int c) { return int((row[c >> 6] >> (c & 63)) & 1ull); }

// One workgroup per (torus, block row a); one 64-bit word (or one site of the fields) per thread.
__global__ void __launch_bounds__(64) pbc_block_kernel(const DevTorus* tor, const DevReal* blk,
                                                        int Lmax, uint64_t* bspins) {
  const DevTorus T = tor[blockIdx.y];
  const DevReal B = blk[blockIdx.y];
  const int L = T.L, Lb = L - 1, a = blockIdx.x;
  const int W = words_per_row(L), Wb = words_per_row(Lb), Wmax = words_per_row(Lmax);
  uint64_t* so = bspins + size_t(blockIdx.y) * Lmax * Wmax + size_t(a) * Wmax;
  if (a >= Lb) {   // rows past this block's side: zero
    for (int w = threadIdx.x; w < Wmax; w += blockDim.x) so[w] = 0ull;
    return;
  }
  const int r = (T.r0 + 1 + a) % L, rup = (r + L - 1) % L, rdn = (r + 1) % L;
  const uint64_t* jh = T.Jh + size_t(r) * W;
  const uint64_t* jv = T.Jv + size_t(r) * W;
  const uint64_t* jvup = T.Jv + size_t(rup) * W;
  const uint64_t* st = T.spins + size_t(r) * W;
  const uint64_t* stup = T.spins + size_t(rup) * W;
  const uint64_t* stdn = T.spins + size_t(rdn) * W;
  uint64_t* bjh = const_cast<uint64_t*>(B.Jh) + size_t(a) * Wb;
  uint64_t* bjv = const_cast<uint64_t*>(B.Jv) + size_t(a) * Wb;
  for (int w = threadIdx.x; w < Wmax; w += blockDim.x) {
    uint64_t wh = 0, wv = 0, ws = 0;
    for (int u = 0; u < 64; ++u) {
      const int b = 64 * w + u;
      if (b >= Lb) break;
      const int c = (T.c0 + 1 + b) % L;
      ws |= uint64_t(tbit(st, c)) << u;
      if (b + 1 < Lb) wh |= uint64_t(tbit(jh, c)) << u;
      if (a + 1 < Lb) wv |= uint64_t(tbit(jv, c)) << u;
    }
    so[w] = ws;
    if (w < Wb) {
      bjh[w] = wh;
      if (a + 1 < Lb) bjv[w] = wv;
    }
  }
  // J s_f = +1 iff the bits of J and s_f agree
  auto js = [](int bj, int bs) { return (bj ^ bs) ? -1 : 1; };
  for (int b = threadIdx.x; b < Lb; b += blockDim.x) {
    const int c = (T.c0 + 1 + b) % L, cl = (c + L - 1) % L, cr = (c + 1) % L;
    int h = 0;
    if (rup == T.r0) h += js(tbit(jvup, c), tbit(stup, c));     // above
    if (rdn == T.r0) h += js(tbit(jv, c), tbit(stdn, c));       // below
    if (cl == T.c0) h += js(tbit(jh, cl), tbit(st, cl));        // left
    if (cr == T.c0) h += js(tbit(jh, c), tbit(st, cr));         // right
    const_cast<int8_t*>(B.field)[size_t(a) * Lb + b] = int8_t(h);
  }
}

hipError_t pbc_block_launch(const DevTorus* d_tor, const DevReal* d_blk, int n, int Lmax,
                            uint64_t* d_block_spins, hipStream_t stream) {
  hipLaunchKernelGGL(pbc_block_kernel, dim3(Lmax, n), dim3(64), 0, stream, d_tor, d_blk, Lmax,
                     d_block_spins);
  return hipGetLastError();
}

// Block configuration back into the torus: one workgroup per (torus, block row), one torus word
// per thread (the frozen column's bit kept).
__global__ void __launch_bounds__(64) pbc_merge_kernel(const DevTorus* tor, int Lmax,
                                                       const uint64_t* bspins) {
  const DevTorus T = tor[blockIdx.y];
  const int L = T.L, Lb = L - 1, a = blockIdx.x;
  if (a >= Lb) return;
  const int W = words_per_row(L), Wmax = words_per_row(Lmax);
  const uint64_t* sb = bspins + size_t(blockIdx.y) * Lmax * Wmax + size_t(a) * Wmax;
  const int r = (T.r0 + 1 + a) % L;
  uint64_t* st = T.spins + size_t(r) * W;
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    uint64_t word = st[w];
    for (int u = 0; u < 64; ++u) {
      const int c = 64 * w + u;
      if (c >= L) break;
      if (c == T.c0) continue;
      const int b = (c - T.c0 - 1 + L) % L;
      word = (word & ~(1ull << u)) | (uint64_t(tbit(sb, b)) << u);
    }
    st[w] = word;
  }
}

// Torus energy E = 2U - 2L^2: one wavefront per torus, lanes over (row, word).
__global__ void __launch_bounds__(64) torus_energy_kernel(const DevTorus* tor, int32_t* E) {
  const DevTorus T = tor[blockIdx.x];
  const int L = T.L, W = words_per_row(L), lane = threadIdx.x;
  int u = 0;
  for (int o = lane; o < L * W; o += WAVE) {
    const int r = o / W, w = o % W;
    const uint64_t* sr = T.spins + size_t(r) * W;
    const uint64_t cw = sr[w];
    // right neighbour of column c is (c + 1) mod L
    uint64_t right = (cw >> 1) | ((w + 1 < W ? sr[w + 1] : 0ull) << 63);
    const int last = L - 1;
    if ((last >> 6) == w) right = (right & ~(1ull << (last & 63))) | (uint64_t(sr[0] & 1ull) << (last & 63));
    const int nb = L - 64 * w;
    const uint64_t m = nb >= 64 ? ~0ull : ((1ull << nb) - 1);
    u += __popcll((cw ^ right ^ T.Jh[size_t(r) * W + w]) & m);
    u += __popcll((cw ^ T.spins[size_t((r + 1) % L) * W + w] ^ T.Jv[size_t(r) * W + w]) & m);
  }
  u = wave_sum(u);
  if (lane == 0) E[blockIdx.x] = 2 * u - 2 * L * L;
}

hipError_t pbc_merge_launch(const DevTorus* d_tor, int n, int Lmax, const uint64_t* d_block_spins,
                            int32_t* d_E_torus, hipStream_t stream) {
  hipLaunchKernelGGL(pbc_merge_kernel, dim3(Lmax, n), dim3(64), 0, stream, d_tor, Lmax,
                     d_block_spins);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && d_E_torus != nullptr) {
    hipLaunchKernelGGL(torus_energy_kernel, dim3(n), dim3(WAVE), 0, stream, d_tor, d_E_torus);
    e = hipGetLastError();
  }
  return e;
}

// ---------------------------------------------------------------------------------------------
// Independence Metropolis: one thread runs one chain over its proposals in order.
__global__ void accept_kernel(const DevReal* reals, int n, int n_chain, int K,
                              const double* prop_logq, const int32_t* prop_E, uint64_t seed,
                              uint64_t first_step, int32_t* chain_E, double* chain_logq,
                              uint8_t* chain_init, uint8_t* accepted, int32_t* current,
                              int32_t* oldE, int32_t* final_idx) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_chain) return;
  const int ri = t / n_chain, j = t % n_chain;
  const DevReal R = reals[ri];
  const int Kc = K / n_chain;
  int E = chain_E[t];
  double lq = chain_logq[t];
  bool init = chain_init[t] != 0;
  oldE[t] = E;
  int cur = -1;
  bool bad_delta = false;
  for (int s = 0; s < Kc; ++s) {
    const int k = j * Kc + s;
    const size_t o = size_t(ri) * K + k;
    const int Ep = prop_E[o];
    const double lp = prop_logq[o];
    const double u = philox_uniform(seed, STREAM_ACCEPT, first_step + uint64_t(s), uint64_t(j),
                                    R.id, 0);
    bool acc = false;
    if (!init) {
      init = true;
      cur = k;
      E = Ep;
      lq = lp;
    } else {
      const double delta = (-R.beta * double(Ep) - lp) - (-R.beta * double(E) - lq);
      bad_delta = bad_delta || !isfinite(delta);
      if (delta >= 0.0 || u < exp(delta)) {
        acc = true;
        cur = k;
        E = Ep;
        lq = lp;
      }
    }
    accepted[o] = acc ? 1 : 0;
    current[o] = cur;
  }
  chain_E[t] = E;
  chain_logq[t] = lq;
  chain_init[t] = init ? 1 : 0;
  final_idx[t] = cur;
  if (bad_delta && R.status != nullptr) atomicOr(R.status, TNMC_ST_DELTA);
}

// Copy each chain's final configuration (if it came from this batch) into the chain state.
__global__ void chain_copy_kernel(int n, int n_chain, int K, int Lmax,
                                  const uint64_t* prop_spins, uint64_t* chain_spins,
                                  const int32_t* final_idx) {
  const int t = blockIdx.y;
  const int idx = final_idx[t];
  if (idx < 0) return;
  const int ri = t / n_chain;
  const size_t words = size_t(Lmax) * words_per_row(Lmax);
  const uint64_t* src = prop_spins + (size_t(ri) * K + idx) * words;
  uint64_t* dst = chain_spins + size_t(t) * words;
  for (size_t o = blockIdx.x * blockDim.x + threadIdx.x; o < words; o += gridDim.x * blockDim.x)
    dst[o] = src[o];
}

// Observables of one configuration: m, m_edge (sites L/4 .. 3L/4-1 of each edge, / 2L).
__device__ __forceinline__ void config_obs(const uint64_t* s, int L, int Wmax, int lane, int& neg,
                                           int& edge_neg) {
  const int W = words_per_row(L);
  neg = 0;
  edge_neg = 0;
  const int a = L / 4, b = (3 * L) / 4;
  for (int o = lane; o < L * W; o += WAVE) {
    const int r = o / W, w = o % W;
    const uint64_t cw = s[size_t(r) * Wmax + w];
    neg += __popcll(cw);
    if (r == 0 || r == L - 1) {
      // columns a..b-1 of the top and bottom rows
      for (int c = max(a, 64 * w); c < min(b, 64 * w + 64); ++c) edge_neg += int((cw >> (c - 64 * w)) & 1ull);
    }
    if (r >= a && r < b) {
      if (w == 0) edge_neg += int(cw & 1ull);
      if (w == (L - 1) / 64) edge_neg += int((cw >> ((L - 1) % 64)) & 1ull);
    }
  }
}

__device__ __forceinline__ int overlap_diff(const uint64_t* s0, const uint64_t* s1, int L, int Wmax,
                                            int lane) {
  const int W = words_per_row(L);
  int d = 0;
  for (int o = lane; o < L * W; o += WAVE) {
    const int r = o / W, w = o % W;
    d += __popcll(s0[size_t(r) * Wmax + w] ^ s1[size_t(r) * Wmax + w]);
  }
  return d;
}

// Accumulate the observables of every (chain, step) of one realization per workgroup, with a
// fixed reduction order (bit-reproducible).  Each wavefront handles steps t = wave, wave + 4, ...
// `steps` = K / n_chain; `current` == nullptr means one sample per chain from the chain state.
__global__ void observables_kernel(const DevReal* reals, int n_chain, int K, int Lmax,
                                   const uint64_t* prop_spins, const int32_t* prop_E,
                                   const int32_t* current, const uint64_t* chain_spins,
                                   const int32_t* chain_E, double* accum) {
  constexpr int NWAVE = 4;
  __shared__ double part[NWAVE][TNMC_OBS_COUNT];
  const int ri = blockIdx.x;
  const DevReal R = reals[ri];
  const int L = R.L;
  const int Wmax = words_per_row(Lmax);
  const size_t words = size_t(Lmax) * Wmax;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int steps = current ? K / n_chain : 1;
  const double N = double(L) * L;
  double acc[TNMC_OBS_COUNT];
  for (int i = 0; i < TNMC_OBS_COUNT; ++i) acc[i] = 0.0;
  for (int t = wv; t < steps; t += NWAVE) {
    const uint64_t* cfg[2] = {nullptr, nullptr};
    for (int j = 0; j < n_chain; ++j) {
      const uint64_t* s;
      int E;
      if (current) {
        const int idx = current[size_t(ri) * K + j * steps + t];
        if (idx >= 0) {
          s = prop_spins + (size_t(ri) * K + idx) * words;
          E = prop_E[size_t(ri) * K + idx];
        } else {
          s = chain_spins + (size_t(ri) * n_chain + j) * words;
          E = chain_E[size_t(ri) * n_chain + j];
        }
      } else {
        s = chain_spins + (size_t(ri) * n_chain + j) * words;
        E = chain_E[size_t(ri) * n_chain + j];
      }
      if (j < 2) cfg[j] = s;
      int neg, eneg;
      config_obs(s, L, Wmax, lane, neg, eneg);
      neg = wave_sum(neg);
      eneg = wave_sum(eneg);
      const double m = (N - 2.0 * neg) / N;
      const double nedge = 2.0 * L;   // 4 segments of L/2 sites (L even); general: see below
      const int seg = (3 * L) / 4 - L / 4;
      const double me = (4.0 * seg - 2.0 * eneg) / nedge;
      acc[0] += 1.0;
      acc[1] += double(E);
      acc[2] += double(E) * double(E);
      acc[3] += m * m;
      acc[4] += m * m * m * m;
      acc[5] += me * me;
    }
    if (n_chain >= 2) {
      int d = overlap_diff(cfg[0], cfg[1], L, Wmax, lane);
      d = wave_sum(d);
      const double q = (N - 2.0 * d) / N;
      acc[6] += q;
      acc[7] += q * q;
      acc[8] += q * q * q * q;
    }
  }
  if (lane == 0)
    for (int i = 0; i < TNMC_OBS_COUNT; ++i) part[wv][i] = acc[i];
  __syncthreads();
  if (threadIdx.x < TNMC_OBS_COUNT) {
    double s = 0.0;
    for (int w = 0; w < NWAVE; ++w) s += part[w][threadIdx.x];
    accum[size_t(ri) * TNMC_OBS_COUNT + threadIdx.x] += s;
  }
}

hipError_t accept_launch(const DevReal* d_reals, int n, int n_chain, int K, int Lmax,
                         const uint64_t* d_prop_spins, const double* d_prop_logq,
                         const int32_t* d_prop_E, uint64_t seed, uint64_t first_step,
                         uint64_t* d_chain_spins, int32_t* d_chain_E, double* d_chain_logq,
                         uint8_t* d_chain_init, uint8_t* d_accepted, int32_t* d_current,
                         double* d_accum, int32_t* d_ws_oldE, int32_t* d_ws_final,
                         hipStream_t stream) {
  const int chains = n * n_chain;
  hipLaunchKernelGGL(accept_kernel, dim3((chains + 63) / 64), dim3(64), 0, stream, d_reals, n,
                     n_chain, K, d_prop_logq, d_prop_E, seed, first_step, d_chain_E, d_chain_logq,
                     d_chain_init, d_accepted, d_current, d_ws_oldE, d_ws_final);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (d_accum) {
    // steps sitting on a configuration from before this call use the saved energies
    hipLaunchKernelGGL(observables_kernel, dim3(n), dim3(256), 0, stream, d_reals, n_chain, K,
                       Lmax, d_prop_spins, d_prop_E, d_current, d_chain_spins, d_ws_oldE, d_accum);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  const size_t words = size_t(Lmax) * words_per_row(Lmax);
  dim3 grid(unsigned((words + 255) / 256), chains);
  hipLaunchKernelGGL(chain_copy_kernel, grid, dim3(256), 0, stream, n, n_chain, K, Lmax,
                     d_prop_spins, d_chain_spins, d_ws_final);
  return hipGetLastError();
}

hipError_t observables_launch(const DevReal* d_reals, int n, int n_chain, int Lmax,
                              const uint64_t* d_chain_spins, const int32_t* d_chain_E,
                              double* d_accum, hipStream_t stream) {
  hipLaunchKernelGGL(observables_kernel, dim3(n), dim3(256), 0, stream, d_reals, n_chain, n_chain,
                     Lmax, nullptr, nullptr, nullptr, d_chain_spins, d_chain_E, d_accum);
  return hipGetLastError();
}

// Disorder averages of Sec. III C over the n rows of accum (one realization each, one
// workgroup, fixed reduction order).  Thermal averages per realization: sum / count for the
// per-chain quantities, sum / (count / n_chain) for the overlap (formed once per step).
__global__ void __launch_bounds__(256) disorder_average_kernel(const double* accum, int n, int L,
                                                               double beta, int n_chain,
                                                               double* out) {
  constexpr int NT = 256, NQ = 9;
  __shared__ double part[NQ][NT];
  const int tid = threadIdx.x;
  double a[NQ];
  for (int j = 0; j < NQ; ++j) a[j] = 0.0;
  for (int i = tid; i < n; i += NT) {
    const double* r = accum + size_t(i) * TNMC_OBS_COUNT;
    const double cnt = r[0], cq = r[0] / double(n_chain);
    for (int j = 0; j < 5; ++j) a[j] += r[1 + j] / cnt;    // <E>, <E^2>, <m^2>, <m^4>, <m_edge^2>
    for (int j = 0; j < 3; ++j) a[5 + j] += r[6 + j] / cq; // <q>, <q^2>, <q^4>
    const double q2 = r[7] / cq;
    a[8] += q2 * q2;                                       // <q^2>^2
  }
  for (int j = 0; j < NQ; ++j) part[j][tid] = a[j];
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int j = 0; j < NQ; ++j) part[j][tid] += part[j][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    double m[NQ];
    for (int j = 0; j < NQ; ++j) m[j] = part[j][0] / double(n);
    for (int j = 0; j < NQ; ++j) out[j] = m[j];
    out[9] = m[7] / m[8];                                      // Q_q = [<q^4>] / [<q^2>^2]
    out[10] = double(L) * double(L) * beta * (m[6] - m[5] * m[5]);   // chi_q
    out[11] = double(L) * m[4];                                // chi_edge = L [<m_edge^2>]
  }
}

hipError_t disorder_average_launch(const double* d_accum, int n, int L, double beta, int n_chain,
                                   double* d_out, hipStream_t stream) {
  hipLaunchKernelGGL(disorder_average_kernel, dim3(1), dim3(256), 0, stream, d_accum, n, L, beta,
                     n_chain, d_out);
  return hipGetLastError();
}

}  // namespace tnmc
