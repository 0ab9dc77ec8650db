// Whole-lattice proposals from the cached environments (Sec. II A-B of arXiv:2409.06538,
// Eqs. (4)-(6)), with log q(s) in FP64 and the exact integer energy (Eq. (8)) of each proposal.
//
// Row r of a proposal is drawn from the row chain
//   f_r(y) = prod_c phi_c(y_c) prod_c w_c(y_c, y_{c+1}) E_r(y),
//   phi_c(y) = exp(beta Jv[r-1][c] s[r-1][c] y),  w_c(y, y') = exp(beta Jh[r][c] y y'),
// exactly marginalised column by column:
//   right sweep (c = L-1 .. 0):  v_c(y) = B_c[y] R_c(y),  R_{c-1}(y) = sum_y' w_{c-1}(y,y') phi_c(y') v_c(y'),
//   left sweep  (c = 0 .. L-1):  Z_c(y) = [w_{c-1}(s_{c-1}, y)] phi_c(y) (l . v_c(y)),  draw s_c,
//                                l <- [w_{c-1}(s_{c-1}, s_c)] phi_c(s_c) l B_c[s_c].
// R and l are rescaled by powers of two (they cancel in p+).  One thread owns one proposal; a
// workgroup of 64 proposals of one realization shares each site tensor through LDS; the v_c of a
// row go to the workspace between the two sweeps.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace tnmc {

constexpr int PROP_NT = 64;
constexpr int MAX_W = 16;   // words per row for L <= 1024
constexpr double P_CLAMP = 1e-12;

template <typename T>
__device__ __forceinline__ T spin_weight(bool af, bool parallel, T ep, T em) {
  return (parallel != af) ? ep : em;
}

// T: arithmetic type; E: storage type of the environments.
template <typename T, typename E, int CHI>
__global__ __launch_bounds__(PROP_NT) void propose_kernel(const DevReal* reals, int K, int Lmax,
                                                          uint64_t seed, uint64_t first,
                                                          const uint64_t* teacher,
                                                          uint64_t* spins_out, double* logq_out,
                                                          int32_t* E_out, uint32_t* fallbacks) {
  __shared__ T Bs[2 * CHI * CHI];
  // bit-packed rows of each proposal: [0] the row above, [1] the row being drawn
  __shared__ uint64_t rows[2][MAX_W][PROP_NT];
  const int tid = threadIdx.x;
  const int ri = blockIdx.y;
  const DevReal R = reals[ri];
  const int L = R.L;
  const int W = words_per_row(L);
  const int Wmax = words_per_row(Lmax);
  const int k = blockIdx.x * PROP_NT + tid;
  const bool active = k < K;
  const int kk = active ? k : K - 1;   // inactive lanes shadow a valid proposal, write nothing
  const T ep = T(exp(R.beta)), em = T(exp(-R.beta));
  const E* env = reinterpret_cast<const E*>(R.env);
  const size_t site = size_t(2) * CHI * CHI;
  // v store for this realization: [c][y][alpha][k]
  T* vs = reinterpret_cast<T*>(R.ws);
  const size_t vstride = size_t(K);
  const uint64_t pid = first + uint64_t(kk);

  uint64_t* prev = &rows[0][0][tid];   // word w at prev[w * PROP_NT]
  uint64_t* cur = &rows[1][0][tid];
  for (int w = 0; w < MAX_W; ++w) { prev[w * PROP_NT] = 0; cur[w * PROP_NT] = 0; }
  double logq = 0.0;
  uint32_t nfb = 0;
  int unsat = 0;
  const uint64_t* tin = teacher ? teacher + (size_t(ri) * K + kk) * size_t(Lmax) * Wmax : nullptr;

  for (int r = 0; r < L; ++r) {
    const E* Arow = env + size_t(r) * site * L;
    const uint64_t* jh = R.Jh + size_t(r) * W;
    const uint64_t* jv = (r > 0) ? R.Jv + size_t(r - 1) * W : nullptr;

    // ---- right sweep ----
    T Rn[2][CHI];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int a = 0; a < CHI; ++a) Rn[y][a] = (a == 0) ? T(1) : T(0);
    for (int c = L - 1; c >= 0; --c) {
      __syncthreads();
      for (int e = tid; e < int(site); e += PROP_NT) Bs[e] = widen(Arow[size_t(c) * site + e]);
      __syncthreads();
      T v[2][CHI];
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int a = 0; a < CHI; ++a) {
          T d = 0;
#pragma unroll
          for (int b = 0; b < CHI; ++b) d += Bs[(y * CHI + a) * CHI + b] * Rn[y][b];
          v[y][a] = d;
        }
      T* vo = vs + (size_t(c) * 2 * CHI) * vstride + kk;
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int a = 0; a < CHI; ++a) if (active) vo[(y * CHI + a) * vstride] = v[y][a];
      if (c > 0) {
        // phi_c(y') and w_{c-1}(y, y')
        T ph[2] = {T(1), T(1)};
        if (r > 0) {
          const bool af = (jv[c >> 6] >> (c & 63)) & 1ull;
          const bool sm = (prev[(c >> 6) * PROP_NT] >> (c & 63)) & 1ull;   // spin above is -1
#pragma unroll
          for (int yp = 0; yp < 2; ++yp) ph[yp] = spin_weight<T>(af, (yp == 1) == sm, ep, em);
        }
        const bool afh = (jh[(c - 1) >> 6] >> ((c - 1) & 63)) & 1ull;
        const T wpp = spin_weight<T>(afh, true, ep, em), wpm = spin_weight<T>(afh, false, ep, em);
        T mx = 0;
#pragma unroll
        for (int a = 0; a < CHI; ++a) {
          const T t0 = ph[0] * v[0][a], t1 = ph[1] * v[1][a];
          Rn[0][a] = wpp * t0 + wpm * t1;
          Rn[1][a] = wpm * t0 + wpp * t1;
          mx = fmax(mx, fmax(fabs(Rn[0][a]), fabs(Rn[1][a])));
        }
        const int e = pow2_exponent(mx);
#pragma unroll
        for (int a = 0; a < CHI; ++a) {
          Rn[0][a] = T(ldexp(Rn[0][a], -e));
          Rn[1][a] = T(ldexp(Rn[1][a], -e));
        }
      }
    }

    // ---- left sweep ----
    T ell[CHI];
#pragma unroll
    for (int a = 0; a < CHI; ++a) ell[a] = (a == 0) ? T(1) : T(0);
    for (int w = 0; w < MAX_W; ++w) cur[w * PROP_NT] = 0;
    Philox4 blk{};
    int sprev = 0;   // 0 <-> +1, 1 <-> -1 (spin at c-1 of this row)
    for (int c = 0; c < L; ++c) {
      __syncthreads();
      for (int e = tid; e < int(site); e += PROP_NT) Bs[e] = widen(Arow[size_t(c) * site + e]);
      __syncthreads();
      T pre[2] = {T(1), T(1)};
      if (r > 0) {
        const bool af = (jv[c >> 6] >> (c & 63)) & 1ull;
        const bool sm = (prev[(c >> 6) * PROP_NT] >> (c & 63)) & 1ull;
#pragma unroll
        for (int y = 0; y < 2; ++y) pre[y] = spin_weight<T>(af, (y == 1) == sm, ep, em);
      }
      if (c > 0) {
        const bool afh = (jh[(c - 1) >> 6] >> ((c - 1) & 63)) & 1ull;
#pragma unroll
        for (int y = 0; y < 2; ++y) pre[y] *= spin_weight<T>(afh, y == sprev, ep, em);
      }
      const T* vi = vs + (size_t(c) * 2 * CHI) * vstride + kk;
      T z[2];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        T d = 0;
#pragma unroll
        for (int a = 0; a < CHI; ++a) d += ell[a] * vi[(y * CHI + a) * vstride];
        z[y] = pre[y] * d;
      }
      double zp = double(z[0]) > 0.0 ? double(z[0]) : 0.0;
      double zm = double(z[1]) > 0.0 ? double(z[1]) : 0.0;
      double tot = zp + zm;
      double pp;
      if (!(tot > 0.0) || !isfinite(tot)) {
        pp = 0.5;
        ++nfb;
      } else {
        pp = zp / tot;
      }
      pp = fmin(fmax(pp, P_CLAMP), 1.0 - P_CLAMP);
      bool up;
      if (teacher) {
        up = !((tin[size_t(r) * Wmax + (c >> 6)] >> (c & 63)) & 1ull);
      } else {
        if ((c & 3) == 0) blk = philox4x64_10(uint64_t(c) >> 2, uint64_t(r), pid, R.id, seed, STREAM_PROPOSAL);
        const int q = c & 3;
        const uint64_t wsel = q == 0 ? blk.w[0] : q == 1 ? blk.w[1] : q == 2 ? blk.w[2] : blk.w[3];
        up = u53(wsel) < pp;
      }
      logq += up ? log(pp) : log(1.0 - pp);
      const int s = up ? 0 : 1;
      if (!up) cur[(c >> 6) * PROP_NT] |= (1ull << (c & 63));
      // l <- pre(s) l B_c[s]
      T nl[CHI];
      T mx = 0;
#pragma unroll
      for (int b = 0; b < CHI; ++b) {
        T d = 0;
#pragma unroll
        for (int a = 0; a < CHI; ++a) d += ell[a] * Bs[(s * CHI + a) * CHI + b];
        nl[b] = (s == 0 ? pre[0] : pre[1]) * d;
        mx = fmax(mx, fabs(nl[b]));
      }
      const int e = pow2_exponent(mx);
#pragma unroll
      for (int b = 0; b < CHI; ++b) ell[b] = T(ldexp(nl[b], -e));
      sprev = s;
    }

    // ---- energy bookkeeping: unsatisfied bonds of row r and between rows r-1, r ----
    for (int w = 0; w < W; ++w) {
      const uint64_t cw = cur[w * PROP_NT];
      const uint64_t nxt = (w + 1 < W) ? cur[(w + 1) * PROP_NT] : 0ull;
      const uint64_t right = (cw >> 1) | (nxt << 63);
      const int nb_h = (L - 1) - 64 * w;   // valid horizontal bonds in this word
      const uint64_t mh = nb_h >= 64 ? ~0ull : (nb_h > 0 ? ((1ull << nb_h) - 1) : 0ull);
      unsat += __popcll((cw ^ right ^ jh[w]) & mh);
      if (r > 0) {
        const int nb_v = L - 64 * w;
        const uint64_t mv = nb_v >= 64 ? ~0ull : ((1ull << nb_v) - 1);
        unsat += __popcll((prev[w * PROP_NT] ^ cw ^ jv[w]) & mv);
      }
    }
    if (active && !teacher) {
      uint64_t* so = spins_out + ((size_t(ri) * K + k) * Lmax + r) * Wmax;
      for (int w = 0; w < Wmax; ++w) so[w] = (w < W) ? cur[w * PROP_NT] : 0ull;
    }
    for (int w = 0; w < MAX_W; ++w) prev[w * PROP_NT] = cur[w * PROP_NT];
  }
  if (active) {
    logq_out[size_t(ri) * K + k] = logq;
    if (!teacher) {
      E_out[size_t(ri) * K + k] = 2 * unsat - 2 * L * (L - 1);
      // rows beyond this realization's L (mixed batches) are zero
      for (int r = L; r < Lmax; ++r) {
        uint64_t* so = spins_out + ((size_t(ri) * K + k) * Lmax + r) * Wmax;
        for (int w = 0; w < Wmax; ++w) so[w] = 0ull;
      }
    }
    if (fallbacks && nfb) atomicAdd(fallbacks + ri, nfb);
  }
}

template <typename T, typename E, int CHI>
hipError_t launch_propose(const DevReal* d_reals, int n, int K, int Lmax, uint64_t seed,
                          uint64_t first, const uint64_t* d_teacher, uint64_t* d_spins,
                          double* d_logq, int32_t* d_E, uint32_t* d_fallbacks,
                          hipStream_t stream) {
  dim3 grid((K + PROP_NT - 1) / PROP_NT, n);
  hipLaunchKernelGGL((propose_kernel<T, E, CHI>), grid, dim3(PROP_NT), 0, stream, d_reals, K, Lmax,
                     seed, first, d_teacher, d_spins, d_logq, d_E, d_fallbacks);
  return hipGetLastError();
}

hipError_t propose(tnmc_precision prec, int chi, const DevReal* d_reals, int n, int K, int Lmax,
                   uint64_t seed, uint64_t first, const uint64_t* d_teacher, uint64_t* d_spins,
                   double* d_logq, int32_t* d_E, uint32_t* d_fallbacks, hipStream_t stream) {
#define TNMC_PROP_CASE(TY, EY, C)                                                               \
  case C:                                                                                       \
    return launch_propose<TY, EY, C>(d_reals, n, K, Lmax, seed, first, d_teacher, d_spins,      \
                                     d_logq, d_E, d_fallbacks, stream);
#define TNMC_PROP_CHIS(TY, EY) \
  TNMC_PROP_CASE(TY, EY, 2) TNMC_PROP_CASE(TY, EY, 4) TNMC_PROP_CASE(TY, EY, 8) \
  TNMC_PROP_CASE(TY, EY, 16) TNMC_PROP_CASE(TY, EY, 32)
  if (prec == TNMC_FP64) {
    switch (chi) { TNMC_PROP_CHIS(double, double) }
  } else if (prec == TNMC_FP32) {
    switch (chi) { TNMC_PROP_CHIS(float, float) }
  } else if (prec == TNMC_BF16) {
    switch (chi) { TNMC_PROP_CHIS(float, bf16_t) }
  }
#undef TNMC_PROP_CHIS
#undef TNMC_PROP_CASE
  return hipErrorInvalidValue;
}

size_t propose_scratch_bytes(tnmc_precision prec, int chi, int L, int K) {
  const size_t elem = (prec == TNMC_FP64) ? 8 : 4;
  return size_t(L) * 2 * chi * size_t(K) * elem;
}

}  // namespace tnmc
