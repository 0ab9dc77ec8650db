// Whole-lattice proposals from the cached environments (Sec. II A-B of arXiv:2409.06538,
// Eqs. (4)-(6)), with log q(s) in FP64 and the exact integer energy (Eq. (10)) of each proposal.
//
// Row r of a proposal is drawn from the row chain
//   f_r(y) = prod_c phi_c(y_c) prod_c w_c(y_c, y_{c+1}) E_r(y),
//   phi_c(y) = exp(beta Jv[r-1][c] s[r-1][c] y),  w_c(y, y') = exp(beta Jh[r][c] y y'),
//   (phi_c also carries exp(beta h[r][c] y) for a realization with site fields),
// exactly marginalised column by column:
//   right sweep (c = L-1 .. 0):  v_c(y) = B_c[y] R_c(y),  R_{c-1}(y) = sum_y' w_{c-1}(y,y') phi_c(y') v_c(y'),
//   left sweep  (c = 0 .. L-1):  Z_c(y) = [w_{c-1}(s_{c-1}, y)] phi_c(y) (l . v_c(y)),  draw s_c,
//                                l <- [w_{c-1}(s_{c-1}, s_c)] phi_c(s_c) l B_c[s_c].
// R and l are rescaled by powers of two (they cancel in p+).  One thread owns one proposal; a
// workgroup of 64 proposals of one realization shares each site tensor through LDS; the v_c of a
// row go to the workspace between the two sweeps.
#include <hip/hip_runtime.h>

#include <type_traits>

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
  const DevReal R = reals[blockIdx.y];
  const int ri = R.slot;   // the caller's index of this realization (outputs, teacher rows)
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
  uint32_t stb = 0;   // status bits of this proposal
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
        if (R.field != nullptr) {   // the site's field, exp(beta h y')
          T g0, g1;
          site_field<T>(R, r, c, ep, em, g0, g1);
          ph[0] *= g0;
          ph[1] *= g1;
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
      if (R.field != nullptr) {
        T g0, g1;
        site_field<T>(R, r, c, ep, em, g0, g1);
        pre[0] *= g0;
        pre[1] *= g1;
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
      if (!isfinite(z[0]) || !isfinite(z[1])) stb |= TNMC_ST_WEIGHT;
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
    if (!isfinite(logq)) stb |= TNMC_ST_LOGQ;
    if (nfb) stb |= TNMC_ST_FALLBACK;
    if (R.status != nullptr && stb != 0) atomicOr(R.status, stb);
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

// ------------------------------------------------------------------------------------------
// MFMA form (chi a multiple of 16).  A wavefront owns 16 proposals; four wavefronts share each
// site tensor through LDS.  Per site and per spin value y the right sweep is the product
// V_y = B_c[y] R_y (chi x chi times chi x 16) and the left sweep U_y^T = B_c[y]^T l (the same
// shape), both as 16x16x4 matrix-core tiles.  The k index of every product runs over the rows
// that the output tile of the previous product leaves in the same lane, so R and l stay in
// registers from site to site: no transposes.  Lane group q = lane / 16 holds, for proposal
// p = lane % 16, rows 16 t + row(q, r) of R, l and V (t < chi / 16, r < 4).

template <typename T>
struct Mf;
template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row of a 16 x 16 tile held by lane group q in register r
  __host__ __device__ static constexpr int row(int q, int r) { return 4 * q + r; }
  // LDS column of index x (< 16) so that the four rows row(q, 0..3) are adjacent
  __host__ __device__ static constexpr int pos(int x) { return x; }
};
template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __host__ __device__ static constexpr int row(int q, int r) { return q + 4 * r; }
  __host__ __device__ static constexpr int pos(int x) { return 4 * (x & 3) + (x >> 2); }
};

// Wavefronts per workgroup (each owns 16 proposals).  More wavefronts share each staged site
// tensor (less environment traffic per proposal) but give fewer workgroups and a larger V store
// per workgroup.  Measured: 8 is faster up to L = 64 when the grid still covers every CU once;
// 4 for larger L and for small grids (a single proposal also runs fastest with the site staging
// spread over 4 wavefronts).
constexpr int MF_MAX_PROP = 128;   // K is padded to this in the workspace (any WAVES <= 8)
constexpr int MF_CUS = 256;
// Launch shape used when the tuning table has no entry for a call: 8 wavefronts (128 proposals
// per workgroup) for L <= 64 when the grid still covers every CU; else 4, unless the grid of
// 4-wavefront workgroups leaves CUs idle, when the fewest wavefronts per workgroup that fill them
// (or 1: small batches of large lattices).
int propose_default_waves(int chi, int n, int K, int Lmax) {
  if (chi % 16 != 0) return 1;
  auto grid = [&](int waves) { return size_t(n) * size_t((K + 16 * waves - 1) / (16 * waves)); };
  if (Lmax <= 64 && grid(8) >= size_t(MF_CUS)) return 8;
  if (grid(4) >= size_t(MF_CUS)) return 4;
  return grid(2) >= size_t(MF_CUS) ? 2 : 1;
}

// Wavefronts per workgroup that the proposal kernel is built for at this chi (16 proposals per
// wavefront with matrix-core tiles; one thread per proposal, 64 per workgroup, otherwise).
int propose_waves_ok(int chi, int waves) {
  if (chi % 16 != 0) return waves == 1;
  return waves == 1 || waves == 2 || waves == 4 || waves == 8;
}

template <typename T, typename E, int CHI, int MF_WAVES>
__global__ __launch_bounds__(64 * MF_WAVES) void propose_mfma_kernel(const DevReal* reals, int K, int Lmax,
                                                             uint64_t seed, uint64_t first,
                                                             const uint64_t* teacher,
                                                             uint64_t* spins_out, double* logq_out,
                                                             int32_t* E_out, uint32_t* fallbacks) {
  constexpr int MF_NT = 64 * MF_WAVES;
  constexpr int MF_PROP = 16 * MF_WAVES;   // proposals per workgroup
  static_assert(MF_PROP <= MF_MAX_PROP, "workspace padding");
  using M = Mf<T>;
  using V4 = typename M::v4;
  constexpr int RT = CHI / 16;                   // 16-row tiles of a site matrix
  constexpr int NV = 2 * RT * 4;                 // V values per lane (y, tile, register)
  constexpr int PV = 16 / int(sizeof(T));        // values per 16-byte chunk
  constexpr int LDB = CHI + PV;                  // LDS row stride of a site matrix
  constexpr int SITE = 2 * CHI * CHI;
  constexpr int SPT = (SITE + MF_NT - 1) / MF_NT;   // site elements loaded per thread
  __shared__ __align__(16) T Bs[2][2 * CHI * LDB];
  __shared__ uint64_t rows[2][MAX_W][MF_PROP];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int pl = lane & 15, q = lane >> 4;
  const int slot = wv * 16 + pl;
  // Workgroups go to the 8 XCDs in turn (linear id w -> XCD w % 8).  When the realizations split
  // evenly, all proposal chunks of realization y run on XCD y % 8, one after the other, so that
  // they read its environments through the same L2.
  int bx = blockIdx.x, by = blockIdx.y;
  if (gridDim.y % 8 == 0) {
    const int w = blockIdx.x + gridDim.x * blockIdx.y;
    const int idx = w >> 3;
    bx = idx % gridDim.x;
    by = (w & 7) + 8 * (idx / gridDim.x);
  }
  const DevReal R = reals[by];
  const int ri = R.slot;   // the caller's index of this realization (outputs, teacher rows)
  const int L = R.L;
  const int W = words_per_row(L);
  const int Wmax = words_per_row(Lmax);
  const int k = bx * MF_PROP + slot;
  const bool active = k < K;
  const int kk = active ? k : K - 1;   // inactive slots shadow a valid proposal, write nothing
  const T ep = T(exp(R.beta)), em = T(exp(-R.beta));
  const gmem<E>* env = as_global(reinterpret_cast<E*>(R.env));
  // V store of this wavefront: [c][chunk][lane][PV]
  gmem<T>* vbase = as_global(reinterpret_cast<T*>(R.ws)) +
                   (size_t(bx) * L * MF_WAVES + wv) * (64 * NV) + lane * PV;
  const size_t vstep = size_t(MF_WAVES) * 64 * NV;   // per site
  const uint64_t pid = first + uint64_t(kk);
  const uint64_t* tin = teacher ? teacher + (size_t(ri) * K + kk) * size_t(Lmax) * Wmax : nullptr;

  for (int e = tid; e < 2 * MAX_W * MF_PROP; e += MF_NT) (&rows[0][0][0])[e] = 0ull;
  // log q accumulates as a product of the chosen conditionals, renormalised to [0.5, 1) with
  // its binary exponent kept apart (no underflow), and one logarithm at the end: the same value
  // to rounding as the sum of the logarithms, without a logarithm per site.
  double qprod = 1.0;
  int qexp = 0;
  uint32_t nfb = 0;
  uint32_t stb = 0;   // status bits of this proposal
  int unsat = 0;
  int pr = 0;   // rows[pr]: row above; rows[pr ^ 1]: row being drawn

  // Site staging: with VEC, thread tid loads the SPT contiguous elements from tid * SPT in
  // 16-byte pieces; otherwise element tid + MF_NT t (strided, one element per load).
  // (8-byte pieces when the thread's share is 8 bytes: 4 BF16 values with 8 wavefronts)
  constexpr int PIECE = ((SPT * sizeof(E)) % 16 == 0) ? 16 : 8;
  constexpr bool VEC = SITE % MF_NT == 0 && (SPT * sizeof(E)) % PIECE == 0 && CHI % SPT == 0;
  constexpr int NQ = VEC ? int(SPT * sizeof(E) / PIECE) : 1;   // pieces per thread
  typedef unsigned int u4 __attribute__((ext_vector_type(PIECE / 4)));
  E pf[SPT];
  u4 pq[NQ];
  // With the bond table at CHI = 64, a site whose bonds are both at most 16 loads only the
  // leading 16 x 16 block of its two matrices (the rest is zero): NN entries per thread instead
  // of SPT.  Smaller sites are staged whole, which measured faster (their narrow test runs on
  // the staged values).
  constexpr int NN = (2 * 256 + MF_NT - 1) / MF_NT;
  E nf[NN];
  bool nsite = false;   // the staged site is narrow by the bond table
  const gmem<const uint8_t>* bonds = R.bonds ? as_global(R.bonds) : nullptr;
  auto load_site = [&](int r, int c) {
    const gmem<E>* src = env + (size_t(r) * L + c) * SITE;
    if (CHI >= 64 && bonds != nullptr) {
      const size_t bi = size_t(r) * (L + 1) + c;
      nsite = bonds[bi] <= 16 && bonds[bi + 1] <= 16;
      if (nsite) {
#pragma unroll
        for (int t = 0; t < NN; ++t) {
          const int e = tid + MF_NT * t;
          if (e < 512) nf[t] = gld<E>(src, ((e >> 8) * CHI + ((e >> 4) & 15)) * CHI + (e & 15));
        }
        return;
      }
    }
    if constexpr (VEC) {
      const gmem<u4>* s4 = reinterpret_cast<const gmem<u4>*>(src + size_t(tid) * SPT);
#pragma unroll
      for (int i = 0; i < NQ; ++i) pq[i] = s4[i];
    } else {
#pragma unroll
      for (int t = 0; t < SPT; ++t) {
        const int e = tid + MF_NT * t;
        if (SITE % MF_NT == 0 || e < SITE) pf[t] = gld<E>(src, e);
      }
    }
  };
  auto elem = [&](int t) {   // element t of this thread's staged part
    if constexpr (VEC) {
      E v[SPT];
      __builtin_memcpy(v, pq, sizeof(v));
      return v[t];
    } else {
      return pf[t];
    }
  };
  auto elem_index = [&](int t) { return VEC ? tid * SPT + t : tid + MF_NT * t; };
  // right sweep: row alpha, column beta; left sweep (transposed): row beta, column alpha.
  // Returns whether this thread stored a nonzero entry outside the leading 16 x 16 block of a
  // matrix: a site whose entries all lie inside it (both bonds at most 16, the rest zero padding)
  // is narrow, and its products and V rows are the first tile only.
  auto store_site = [&](T* dst, bool transposed) {
    bool wide = false;
    if (nsite) {
#pragma unroll
      for (int t = 0; t < NN; ++t) {
        const int e = tid + MF_NT * t;
        if (e < 512) {
          const int y = e >> 8, a = (e >> 4) & 15, b = e & 15;
          const int rr = transposed ? b : a, cc = transposed ? a : b;
          dst[(y * CHI + rr) * LDB + M::pos(cc)] = widen(nf[t]);
        }
      }
      return false;
    }
#pragma unroll
    for (int t = 0; t < SPT; ++t) {
      const int e = elem_index(t);
      if (SITE % MF_NT == 0 || e < SITE) {
        const int y = e / (CHI * CHI), a = (e / CHI) % CHI, b = e % CHI;
        const int rr = transposed ? b : a, cc = transposed ? a : b;
        const T v = widen(elem(t));
        dst[(y * CHI + rr) * LDB + (cc & ~15) + M::pos(cc & 15)] = v;
        wide = wide || ((a >= 16 || b >= 16) && v != T(0));
      }
    }
    return wide;
  };
  // C = sum over the chi contraction index of Bsb[y][16 ro + pl][.] times the register operand;
  // nt (1 or RT, wave-uniform) tiles of rows and of the contraction index
  auto tile_products = [&](const T* Bsb, const T (&opnd)[2][RT][4], V4 (&acc)[2][RT], int nt) {
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int ro = 0; ro < RT; ++ro) {
        V4 a = {T(0), T(0), T(0), T(0)};
        if (ro < nt) {
          const T* ap = Bsb + (y * CHI + 16 * ro + pl) * LDB + 4 * q;
#pragma unroll
          for (int m = 0; m < RT; ++m) {
            if (m < nt) {
              T av[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) av[r] = ap[16 * m + r];
#pragma unroll
              for (int r = 0; r < 4; ++r) a = M::mac(av[r], opnd[y][m][r], a);
            }
          }
        }
        acc[y][ro] = a;
      }
  };
  // maximum over the four lane groups of a proposal (identical in all four lanes)
  auto group4_max = [&](T v) {
    v = fmax(v, __shfl_xor(v, 16));
    return fmax(v, __shfl_xor(v, 32));
  };
  auto group4_sum = [&](T v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
  };

  int b = 0;
  for (int r = 0; r < L; ++r) {
    const gmem<const uint64_t>* jh = as_global(R.Jh) + size_t(r) * W;
    const gmem<const uint64_t>* jv = (r > 0) ? as_global(R.Jv) + size_t(r - 1) * W : nullptr;
    const uint64_t* prow = &rows[pr][0][slot];       // word w at prow[w * MF_PROP]
    uint64_t* crow = &rows[pr ^ 1][0][slot];

    // ---- right sweep: V_c(y) = B_c[y] R_c(y) for c = L-1 .. 0 ----
    T rc[2][RT][4];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[y][t][i] = (t == 0 && M::row(q, i) == 0) ? T(1) : T(0);
    load_site(r, L - 1);
    int nt = __syncthreads_or(store_site(Bs[b], false)) ? RT : 1;
    for (int c = L - 1; c >= 0; --c) {
      if (c > 0) load_site(r, c - 1);
      bool wide = false;
      V4 acc[2][RT];
      tile_products(Bs[b], rc, acc, nt);
      gmem<T>* vo = vbase + size_t(c) * vstep;
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (t < nt)   // rows past the first tile of a narrow site are zero and not stored
#pragma unroll
          for (int h = 0; h < 4; h += PV) {
            const int chunk = ((y * RT + t) * 4 + h) / PV;
            if constexpr (PV == 4) {
              *reinterpret_cast<gmem<V4>*>(vo + chunk * 64 * PV) = acc[y][t];
            } else {
              typedef T v2 __attribute__((ext_vector_type(2)));
              v2 d = {acc[y][t][h], acc[y][t][h + 1]};
              *reinterpret_cast<gmem<v2>*>(vo + chunk * 64 * PV) = d;
            }
          }
      if (c > 0) {
        T ph[2] = {T(1), T(1)};
        if (r > 0) {
          const bool af = (jv[c >> 6] >> (c & 63)) & 1ull;
          const bool sm = (prow[(c >> 6) * MF_PROP] >> (c & 63)) & 1ull;   // spin above is -1
          ph[0] = spin_weight<T>(af, !sm, ep, em);
          ph[1] = spin_weight<T>(af, sm, ep, em);
        }
        if (R.field != nullptr) {   // the site's field, exp(beta h y)
          T g0, g1;
          site_field<T>(R, r, c, ep, em, g0, g1);
          ph[0] *= g0;
          ph[1] *= g1;
        }
        const bool afh = (jh[(c - 1) >> 6] >> ((c - 1) & 63)) & 1ull;
        const T wpp = spin_weight<T>(afh, true, ep, em), wpm = spin_weight<T>(afh, false, ep, em);
        T mx = 0;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T t0 = ph[0] * acc[0][t][i], t1 = ph[1] * acc[1][t][i];
            rc[0][t][i] = wpp * t0 + wpm * t1;
            rc[1][t][i] = wpm * t0 + wpp * t1;
            mx = fmax(mx, fmax(fabs(rc[0][t][i]), fabs(rc[1][t][i])));
          }
        const int e = pow2_exponent(group4_max(mx));
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) rc[y][t][i] = T(ldexp(rc[y][t][i], -e));
        wide = store_site(Bs[b ^ 1], false);
      }
      const int nt_next = __syncthreads_or(wide) ? RT : 1;
      if (c > 0) {
        b ^= 1;
        nt = nt_next;
      }
    }

    // ---- left sweep: draw s_c from Z_c(y) = pre(y) (l . V_c(y)), then l <- pre(s) B_c[s]^T l ----
    T el[2][RT][4];   // el[0] = l (el[1] unused: same shape as the product operand)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) el[y][t][i] = (t == 0 && M::row(q, i) == 0) ? T(1) : T(0);
    b ^= 1;
    load_site(r, 0);
    nt = __syncthreads_or(store_site(Bs[b], true)) ? RT : 1;
    Philox4 blk{};
    int sprev = 0;   // 0 <-> +1, 1 <-> -1 (spin at c-1 of this row)
    uint64_t curw = 0, tword = 0;
    for (int c = 0; c < L; ++c) {
      if (c + 1 < L) load_site(r, c + 1);
      const gmem<T>* vi = vbase + size_t(c) * vstep;
      T vv[2][RT][4];
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int h = 0; h < 4; h += PV) {
            const int chunk = ((y * RT + t) * 4 + h) / PV;
#pragma unroll
            for (int u = 0; u < PV; ++u) vv[y][t][h + u] = (t < nt) ? vi[chunk * 64 * PV + u] : T(0);
          }
      T pre[2] = {T(1), T(1)};
      if (r > 0) {
        const bool af = (jv[c >> 6] >> (c & 63)) & 1ull;
        const bool sm = (prow[(c >> 6) * MF_PROP] >> (c & 63)) & 1ull;
        pre[0] = spin_weight<T>(af, !sm, ep, em);
        pre[1] = spin_weight<T>(af, sm, ep, em);
      }
      if (R.field != nullptr) {
        T g0, g1;
        site_field<T>(R, r, c, ep, em, g0, g1);
        pre[0] *= g0;
        pre[1] *= g1;
      }
      if (c > 0) {
        const bool afh = (jh[(c - 1) >> 6] >> ((c - 1) & 63)) & 1ull;
        pre[0] *= spin_weight<T>(afh, sprev == 0, ep, em);
        pre[1] *= spin_weight<T>(afh, sprev == 1, ep, em);
      }
      T zp = 0, zm = 0;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          zp += el[0][t][i] * vv[0][t][i];
          zm += el[0][t][i] * vv[1][t][i];
        }
      zp = pre[0] * group4_sum(zp);
      zm = pre[1] * group4_sum(zm);
      const double dzp = double(zp) > 0.0 ? double(zp) : 0.0;
      const double dzm = double(zm) > 0.0 ? double(zm) : 0.0;
      const double tot = dzp + dzm;
      double pp;
      if (!isfinite(zp) || !isfinite(zm)) stb |= TNMC_ST_WEIGHT;
      if (!(tot > 0.0) || !isfinite(tot)) {
        pp = 0.5;
        ++nfb;
      } else {
        pp = dzp / tot;
      }
      pp = fmin(fmax(pp, P_CLAMP), 1.0 - P_CLAMP);
      bool up;
      if (teacher) {
        if ((c & 63) == 0) tword = tin[size_t(r) * Wmax + (c >> 6)];
        up = !((tword >> (c & 63)) & 1ull);
      } else {
        // The four lane groups of a proposal draw for sites c .. c + 15 at once: group q forms the
        // Philox block of sites c + 4 q .. c + 4 q + 3, and the word of site c comes from group
        // (c / 4) mod 4 by a shuffle (the same words as one block per group every four sites).
        if ((c & 15) == 0)
          blk = philox4x64_10((uint64_t(c) >> 2) + uint64_t(q), uint64_t(r), pid, R.id, seed,
                              STREAM_PROPOSAL);
        const int qq = c & 3;
        const uint64_t mine = qq == 0 ? blk.w[0] : qq == 1 ? blk.w[1] : qq == 2 ? blk.w[2] : blk.w[3];
        const int src = pl + 16 * ((c >> 2) & 3);
        const unsigned lo = __shfl(unsigned(mine & 0xffffffffull), src);
        const unsigned hi = __shfl(unsigned(mine >> 32), src);
        up = u53((uint64_t(hi) << 32) | lo) < pp;
      }
      {
        int ex;
        qprod = frexp(qprod * (up ? pp : 1.0 - pp), &ex);
        qexp += ex;
      }
      const int s = up ? 0 : 1;
      if (!up) curw |= (1ull << (c & 63));
      if ((c & 63) == 63 || c == L - 1) {
        if (q == 0) crow[(c >> 6) * MF_PROP] = curw;
        curw = 0;
      }
      // l <- pre(s) B_c[s]^T l (both products; each proposal keeps its own)
      V4 u[2][RT];
      tile_products(Bs[b], el, u, nt);
      T mx = 0;
      const T ps = s == 0 ? pre[0] : pre[1];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          el[0][t][i] = ps * (s == 0 ? u[0][t][i] : u[1][t][i]);
          mx = fmax(mx, fabs(el[0][t][i]));
        }
      const int e = pow2_exponent(group4_max(mx));
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          el[0][t][i] = T(ldexp(el[0][t][i], -e));
          el[1][t][i] = el[0][t][i];
        }
      sprev = s;
      const bool wide_next = (c + 1 < L) ? store_site(Bs[b ^ 1], true) : false;
      const int nt_next = __syncthreads_or(wide_next) ? RT : 1;
      if (c + 1 < L) {
        b ^= 1;
        nt = nt_next;
      }
    }
    b ^= 1;

    // ---- energy bookkeeping (one lane per proposal): unsatisfied bonds of row r and r-1, r ----
    if (q == 0) {
      for (int w = 0; w < W; ++w) {
        const uint64_t cw = crow[w * MF_PROP];
        const uint64_t nxt = (w + 1 < W) ? crow[(w + 1) * MF_PROP] : 0ull;
        const uint64_t right = (cw >> 1) | (nxt << 63);
        const int nb_h = (L - 1) - 64 * w;
        const uint64_t mh = nb_h >= 64 ? ~0ull : (nb_h > 0 ? ((1ull << nb_h) - 1) : 0ull);
        unsat += __popcll((cw ^ right ^ jh[w]) & mh);
        if (r > 0) {
          const int nb_v = L - 64 * w;
          const uint64_t mv = nb_v >= 64 ? ~0ull : ((1ull << nb_v) - 1);
          unsat += __popcll((prow[w * MF_PROP] ^ cw ^ jv[w]) & mv);
        }
      }
      if (active && !teacher) {
        uint64_t* so = spins_out + ((size_t(ri) * K + k) * Lmax + r) * Wmax;
        for (int w = 0; w < Wmax; ++w) so[w] = (w < W) ? crow[w * MF_PROP] : 0ull;
      }
    }
    pr ^= 1;
  }
  if (active && q == 0) {
    const double lq = log(qprod) + double(qexp) * 0.69314718055994530942;
    logq_out[size_t(ri) * K + k] = lq;
    if (!isfinite(lq)) stb |= TNMC_ST_LOGQ;
    if (nfb) stb |= TNMC_ST_FALLBACK;
    if (R.status != nullptr && stb != 0) atomicOr(R.status, stb);
    if (!teacher) {
      E_out[size_t(ri) * K + k] = 2 * unsat - 2 * L * (L - 1);
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
                          double* d_logq, int32_t* d_E, uint32_t* d_fallbacks, int waves,
                          hipStream_t stream) {
  if constexpr (CHI % 16 == 0) {
    auto go = [&](auto wc) {
      constexpr int WAVES = decltype(wc)::value;
      dim3 grid((K + 16 * WAVES - 1) / (16 * WAVES), n);
      hipLaunchKernelGGL((propose_mfma_kernel<T, E, CHI, WAVES>), grid, dim3(64 * WAVES), 0, stream,
                         d_reals, K, Lmax, seed, first, d_teacher, d_spins, d_logq, d_E, d_fallbacks);
    };
    if (waves <= 0) waves = propose_default_waves(CHI, n, K, Lmax);
    switch (waves) {
      case 1: go(std::integral_constant<int, 1>{}); break;
      case 2: go(std::integral_constant<int, 2>{}); break;
      case 4: go(std::integral_constant<int, 4>{}); break;
      case 8: go(std::integral_constant<int, 8>{}); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    dim3 grid((K + PROP_NT - 1) / PROP_NT, n);
    hipLaunchKernelGGL((propose_kernel<T, E, CHI>), grid, dim3(PROP_NT), 0, stream, d_reals, K,
                       Lmax, seed, first, d_teacher, d_spins, d_logq, d_E, d_fallbacks);
  }
  return hipGetLastError();
}

hipError_t propose(tnmc_precision prec, int chi, const DevReal* d_reals, int n, int K, int Lmax,
                   uint64_t seed, uint64_t first, const uint64_t* d_teacher, uint64_t* d_spins,
                   double* d_logq, int32_t* d_E, uint32_t* d_fallbacks, int waves,
                   hipStream_t stream) {
#define TNMC_PROP_CASE(TY, EY, C)                                                               \
  case C:                                                                                       \
    return launch_propose<TY, EY, C>(d_reals, n, K, Lmax, seed, first, d_teacher, d_spins,      \
                                     d_logq, d_E, d_fallbacks, waves, stream);
#define TNMC_PROP_CHIS(TY, EY) \
  TNMC_PROP_CASE(TY, EY, 2) TNMC_PROP_CASE(TY, EY, 4) TNMC_PROP_CASE(TY, EY, 8) \
  TNMC_PROP_CASE(TY, EY, 16) TNMC_PROP_CASE(TY, EY, 32)
  if (prec == TNMC_FP64) {
    switch (chi) { TNMC_PROP_CHIS(double, double) }
  } else if (prec == TNMC_FP32) {
    switch (chi) {
      TNMC_PROP_CHIS(float, float) TNMC_PROP_CASE(float, float, 48) TNMC_PROP_CASE(float, float, 64)
    }
  } else if (prec == TNMC_BF16) {
    switch (chi) {
      TNMC_PROP_CHIS(float, bf16_t) TNMC_PROP_CASE(float, bf16_t, 48)
      TNMC_PROP_CASE(float, bf16_t, 64)
    }
  }
#undef TNMC_PROP_CHIS
#undef TNMC_PROP_CASE
  return hipErrorInvalidValue;
}

size_t propose_scratch_bytes(tnmc_precision prec, int chi, int L, int K) {
  static_assert(MF_MAX_PROP % PROP_NT == 0, "one padding serves both forms");
  const size_t elem = (prec == TNMC_FP64) ? 8 : 4;
  const size_t kpad = size_t(K + MF_MAX_PROP - 1) / MF_MAX_PROP * MF_MAX_PROP;
  return size_t(L) * 2 * chi * kpad * elem;   // V_c(y) of one row for every proposal
}

}  // namespace tnmc
