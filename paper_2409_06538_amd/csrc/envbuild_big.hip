// Boundary-MPS environment build (Sec. II B of arXiv:2409.06538) in the Gram form with the
// per-site matrices in global memory: the row MPO applied to an MPS, then canonical compression
// back to CHI.  The build of CHI = 64, whose matrices do not fit in LDS; also selectable at
// CHI = 8 .. 48.
//
// One workgroup of 512 threads owns one realization and walks its rows r = L-1 .. 1.  With
// At_c[(a,al), x, (b,al')] = wh(a,b) wv(x,b) A_c[b][al][al'] the operator-applied site (never
// stored) and l, m the left and right bonds of site c of E_r:
//   left to right, c = 0 .. L-2: the Gram matrix of the left part, G_c = sum_x At_c(x)^T G_{c-1}
//     At_c(x), block (b, b'): kx(b,b') A_c[b]^T P_bb' A_c[b'] with P_bb' = sum_{a,a'} wh(a,b)
//     wh(a',b') G_{c-1}^{(a,a')} and kx(b,b') = sum_x wv(x,b) wv(x,b').  G_c = R_c^T R_c for the
//     R factor of the QR sweep of the canonical compression; it is stored per site (2m x 2m).
//   right to left, c = L-1 .. 1, carrying Xt (the kept right factor, rows (b, al')):
//     Z_c[(a,al), (x,be)] = sum_b wh(a,b) wv(x,b) (A_c[b] Xt^{(b)})[al][be],
//     H = Z_c^T G_{c-1} Z_c = T_c^T T_c for the SVD step's matrix T_c = R_{c-1} Z_c.  A pivoted
//     Cholesky of H, stopped at the numerical rank, gives the rows J of the R factor of the
//     pivoted QR of T_c: they span T_c's row space.  If the rank is at most CHI every direction is
//     kept and the rows of J are orthonormalised (Gram-Schmidt, twice); otherwise one-sided
//     Jacobi on the rows of J gives the singular directions and the CHI largest are kept.  The
//     kept rows V become site c of E_{r-1}; Xt_c = Z_c V^T, rescaled by a power of two.
//   site 0: Z_0 = sum_b wv(x,b) A_0[b] Xt^{(b)}, whose norm is divided out:
//     lambda_{r-1} = lambda_r + (sum of the exponents of Xt) ln 2 + ln ||Z_0||.
// The scale of G never enters (H only fixes V and the relative rank cut).  Arithmetic type T:
// float for bfloat16 environments, double for FP32 ones; products on 16x16x4 matrix-core tiles.
// The Gram matrices of a row, Z, W = G Z, the carried factors (and H in FP64) live in a
// per-realization global scratch that stays in L2; the site, H (FP32) and V are in LDS.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace tnmc {

namespace {

template <typename T>
struct BigTol;
// FP64 Gram matrices (FP32 environments): the cut of the other FP32 builds, singular values above
// 3e-7 of ||T_c||_F.
template <>
struct BigTol<double> {
  static constexpr double rank2 = 9e-14;   // pivots d > rank2 trace(H)
  static constexpr double rot = 2e-6;      // Jacobi: rotate while c^2 > rot^2 a b
  static constexpr double eta = 1e-5;      // Gram-Schmidt: residual^2 / norm^2 below: dependent
};
// FP32 Gram matrices (bfloat16 environments): rounding leaves H's smallest eigenvalues uncertain
// at about 1e-7 of its trace; pivots down to 1e-8 of the trace (singular values down to 1e-4 of
// ||T_c||_F) are kept.  Directions at that level are partly rounding, but every kept direction is
// orthonormalised, so they only widen the bond; cutting at 1e-6 or 1e-7 of the trace instead
// lowered the acceptance (0.21 and 0.45 against 0.64 on the L = 256, chi = 48 bfloat16 batch).
template <>
struct BigTol<float> {
  static constexpr float rank2 = 1e-8f;
  static constexpr float rot = 1e-5f;
  static constexpr float eta = 1e-5f;
};

constexpr int BIG_NT = 512;
constexpr int BIG_NW = BIG_NT / WAVE;
constexpr int BIG_MAX_SWEEPS = 40;

template <typename T>
struct MfmaTile;
template <>
struct MfmaTile<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 output tile held in register r of lane group q
  __device__ __forceinline__ static int row(int q, int r) { return 4 * q + r; }
};
template <>
struct MfmaTile<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int q, int r) { return q + 4 * r; }
};

// C = A B for M x K times K x N (runtime sizes up to 128) on 16x16x4 matrix-core tiles, the
// output tiles dealt to the wavefronts in turn.  fa(i, k) and fb(k, j) return the operands
// (zero outside the matrices), fs(i, j, v) stores an entry inside M x N.  Lane (i, q) feeds
// A(i, k0 + q) and B(k0 + q, j) and receives the rows MfmaTile::row(q, r) of column i.
// The tiles start at wavefront `wave0`, so that independent products issued one after the other
// without a barrier between them occupy different wavefronts.
template <typename T, typename FA, typename FB, typename FS>
__device__ __forceinline__ void big_gemm(int M, int N, int K, FA fa, FB fb, FS fs, int wave0 = 0) {
  using MT = MfmaTile<T>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  const int TM = (M + 15) >> 4, TN = (N + 15) >> 4;
  for (int t = (wv + BIG_NW - wave0 % BIG_NW) % BIG_NW; t < TM * TN; t += BIG_NW) {
    const int ti = t / TN, tj = t % TN;
    typename MT::v4 acc = {T(0), T(0), T(0), T(0)};
    // four k-steps per round: the operand loads are issued before the first product waits
    for (int k0 = 0; k0 < K; k0 += 16) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = fa(ti * 16 + i16, k0 + 4 * u + q);
        b[u] = fb(k0 + 4 * u + q, tj * 16 + i16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = MT::mac(a[u], b[u], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti * 16 + MT::row(q, r), j = tj * 16 + i16;
      if (i < M && j < N) fs(i, j, acc[r]);
    }
  }
}

}  // namespace

// LDS layout of the kernel (elements of T, then ints and bytes).
template <typename T, int CHI>
struct BigSmem {
  static constexpr int N2 = 2 * CHI;
  static constexpr int LDA = CHI + 1;            // staged site [b][al][be]
  static constexpr int LDH = N2 + 1;             // H and V rows
  static constexpr size_t sA = size_t(2) * CHI * LDA;
  // H in LDS whenever it fits beside the rest (FP32 always; FP64 up to CHI = 48)
  static constexpr size_t rest_bytes = (sA + size_t(CHI) * LDH + 2 * N2 + 4 * BIG_NW + 8) * sizeof(T) +
                                       (2 * N2 + 16) * sizeof(int) + 2 * 1028;
  static constexpr bool H_IN_LDS = rest_bytes + size_t(N2) * LDH * sizeof(T) <= 160 * 1024;
  // otherwise H of at most HS rows (ld HS + 1) borrows the V buffer (V is formed after H is read)
  static constexpr int hs_fit(int n) { return (n + 1) * (n + 2) <= CHI * LDH ? hs_fit(n + 1) : n; }
  static constexpr int HS = H_IN_LDS ? N2 : hs_fit(1);
  static constexpr size_t sH = H_IN_LDS ? size_t(N2) * LDH : 0;
  static constexpr size_t sV = size_t(CHI) * LDH;
  static constexpr size_t reals = sA + sH + sV + 2 * N2 + 4 * BIG_NW + 8;
  static constexpr size_t ints = 2 * N2 + 16;
  static constexpr size_t bytes = reals * sizeof(T) + ints * sizeof(int) + 2 * 1028;
};

// Per-realization global scratch (elements of T): L Gram matrices, then Z, W (also the first
// sweep's P and Q, the Y products and the Jacobi rows), the two carried factors, and H in FP64.
template <int CHI>
constexpr size_t big_block() {
  return size_t(2 * CHI) * (2 * CHI);
}

template <typename T, typename E, int CHI, bool ZIP, bool FLD>
__global__ __launch_bounds__(BIG_NT) void env_build_big_kernel(const DevReal* reals,
                                                               double* lnZ_out) {
  using S = BigSmem<T, CHI>;
  using Tol = BigTol<T>;
  constexpr int N2 = S::N2, LDA = S::LDA, LDH = S::LDH, NT = BIG_NT;
  constexpr size_t BLK = big_block<CHI>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sHl = sA + S::sA;
  T* sV = sHl + S::sH;
  T* vec = sV + S::sV;            // 2 N2: Z_0, norms
  T* red = vec + 2 * N2;          // 4 NW
  T* misc = red + 4 * BIG_NW;     // 8
  int* perm = reinterpret_cast<int*>(misc + 8);   // N2 pivot order
  int* ord = perm + N2;                           // N2 Jacobi row order
  int* imisc = ord + N2;                          // 16
  unsigned char* bdin = reinterpret_cast<unsigned char*>(imisc + 16);   // bonds of E_r
  unsigned char* bdout = bdin + 1028;                                    // bonds of E_{r-1}

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const DevReal R = reals[blockIdx.x];
  const int L = R.L;
  const T ep = T(exp(R.beta)), em = T(exp(-R.beta));
  gmem<E>* env = as_global(reinterpret_cast<E*>(R.env));
  gmem<double>* lognorm = as_global(R.lognorm);
  // the scratch in the global address space (global_load / global_store, counted by the
  // vector-memory counter only: FLAT accesses would also hold every LDS wait)
  gmem<T>* ws = as_global(reinterpret_cast<T*>(R.ws));
  gmem<T>* Gs = ws;                       // L blocks: G_c at Gs + c BLK, row-major, ld N2
  gmem<T>* Zs = ws + size_t(L) * BLK;     // Z_c (ld N2); first sweep: P_bb' (3 x CHI x CHI)
  gmem<T>* Ws = Zs + BLK;                 // W (ld N2); Y_b; first sweep: Q_bb'; Jacobi rows
  gmem<T>* Xs = Ws + BLK;                 // two carried factors, N2 x CHI each
  T* Hg = reinterpret_cast<T*>(R.ws) + size_t(L + 3) * BLK;   // H in global memory (FP64)
  const size_t site = size_t(2) * CHI * CHI;
  const size_t rowst = site * L;

  // exp(beta J s s') for the bond whose coupling bit is `af`; spin index 0 <-> +1, 1 <-> -1
  auto w = [&](bool af, int s, int t) { return ((s == t) != af) ? ep : em; };
  // site c of E_r -> sA[b][al][be], al < l, be < m, times the site's field weights exp(beta h b)
  auto stage = [&](const gmem<E>* src, int l, int m, int r, int c) {
    T g0, g1;
    site_field_t<FLD, T>(R, r, c, ep, em, g0, g1);
    for (int o = tid; o < 2 * l * m; o += NT) {
      const int b = o / (l * m), al = (o / m) % l, be = o % m;
      sA[(b * CHI + al) * LDA + be] = (b ? g1 : g0) * T(widen(gld<E>(src, (b * CHI + al) * CHI + be)));
    }
  };
  // Write one whole site (2 CHI^2 entries, the zero padding included) in 16-byte stores:
  // val(x, ka, be) gives the entry.  The padding is most of a site at CHI = 64 (bonds of a few to
  // a few tens), so the store count, not the arithmetic, sets the cost of this step.
  constexpr int PACK = 16 / int(sizeof(E));
  static_assert((2 * CHI * CHI) % PACK == 0 && CHI % PACK == 0, "whole 16-byte pieces");
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  auto write_site = [&](gmem<E>* dst, auto val) {
    gmem<u4v>* d4 = reinterpret_cast<gmem<u4v>*>(dst);
    for (int pc = tid; pc < 2 * CHI * CHI / PACK; pc += NT) {
      const int o = pc * PACK;
      const int x = o / (CHI * CHI), ka = (o / CHI) % CHI, be0 = o % CHI;
      E e[PACK];
#pragma unroll
      for (int u = 0; u < PACK; ++u) e[u] = narrow<E>(val(x, ka, be0 + u));
      u4v pk;
      __builtin_memcpy(&pk, e, 16);
      d4[pc] = pk;
    }
  };
  auto block_absmax = [&](T v) { return block_max<NT>(v, red); };

  // E_{L-1} = 1: every site 1/sqrt(2) for both spins, bonds 1
  for (int c = 0; c < L; ++c)
    write_site(env + size_t(L - 1) * rowst + size_t(c) * site, [&](int, int a, int b) {
      return (a == 0 && b == 0) ? T(0.70710678118654752440) : T(0);
    });
  double lambda = 0.5 * double(L) * 0.69314718055994530942;
  if (tid == 0) lognorm[L - 1] = lambda;
  for (int c = tid; c <= L; c += NT) {
    bdin[c] = 1;
    bdout[c] = 1;
    if (R.bonds != nullptr) R.bonds[size_t(L - 1) * (L + 1) + c] = 1;
  }
  __syncthreads();

  // H (nk x nk, symmetric, formed by fill_h(H, ldh)) -> the kept orthonormal rows of its
  // factor in sV (nk entries each); returns how many.  Pivoted Cholesky stopped at the
  // numerical rank, one-sided Jacobi and the CHI largest directions when the rank exceeds CHI,
  // Gram-Schmidt twice.  Shared by both sweep directions.
  // The small-H factorisation behind factor_rows (run by wavefront 0): rank and the kept rows
  // of V (orthonormal, in sV) from H (nk x nk, ld ldh, in LDS); the rank goes to imisc[0].
  auto small_factor = [&](auto gsize, const T* H, const int ldh, const int nk) {
    constexpr int G = decltype(gsize)::value;
    const int a = lane & (G - 1);
    const bool va = a < nk;
    T Lr[G];
#pragma unroll
    for (int u = 0; u < G; ++u) Lr[u] = T(0);
    T d = va ? H[a * ldh + a] : T(0);
    const T tol2 = T(Tol::rank2) * group_sum<G>(fmax(d, T(0)));
    bool pk = !va;
    int rk = nk;
    for (int j = 0; j < nk; ++j) {
      const uint32_t key =
          pk ? 0u : ((__float_as_uint(float(fmax(d, T(0)))) & ~127u) | uint32_t(127 - a));
      const uint32_t bk = group_max_u32<G>(key);
      const int piv = 127 - int(readlane_i(int(bk), 0) & 127);
      const T best = readlane_v(d, piv);
      if (readlane_i(int(bk), 0) == 0 || !(best > tol2)) {
        rk = j;
        break;
      }
      const T h = va ? H[a * ldh + piv] : T(0);
      const T inv = T(1) / sqrt(best);
      T dot = 0;   // entries j.. of both rows are still zero
#pragma unroll
      for (int g = 0; g < G; g += 4)
        if (g < j) {
#pragma unroll
          for (int u = 0; u < 4; ++u) dot += Lr[g + u] * readlane_v(Lr[g + u], piv);
        }
      const T l = (a == piv) ? best * inv : (!pk ? (h - dot) * inv : T(0));
#pragma unroll
      for (int i = 0; i < G; ++i) Lr[i] = (i == j) ? l : Lr[i];
      if (!pk && a != piv) d -= l * l;
      if (a == piv) pk = true;
    }
    // rows J[j][a] = Lr[j]: classical Gram-Schmidt, the projections of a pass taken from the
    // same vector, with a second pass only where the first removed more than half of the
    // squared norm (Kahan's "twice is enough" test: otherwise one pass leaves the row
    // orthogonal to working precision).  The 64 / G lane groups hold the same vector, so one
    // group sum gives 64 / G projections at once, group u taking row g + u.
    constexpr int P = 64 / G;
    const int slot = lane / G;
    for (int j = 0; j < rk; ++j) {
      T x = 0;
#pragma unroll
      for (int i = 0; i < G; ++i) x = (i == j) ? Lr[i] : x;
      const T n2 = group_sum<G>(x * x);
      T r2 = n2;
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        if (pass == 1 && readlane_v(r2, 0) > T(0.5) * readlane_v(n2, 0)) break;
        T acc = 0;
#pragma unroll
        for (int g = 0; g < G; g += P) {
          if (g < j) {
            T ls = Lr[g];
#pragma unroll
            for (int u = 1; u < P; ++u) ls = (slot == u) ? Lr[g + u] : ls;
            const T dv = group_sum<G>(g + slot < j ? x * ls : T(0));
#pragma unroll
            for (int u = 0; u < P; ++u) acc += readlane_v(dv, u * G) * Lr[g + u];   // 0 past j
          }
        }
        x -= acc;
        r2 = group_sum<G>(x * x);
      }
      const T sc = (n2 > T(0) && r2 > T(Tol::eta) * n2) ? T(1) / sqrt(r2) : T(0);
      x *= sc;
#pragma unroll
      for (int i = 0; i < G; ++i) Lr[i] = (i == j) ? x : Lr[i];
    }
    // H is dead (it may share the V buffer): this wavefront's reads of it are done
    if (lane < G && va)
#pragma unroll
      for (int i = 0; i < G; ++i)
        if (i < rk) sV[i * LDH + a] = Lr[i];
    if (lane == 0) imisc[0] = rk;
  };
  auto factor_rows = [&](const int nk, auto fill_h) -> int {
    // H in LDS (its own buffer, or the V buffer when it is small enough), else global memory
    const bool h_in_v = !S::H_IN_LDS && nk <= S::HS;
    T* H = S::H_IN_LDS ? sHl : (h_in_v ? sV : Hg);
    const int ldh = S::H_IN_LDS ? LDH : (h_in_v ? nk + 1 : N2);
    const bool h_global = !S::H_IN_LDS && !h_in_v;
    fill_h(H, ldh);
    __syncthreads();

    // ---- small H (nk <= G, G = 16 or 32, and nk <= CHI, so the rank cannot exceed CHI): one
    // wavefront holds the problem G lanes wide, replicated 64 / G times, with row `a` of the
    // Cholesky factor in registers of lane a from the factorisation through Gram-Schmidt; sums
    // and the pivot search are butterflies inside each group of G lanes (every lane gets the
    // result), the pivot row's entries come by readlane, and only H and the final rows of V
    // touch LDS.  Same steps and tolerances as the general path below. ----
    if (nk <= CHI && nk <= (sizeof(T) == 4 ? 32 : 16)) {
      if (wv == 0) {
        if (nk <= 16)
          small_factor(std::integral_constant<int, 16>{}, H, ldh, nk);
        else
          small_factor(std::integral_constant<int, 32>{}, H, ldh, nk);
      }
      __syncthreads();
      return int(imisc[0]);
    }

    // ---- pivoted Cholesky of H in place (one wavefront, rows lane and lane + 64) ----
    // Left-looking: with p_j the row of largest remaining diagonal d,
    //   L[a][j] = (H[a][p_j] - sum_{i<j} L[a][i] L[p_j][i]) / sqrt(d[p_j]),  d[a] -= L[a][j]^2,
    // and L[.][j] overwrites column p_j of H (no entry of that column is read again).
    if (wv == 0) {
      const int a0 = lane, a1 = lane + 64;
      const bool v0 = a0 < nk, v1 = a1 < nk;
      T d0 = v0 ? H[a0 * ldh + a0] : T(0), d1 = v1 ? H[a1 * ldh + a1] : T(0);
      const T tr = wave_sum(fmax(d0, T(0)) + fmax(d1, T(0)));
      const T tol2 = T(Tol::rank2) * tr;
      bool pk0 = !v0, pk1 = !v1;
      int rk = nk;
      for (int j = 0; j < nk; ++j) {
        const uint32_t key0 =
            pk0 ? 0u : ((__float_as_uint(float(fmax(d0, T(0)))) & ~127u) | uint32_t(127 - a0));
        const uint32_t key1 =
            pk1 ? 0u : ((__float_as_uint(float(fmax(d1, T(0)))) & ~127u) | uint32_t(127 - a1));
        const uint32_t bk = wave_max_u32(key0 > key1 ? key0 : key1);
        const int piv = 127 - int(bk & 127u);
        const T best = piv < 64 ? readlane_v(d0, piv) : readlane_v(d1, piv - 64);
        if (bk == 0u || !(best > tol2)) {
          rk = j;
          break;
        }
        const T inv = T(1) / sqrt(best);
        const T sq = best * inv;
        T dot0 = 0, dot1 = 0;
        for (int i = 0; i < j; ++i) {
          const int pc = perm[i];
          const T lp = H[piv * ldh + pc];
          dot0 += (v0 ? H[a0 * ldh + pc] : T(0)) * lp;
          dot1 += (v1 ? H[a1 * ldh + pc] : T(0)) * lp;
        }
        const T h0 = v0 ? H[a0 * ldh + piv] : T(0), h1 = v1 ? H[a1 * ldh + piv] : T(0);
        const T l0 = (a0 == piv) ? sq : (!pk0 ? (h0 - dot0) * inv : T(0));
        const T l1 = (a1 == piv) ? sq : (!pk1 ? (h1 - dot1) * inv : T(0));
        // (this step reads no entry of column piv after writing it: no wait before the writes)
        if (v0) H[a0 * ldh + piv] = l0;
        if (v1) H[a1 * ldh + piv] = l1;
        if (!pk0 && a0 != piv) d0 -= l0 * l0;
        if (!pk1 && a1 != piv) d1 -= l1 * l1;
        if (a0 == piv) pk0 = true;
        if (a1 == piv) pk1 = true;
        if (lane == 0) perm[j] = piv;
        if (h_global) __threadfence_block();   // the writes before the next step's reads
      }
      if (lane == 0) imisc[0] = rk;
    }
    __syncthreads();
    const int rank = imisc[0];
    int kept = rank < CHI ? rank : CHI;
    // J row j = column perm[j] of the factor: J[j][a] = H[a][perm[j]]
    if (rank > CHI) {
      // ---- one-sided Jacobi on the rows of J (rank x nk), then the CHI largest ----
      gmem<T>* Jr = Ws;   // rows, ld N2 (W is no longer needed)
      const int nr = rank + (rank & 1);
      for (int o = tid; o < nr * nk; o += NT) {
        const int j = o / nk, a = o % nk;
        Jr[j * N2 + a] = j < rank ? H[a * ldh + perm[j]] : T(0);
      }
      __syncthreads();
      constexpr int TPP = 8;   // threads per row pair
      const int g = tid / TPP, gl = tid % TPP, npair = nr / 2;
      for (int sweep = 0; sweep < BIG_MAX_SWEEPS; ++sweep) {
        int rotated = 0;
        for (int rd = 0; rd < nr - 1; ++rd) {
          for (int pg = g; pg < npair; pg += NT / TPP) {
            int p, qq;
            if (pg == 0) {
              p = nr - 1;
              qq = rd;
            } else {
              p = (rd + pg) % (nr - 1);
              qq = (rd - pg + nr - 1) % (nr - 1);
            }
            T aa = 0, bb = 0, cc = 0;
            for (int e = gl; e < nk; e += TPP) {
              const T xp = Jr[p * N2 + e], xq = Jr[qq * N2 + e];
              aa += xp * xp;
              bb += xq * xq;
              cc += xp * xq;
            }
            aa = group_sum<TPP>(aa);
            bb = group_sum<TPP>(bb);
            cc = group_sum<TPP>(cc);
            if (aa > T(0) && bb > T(0) && cc * cc > T(Tol::rot) * T(Tol::rot) * aa * bb) {
              // rotation zeroing the inner product of rows p and q
              const T zeta = (bb - aa) / (T(2) * cc);
              const T tt = (zeta >= T(0) ? T(1) : T(-1)) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
              const T cs = T(1) / sqrt(T(1) + tt * tt), sn = cs * tt;
              for (int e = gl; e < nk; e += TPP) {
                const T xp = Jr[p * N2 + e], xq = Jr[qq * N2 + e];
                Jr[p * N2 + e] = cs * xp - sn * xq;
                Jr[qq * N2 + e] = sn * xp + cs * xq;
              }
              rotated = 1;
            }
          }
          __syncthreads();
        }
        if (!__syncthreads_or(rotated)) break;
      }
      // row norms, then each row's place in decreasing order (ties: smaller index first)
      for (int j = tid; j < nr; j += NT) {
        T s = 0;
        for (int e = 0; e < nk; ++e) s += Jr[j * N2 + e] * Jr[j * N2 + e];
        vec[j] = j < rank ? s : T(-1);
      }
      __syncthreads();
      for (int j = tid; j < rank; j += NT) {
        int place = 0;
        for (int i = 0; i < rank; ++i) place += (vec[i] > vec[j] || (vec[i] == vec[j] && i < j));
        if (place < CHI) ord[place] = j;
      }
      __syncthreads();
      for (int o = tid; o < CHI * nk; o += NT) {
        const int kk = o / nk, a = o % nk;
        sV[kk * LDH + a] = Jr[ord[kk] * N2 + a];
      }
      kept = CHI;
    } else if (h_in_v) {
      // H occupies the V buffer: the rows of J pass through registers
      constexpr int PER = (CHI * S::HS + NT - 1) / NT;
      T tmp[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int o = tid + u * NT;
        if (o < kept * nk) tmp[u] = H[(o % nk) * ldh + perm[o / nk]];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int o = tid + u * NT;
        if (o < kept * nk) sV[(o / nk) * LDH + o % nk] = tmp[u];
      }
    } else {
      for (int o = tid; o < kept * nk; o += NT) {
        const int kk = o / nk, a = o % nk;
        sV[kk * LDH + a] = H[a * ldh + perm[kk]];
      }
    }
    __syncthreads();
    // ---- Gram-Schmidt on the kept rows, twice (one wavefront, entries lane and lane + 64) ----
    if (wv == 0) {
      const int a0 = lane, a1 = lane + 64;
      const bool v0 = a0 < nk, v1 = a1 < nk;
      for (int j = 0; j < kept; ++j) {
        T x0 = v0 ? sV[j * LDH + a0] : T(0), x1 = v1 ? sV[j * LDH + a1] : T(0);
        const T n2 = wave_sum(x0 * x0 + x1 * x1);
        // classical Gram-Schmidt, twice: the projections on the earlier rows are independent
        // reductions, taken four at a time
        for (int pass = 0; pass < 2; ++pass)
          for (int i0 = 0; i0 < j; i0 += 4) {
            T u0[4], u1[4], d[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + u < j ? i0 + u : j - 1;
              u0[u] = (v0 && i0 + u < j) ? sV[i * LDH + a0] : T(0);
              u1[u] = (v1 && i0 + u < j) ? sV[i * LDH + a1] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u] = wave_sum(x0 * u0[u] + x1 * u1[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              x0 -= d[u] * u0[u];
              x1 -= d[u] * u1[u];
            }
          }
        const T r2 = wave_sum(x0 * x0 + x1 * x1);
        const T s = (n2 > T(0) && r2 > T(Tol::eta) * n2) ? T(1) / sqrt(r2) : T(0);
        if (v0) sV[j * LDH + a0] = x0 * s;
        if (v1) sV[j * LDH + a1] = x1 * s;
      }
    }
    __syncthreads();
    return kept;
  };

  for (int r = L - 1; r >= 1; --r) {
    const gmem<E>* Ain = env + size_t(r) * rowst;
    gmem<E>* Aout = env + size_t(r - 1) * rowst;
    const gmem<const uint64_t>* jh = as_global(R.Jh) + size_t(r) * words_per_row(L);
    const gmem<const uint64_t>* jv = as_global(R.Jv) + size_t(r - 1) * words_per_row(L);
    auto hbit = [&](int c) { return bool((jh[c >> 6] >> (c & 63)) & 1ull); };   // bond (c, c+1)
    auto vbit = [&](int c) { return bool((jv[c >> 6] >> (c & 63)) & 1ull); };   // bond (r-1, r) at c

    // zip-up: one sweep per row, right to left on the first row applied, then alternating
    const bool rl = !ZIP || ((L - 1 - r) % 2 == 0);

    // ------------------------------ left to right: Gram matrices ------------------------------
    for (int c = 0; c <= L - 2 && !ZIP; ++c) {
      const int l = bdin[c], m = bdin[c + 1];
      stage(Ain + size_t(c) * site, l, m, r, c);
      const bool fv = vbit(c);
      T kx[2][2];
      for (int b = 0; b < 2; ++b)
        for (int b2 = 0; b2 < 2; ++b2) kx[b][b2] = w(fv, 0, b) * w(fv, 0, b2) + w(fv, 1, b) * w(fv, 1, b2);
      gmem<T>* P = Zs;   // P_bb' for (b, b') = (0,0), (0,1), (1,1): CHI x CHI each, ld CHI
      if (c > 0) {
        const bool fh = hbit(c - 1);
        const gmem<T>* Gp = Gs + size_t(c - 1) * BLK;
        for (int o = tid; o < 3 * l * l; o += NT) {
          const int pb = o / (l * l), al = (o / l) % l, be = o % l;
          const int b = pb == 2 ? 1 : 0, b2 = pb == 0 ? 0 : 1;
          T v = 0;
          for (int a = 0; a < 2; ++a)
            for (int a2 = 0; a2 < 2; ++a2)
              v += w(fh, a, b) * w(fh, a2, b2) * Gp[(a * l + al) * N2 + a2 * l + be];
          P[(pb * CHI + al) * CHI + be] = v;
        }
      }
      __syncthreads();
      // Q_bb' = P_bb' A_c[b'] (l x m)
      gmem<T>* Q = Ws;
      for (int pb = 0; pb < 3; ++pb) {
        const int b2 = pb == 0 ? 0 : 1;
        const gmem<T>* Pp = P + size_t(pb) * CHI * CHI;
        big_gemm<T>(
            l, m, l,
            [&](int i, int k) { return (i < l && k < l) ? (c > 0 ? Pp[i * CHI + k] : T(1)) : T(0); },
            [&](int k, int j) { return (k < l && j < m) ? sA[(b2 * CHI + k) * LDA + j] : T(0); },
            [&](int i, int j, T v) { Q[(pb * CHI + i) * CHI + j] = v; }, 3 * pb);
      }
      __syncthreads();
      // G_c^(b,b') = kx(b,b') A_c[b]^T Q_bb' (m x m); (1,0) is the transpose of (0,1)
      gmem<T>* Gc = Gs + size_t(c) * BLK;
      T mx = 0;
      for (int pb = 0; pb < 3; ++pb) {
        const int b = pb == 2 ? 1 : 0, b2 = pb == 0 ? 0 : 1;
        const gmem<T>* Qp = Q + size_t(pb) * CHI * CHI;
        const T k = kx[b][b2];
        big_gemm<T>(
            m, m, l,
            [&](int i, int kk) { return (i < m && kk < l) ? sA[(b * CHI + kk) * LDA + i] : T(0); },
            [&](int kk, int j) { return (kk < l && j < m) ? Qp[kk * CHI + j] : T(0); },
            [&](int i, int j, T v) {
              v *= k;
              Gc[(b * m + i) * N2 + b2 * m + j] = v;
              if (b != b2) Gc[(b2 * m + j) * N2 + b * m + i] = v;
              mx = fmax(mx, fabs(v));
            },
            3 * pb);
      }
      const int e = pow2_exponent(block_absmax(mx));   // contains the barriers
      for (int o = tid; o < 4 * m * m; o += NT) {
        const int i = o / (2 * m), j = o % (2 * m);
        Gc[i * N2 + j] = T(ldexp(Gc[i * N2 + j], -e));
      }
      __syncthreads();
    }

    // ------------------------------ right to left: SVD steps ------------------------------
    int xb = 0;          // carried factor in Xs + xb N2 CHI: rows (b, al') < 2m, columns < k
    int texp = 0;        // sum of the power-of-two exponents taken out of the carried factors
    if (rl) {
    for (int o = tid; o < 2; o += NT) Xs[o * CHI] = T(1);   // Xt_L: b summed (m = k = 1)
    __syncthreads();
    for (int c = L - 1; c >= 1; --c) {
      const int l = bdin[c], m = bdin[c + 1], k = bdout[c + 1];
      const bool fh = hbit(c - 1), fv = vbit(c);
      stage(Ain + size_t(c) * site, l, m, r, c);
      __syncthreads();
      const gmem<T>* X = Xs + size_t(xb) * N2 * CHI;
      // Z_c[(a,al),(x,be)] = sum_b wh(a,b) wv(x,b) (A_c[b] Xt^(b))[al][be], both b in one tile loop
      {
        using MT = MfmaTile<T>;
        const int i16 = lane & 15, q = lane >> 4;
        const int TM = (l + 15) >> 4, TN = (k + 15) >> 4;
        for (int t = wv; t < TM * TN; t += BIG_NW) {
          const int ti = t / TN, tj = t % TN;
          typename MT::v4 y0 = {T(0), T(0), T(0), T(0)}, y1 = y0;
          for (int k0 = 0; k0 < m; k0 += 16) {
            T a0[4], a1[4], b0[4], b1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = ti * 16 + i16, kk = k0 + 4 * u + q, j = tj * 16 + i16;
              const bool ok_a = i < l && kk < m, ok_b = kk < m && j < k;
              a0[u] = ok_a ? sA[(0 * CHI + i) * LDA + kk] : T(0);
              a1[u] = ok_a ? sA[(1 * CHI + i) * LDA + kk] : T(0);
              b0[u] = ok_b ? X[kk * CHI + j] : T(0);
              b1[u] = ok_b ? X[(m + kk) * CHI + j] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              y0 = MT::mac(a0[u], b0[u], y0);
              y1 = MT::mac(a1[u], b1[u], y1);
            }
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int al = ti * 16 + MT::row(q, rr), be = tj * 16 + i16;
            if (al < l && be < k)
              for (int a = 0; a < 2; ++a)
                for (int x = 0; x < 2; ++x)
                  Zs[(a * l + al) * N2 + x * k + be] =
                      w(fh, a, 0) * w(fv, x, 0) * y0[rr] + w(fh, a, 1) * w(fv, x, 1) * y1[rr];
          }
        }
      }
      __syncthreads();
      const int nz = 2 * l, nk = 2 * k;
      // W = G_{c-1} Z (nz x nk), then H = Z^T W (nk x nk, symmetric); the zip-up takes G = 1
      const gmem<T>* Wz = ZIP ? Zs : Ws;
      if (!ZIP) {
        const gmem<T>* Gp = Gs + size_t(c - 1) * BLK;
        big_gemm<T>(
            nz, nk, nz, [&](int i, int kk) { return (i < nz && kk < nz) ? Gp[i * N2 + kk] : T(0); },
            [&](int kk, int j) { return (kk < nz && j < nk) ? Zs[kk * N2 + j] : T(0); },
            [&](int i, int j, T v) { Ws[i * N2 + j] = v; });
        __syncthreads();
      }
      const int kept = factor_rows(nk, [&](T* H, int ldh) {
        big_gemm<T>(
            nk, nk, nz, [&](int i, int kk) { return (i < nk && kk < nz) ? Zs[kk * N2 + i] : T(0); },
            [&](int kk, int j) { return (kk < nz && j < nk) ? Wz[kk * N2 + j] : T(0); },
            [&](int i, int j, T v) { H[i * ldh + j] = v; });
      });
      // site c of E_{r-1}: A'[x][ka][be] = V[ka][x k + be]
      write_site(Aout + size_t(c) * site, [&](int x, int ka, int be) {
        return (ka < kept && be < k) ? sV[ka * LDH + x * k + be] : T(0);
      });
      if (tid == 0) bdout[c] = (unsigned char)kept;
      // Xt_c = Z V^T (nz x kept), rescaled by 2^-e
      gmem<T>* Xn = Xs + size_t(xb ^ 1) * N2 * CHI;
      T mx = 0;
      big_gemm<T>(
          nz, kept, nk, [&](int i, int kk) { return (i < nz && kk < nk) ? Zs[i * N2 + kk] : T(0); },
          [&](int kk, int j) { return (kk < nk && j < kept) ? sV[j * LDH + kk] : T(0); },
          [&](int i, int j, T v) {
            Xn[i * CHI + j] = v;
            mx = fmax(mx, fabs(v));
          });
      const int e = pow2_exponent(block_absmax(mx));
      for (int o = tid; o < nz * kept; o += NT) {
        const int i = o / kept, j = o % kept;
        Xn[i * CHI + j] = T(ldexp(Xn[i * CHI + j], -e));
      }
      texp += e;
      xb ^= 1;
      __syncthreads();
    }
    // ---- site 0: Z_0[(x,be)] = sum_b wv(x,b) (A_0[b] Xt^(b))[0][be]; its norm is divided out ----
    {
      const int m = bdin[1], k = bdout[1];
      const bool fv = vbit(0);
      stage(Ain, 1, m, r, 0);
      __syncthreads();
      const gmem<T>* X = Xs + size_t(xb) * N2 * CHI;
      T part = 0;
      for (int o = tid; o < 2 * k; o += NT) {
        const int x = o / k, be = o % k;
        T y0 = 0, y1 = 0;
        for (int g = 0; g < m; ++g) {
          y0 += sA[(0 * CHI) * LDA + g] * X[g * CHI + be];
          y1 += sA[(1 * CHI) * LDA + g] * X[(m + g) * CHI + be];
        }
        const T z = w(fv, x, 0) * y0 + w(fv, x, 1) * y1;
        vec[o] = z;
        part += z * z;
      }
      const T nrm = sqrt(block_sum<NT>(part, red));
      write_site(Aout, [&](int x, int al, int be) {
        return (al == 0 && be < k && nrm > T(0)) ? vec[x * k + be] / nrm : T(0);
      });
      lambda += double(texp) * 0.69314718055994530942 + log(double(nrm));
      if (tid == 0) {
        lognorm[r - 1] = lambda;
        bdout[0] = 1;
        bdout[L] = 1;
      }
    }
    } else {
    // ------------------------- zip-up, left to right (alternate rows) -------------------------
    // The carried factor C (rows kappa < k of the new left bond, columns (a, al) of the left bond
    // of the operator-applied site) is kept transposed in Xs: Ct[(a l + al) CHI + kappa].  At
    // site c: T_c[x k + kappa][b m + al'] = wv(x,b) sum_a wh(a,b) (C^(a) A_c[b])[kappa][al'];
    // its leading left singular directions (H = T T^T, factor_rows) become site c of E_{r-1}
    // (A'[x][kappa][kappa'] = V[kappa'][x k + kappa]) and C_c = V T_c is carried right.  The last
    // site sums b and takes the norm.
    if (tid == 0) Xs[0] = T(1);                        // C_{-1} = [1]: k = 1, no a
    __syncthreads();
    for (int c = 0; c <= L - 1; ++c) {
      const int l = bdin[c], m = bdin[c + 1], k = bdout[c];
      const bool fv = vbit(c);
      const bool fh = c > 0 ? hbit(c - 1) : false;
      stage(Ain + size_t(c) * site, l, m, r, c);
      __syncthreads();
      const gmem<T>* Ct = Xs + size_t(xb) * N2 * CHI;
      {
        using MT = MfmaTile<T>;
        const int i16 = lane & 15, q = lane >> 4;
        const int TM = (k + 15) >> 4, TN = (m + 15) >> 4;
        for (int t = wv; t < TM * TN; t += BIG_NW) {
          const int ti = t / TN, tj = t % TN;
          typename MT::v4 y0 = {T(0), T(0), T(0), T(0)}, y1 = y0;
          for (int k0 = 0; k0 < l; k0 += 16) {
            T a0[4], a1[4], b0[4], b1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int ka = ti * 16 + i16, al = k0 + 4 * u + q, j = tj * 16 + i16;
              const bool ok_a = ka < k && al < l, ok_b = al < l && j < m;
              const T c0 = ok_a ? Ct[al * CHI + ka] : T(0);                       // a = 0
              const T c1 = (ok_a && c > 0) ? Ct[(l + al) * CHI + ka] : T(0);      // a = 1
              a0[u] = c > 0 ? w(fh, 0, 0) * c0 + w(fh, 1, 0) * c1 : c0;          // P_0
              a1[u] = c > 0 ? w(fh, 0, 1) * c0 + w(fh, 1, 1) * c1 : c0;          // P_1
              b0[u] = ok_b ? sA[(0 * CHI + al) * LDA + j] : T(0);
              b1[u] = ok_b ? sA[(1 * CHI + al) * LDA + j] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              y0 = MT::mac(a0[u], b0[u], y0);
              y1 = MT::mac(a1[u], b1[u], y1);
            }
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int ka = ti * 16 + MT::row(q, rr), ap = tj * 16 + i16;
            if (ka < k && ap < m)
              for (int x = 0; x < 2; ++x) {
                Zs[(x * k + ka) * N2 + ap] = w(fv, x, 0) * y0[rr];
                Zs[(x * k + ka) * N2 + m + ap] = w(fv, x, 1) * y1[rr];
              }
          }
        }
      }
      __syncthreads();
      const int nr = 2 * k, nc = 2 * m;
      if (c == L - 1) {
        // last site: b summed (m = 1); its norm is divided out
        T part = 0;
        for (int o = tid; o < nr; o += NT) {
          const T z = Zs[o * N2 + 0] + Zs[o * N2 + 1];
          vec[o] = z;
          part += z * z;
        }
        const T nrm = sqrt(block_sum<NT>(part, red));
        write_site(Aout + size_t(c) * site, [&](int x, int ka, int be) {
          return (be == 0 && ka < k && nrm > T(0)) ? vec[x * k + ka] / nrm : T(0);
        });
        lambda += double(texp) * 0.69314718055994530942 + log(double(nrm));
        if (tid == 0) {
          lognorm[r - 1] = lambda;
          bdout[0] = 1;
          bdout[L] = 1;
        }
        break;
      }
      const int kept = factor_rows(nr, [&](T* H, int ldh) {
        big_gemm<T>(
            nr, nr, nc, [&](int i, int kk) { return (i < nr && kk < nc) ? Zs[i * N2 + kk] : T(0); },
            [&](int kk, int j) { return (kk < nc && j < nr) ? Zs[j * N2 + kk] : T(0); },
            [&](int i, int j, T v) { H[i * ldh + j] = v; });
      });
      // site c of E_{r-1}: A'[x][ka][ka'] = V[ka'][x k + ka]
      write_site(Aout + size_t(c) * site, [&](int x, int ka, int kp) {
        return (ka < k && kp < kept) ? sV[kp * LDH + x * k + ka] : T(0);
      });
      if (tid == 0) bdout[c + 1] = (unsigned char)kept;
      // C_c = V T_c (kept x nc), kept transposed, rescaled by 2^-e
      gmem<T>* Cn = Xs + size_t(xb ^ 1) * N2 * CHI;
      T mx = 0;
      big_gemm<T>(
          nc, kept, nr, [&](int i, int kk) { return (i < nc && kk < nr) ? Zs[kk * N2 + i] : T(0); },
          [&](int kk, int j) { return (kk < nr && j < kept) ? sV[j * LDH + kk] : T(0); },
          [&](int i, int j, T v) {
            Cn[i * CHI + j] = v;
            mx = fmax(mx, fabs(v));
          });
      const int e = pow2_exponent(block_absmax(mx));
      for (int o = tid; o < nc * kept; o += NT) {
        const int i = o / kept, j = o % kept;
        Cn[i * CHI + j] = T(ldexp(Cn[i * CHI + j], -e));
      }
      texp += e;
      xb ^= 1;
      __syncthreads();
    }
    }
    __syncthreads();
    if (R.bonds != nullptr)
      for (int c = tid; c <= L; c += NT) R.bonds[size_t(r - 1) * (L + 1) + c] = bdout[c];
    {   // the bonds of E_{r-1} are the input bonds of the next row
      unsigned char* t = bdin;
      bdin = bdout;
      bdout = t;
    }
  }
  if (tid == 0 && R.status != nullptr && !isfinite(lambda)) atomicOr(R.status, TNMC_ST_LOGNORM);

  // ---------------- ln Z_TN from the top row: sum_x H_0(x) E_0(x) ----------------
  if (lnZ_out != nullptr) {
    __syncthreads();
    const gmem<E>* A0 = env;
    const gmem<const uint64_t>* jh0 = as_global(R.Jh);
    T* sc = vec;   // 2 CHI: running vector v[sigma][be]
    // (row 0's fields, if any, weight each site of E_0 by exp(beta h s))
    {
      T g0, g1;
      site_field_t<FLD, T>(R, 0, 0, ep, em, g0, g1);
      for (int o = tid; o < 2 * CHI; o += NT)
        sc[o] = (o >= CHI ? g1 : g0) * T(widen(gld<E>(A0, (o / CHI) * CHI * CHI + (o % CHI))));
    }
    double logacc = 0;
    for (int c = 1; c < L; ++c) {
      __syncthreads();
      const gmem<E>* A = A0 + size_t(c) * site;
      const bool fh = bool((jh0[(c - 1) >> 6] >> ((c - 1) & 63)) & 1ull);
      T mxv = 0, val = 0;
      if (tid < 2 * CHI) {
        const int sp = tid / CHI, be = tid % CHI;
        T g0, g1;
        site_field_t<FLD, T>(R, 0, c, ep, em, g0, g1);
        for (int s2 = 0; s2 < 2; ++s2) {
          const T wgt = w(fh, s2, sp);
          T dd = 0;
          for (int al = 0; al < CHI; ++al) dd += sc[s2 * CHI + al] * T(widen(gld<E>(A, (sp * CHI + al) * CHI + be)));
          val += wgt * dd;
        }
        val *= sp ? g1 : g0;
        mxv = fabs(val);
      }
      mxv = block_max<NT>(mxv, red);
      const int e = pow2_exponent(mxv);
      logacc += double(e) * 0.69314718055994530942;
      __syncthreads();
      if (tid < 2 * CHI) sc[tid] = T(ldexp(val, -e));
    }
    __syncthreads();
    if (tid == 0) {
      const double s = double(sc[0]) + double(sc[CHI]);
      const double lz = lambda + logacc + log(s);
      lnZ_out[R.slot] = lz;
      if (R.status != nullptr && !isfinite(lz)) atomicOr(R.status, TNMC_ST_LOGNORM);
    }
  }
}

template <typename T, typename E, int CHI, bool ZIP, bool FLD>
hipError_t launch_env_build_big(const DevReal* d_reals, int n, double* d_lnZ, hipStream_t stream) {
  using S = BigSmem<T, CHI>;
  static_assert(S::bytes <= 160 * 1024, "LDS of one workgroup");
  constexpr int MAX_DEVICES = 64;
  static std::once_flag once[MAX_DEVICES];
  static hipError_t attr[MAX_DEVICES];
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::call_once(once[dev], [dev] {
    attr[dev] = hipFuncSetAttribute(reinterpret_cast<const void*>(&env_build_big_kernel<T, E, CHI, ZIP, FLD>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(S::bytes));
  });
  if (attr[dev] != hipSuccess) return attr[dev];
  hipLaunchKernelGGL((env_build_big_kernel<T, E, CHI, ZIP, FLD>), dim3(n), dim3(BIG_NT), S::bytes, stream,
                     d_reals, d_lnZ);
  return hipGetLastError();
}

int env_build_big_ok(tnmc_precision prec, int chi) {
  return (prec == TNMC_BF16 || prec == TNMC_FP32) &&
         (chi == 8 || chi == 16 || chi == 32 || chi == 48 || chi == 64);
}

hipError_t env_build_big(tnmc_precision prec, int chi, bool zipup, bool fields,
                         const DevReal* d_reals, int n, double* d_lnZ, hipStream_t stream) {
#define TNMC_BIG_LAUNCH(C, Z, F)                                                               \
  return prec == TNMC_BF16 ? launch_env_build_big<float, bf16_t, C, Z, F>(d_reals, n, d_lnZ, stream) \
                           : launch_env_build_big<double, float, C, Z, F>(d_reals, n, d_lnZ, stream);
#define TNMC_BIG_CASE(C)                                                                       \
  case C:                                                                                      \
    if (zipup) {                                                                               \
      if (fields) { TNMC_BIG_LAUNCH(C, true, true) }                                           \
      TNMC_BIG_LAUNCH(C, true, false)                                                          \
    }                                                                                          \
    if (fields) { TNMC_BIG_LAUNCH(C, false, true) }                                            \
    TNMC_BIG_LAUNCH(C, false, false)
  if (prec != TNMC_BF16 && prec != TNMC_FP32) return hipErrorInvalidValue;
  switch (chi) {
    TNMC_BIG_CASE(8)
    TNMC_BIG_CASE(16)
    TNMC_BIG_CASE(32)
    TNMC_BIG_CASE(48)
    TNMC_BIG_CASE(64)
  }
#undef TNMC_BIG_CASE
#undef TNMC_BIG_LAUNCH
  return hipErrorInvalidValue;
}

size_t env_build_big_scratch_bytes(tnmc_precision prec, int chi, int L) {
  const size_t elem = prec == TNMC_BF16 ? sizeof(float) : sizeof(double);
  return (size_t(L) + 4) * size_t(2 * chi) * (2 * chi) * elem;
}

}  // namespace tnmc
