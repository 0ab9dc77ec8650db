// Boundary-MPS environment build (Sec. II B of arXiv:2409.06538): row-transfer MPO applied to
// an MPS, then canonical SVD compression back to bond dimension CHI.
//
// One workgroup owns one realization and walks its rows r = L-1 .. 1 (the bottom environment
// E_{r-1} needs E_r).  Per row:
//   QR sweep, c = 0 .. L-1: M_c = R_{c-1} At_c, where At_c is the site tensor of the row operator
//     applied to E_r (left bond (a, alpha), physical x, right bond (b, alpha')),
//       At_c[(a,alpha), x, (b,alpha')] = wh(a,b) wv(x,b) A_c[b][alpha][alpha'],
//     built on the fly from two coupling bits; M_c (4 CHI x 2 CHI) is factorised by Householder
//     QR; Q_c goes to global scratch, R_c (rescaled by a power of two) is carried.
//   SVD sweep, c = L-1 .. 1: T_c = Q_c X_{c+1} viewed as (2 CHI) x (2 x CHI); its right singular
//     subspace is found by QR with column pivoting (stopping at the numerical rank) followed by
//     one-sided Jacobi on the rows of the triangular factor; the CHI leading right singular
//     vectors become site c of E_{r-1}, and X_c = T_c V_k is carried left.
//   Site 0 keeps the norm, which is divided out: lambda_{r-1} = lambda_r + (power-of-two
//   exponents) ln 2 + ln ||A_0||.
// This reaches the same truncated state as the textbook QR-then-SVD sweep: every kept subspace is
// the span of the CHI leading right singular vectors of the same matrix.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace tnmc {

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<double> {
  // rotate a row pair while |c| > tol * ||T||_F * max(|row_p|, |row_q|)
  static constexpr double rot = 1e-14;
  // columns whose remaining norm is below rank * ||T||_F are dropped by the pivoted QR
  static constexpr double rank = 1e-15;
  // a kept row whose Cholesky pivot (squared residual norm) falls below eta is dependent
  static constexpr double eta = 1e-12;
};
template <>
struct JacobiTol<float> {
  static constexpr float rot = 2e-6f;
  static constexpr float rank = 3e-7f;
  static constexpr float eta = 1e-5f;
};

// Orthonormalise rows 0..k-1 of V (row stride ldv, n columns) in place by Cholesky QR applied
// twice; G (k x (CHI+1) workspace) holds the Gram matrix and then its Cholesky factor.  Rows are
// processed in order; a row whose pivot falls below eta lies in the span of the earlier rows (to
// rounding) and is set to zero.  The span of the surviving rows is unchanged.
template <typename T, int CHI, int NT>
__device__ void cholqr2_rows(T* V, int ldv, int n, int k, T* G, T eta) {
  constexpr int LDG = CHI + 1;
  const int tid = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
    for (int o = tid; o < k * k; o += NT) {
      const int a = o / k, b = o % k;
      if (b <= a) {
        T d = 0;
        for (int j = 0; j < n; ++j) d += V[a * ldv + j] * V[b * ldv + j];
        G[a * LDG + b] = d;
      }
    }
    __syncthreads();
    if (tid < WAVE) {
      for (int a = 0; a < k; ++a) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const T piv = G[a * LDG + a];
        const bool alive = piv > eta;
        const T l = alive ? sqrt(piv) : T(1);
        for (int i = a + 1 + tid; i < k; i += WAVE) G[i * LDG + a] = alive ? G[i * LDG + a] / l : T(0);
        if (tid == 0) G[a * LDG + a] = alive ? l : T(0);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int m = k - a - 1;
        for (int o = tid; o < m * m; o += WAVE) {
          const int i = a + 1 + o / m, j = a + 1 + o % m;
          if (j <= i) G[i * LDG + j] -= G[i * LDG + a] * G[j * LDG + a];
        }
      }
    }
    __syncthreads();
    for (int j = tid; j < n; j += NT) {
      for (int a = 0; a < k; ++a) {
        const T laa = G[a * LDG + a];
        T v = V[a * ldv + j];
        for (int b = 0; b < a; ++b) v -= G[a * LDG + b] * V[b * ldv + j];
        V[a * ldv + j] = (laa > T(0)) ? v / laa : T(0);
      }
    }
  }
  __syncthreads();
}

constexpr int MAX_SWEEPS = 40;

__host__ __device__ constexpr int env_threads(int chi) { return (8 * chi < 64) ? 64 : 8 * chi; }

// Shared-memory carve-up for one workgroup.
template <typename T, int CHI>
struct EnvSmem {
  static constexpr int N2 = 2 * CHI;     // bond of the operator-applied MPS; SVD matrix side
  static constexpr int MQ = 4 * CHI;     // rows of the QR-sweep matrix
  static constexpr int LDA = MQ + 1;     // column stride of M / Q
  static constexpr int LDT = N2 + 1;     // column stride of T, T0, R, X; row stride of J
  static constexpr int NT = env_threads(CHI);
  static constexpr size_t bufA = size_t(2) * N2 * LDT > size_t(LDA) * N2 ? size_t(2) * N2 * LDT
                                                                         : size_t(LDA) * N2;
  static constexpr size_t bufR = size_t(N2) * LDT;
  static constexpr size_t bufS = size_t(2) * CHI * CHI;
  static constexpr size_t reals = bufA + bufR + bufS + 3 * N2 + NT / 64 + 8;
  static constexpr size_t ints = 2 * N2 + 8 + 1024;
  static constexpr size_t bytes = reals * sizeof(T) + ints * sizeof(int);
};

template <typename T>
__device__ __forceinline__ T bond_weight(const uint64_t* row_bits, int c, int sa, int sb, T ep,
                                         T em) {
  // exp(beta J s_a s_b): J = -1 iff bit c is set; spins index 0 <-> +1, 1 <-> -1.
  const bool af = (row_bits[c >> 6] >> (c & 63)) & 1ull;
  const bool parallel = (sa == sb);
  return (parallel != af) ? ep : em;
}

template <typename T, int CHI>
__global__ __launch_bounds__(env_threads(CHI)) void env_build_kernel(const DevReal* reals,
                                                                     double* lnZ_out) {
  using S = EnvSmem<T, CHI>;
  constexpr int N2 = S::N2, MQ = S::MQ, LDA = S::LDA, LDT = S::LDT, NT = S::NT;
  constexpr int EPT = (N2 + 7) / 8;   // elements per thread of a Jacobi row
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* bufA = reinterpret_cast<T*>(smem_raw);
  T* bufR = bufA + S::bufA;
  T* bufS = bufR + S::bufR;
  T* cn2 = bufS + S::bufS;          // N2 column norms^2
  T* sc = cn2 + N2;                 // 2 N2 scalars scratch
  T* red = sc + 2 * N2;             // NT/64
  T* misc = red + NT / 64;          // 8
  int* perm = reinterpret_cast<int*>(misc + 8);   // N2
  int* ord = perm + N2;                           // N2
  int* imisc = ord + N2;                          // 8
  int* rexp = imisc + 8;                          // MAX_L exponents of the carried R_c

  const int tid = threadIdx.x;
  const DevReal R = reals[blockIdx.x];
  const int L = R.L;
  const int W = words_per_row(L);
  const T ep = T(exp(R.beta)), em = T(exp(-R.beta));
  T* env = reinterpret_cast<T*>(R.env);
  T* rs = reinterpret_cast<T*>(R.ws);                 // L x N2 x N2 scratch: R_c column-major
  const size_t site = size_t(2) * CHI * CHI;
  const size_t rowst = site * L;
  T* Zb = bufA;                      // Z_c: N2 x N2 column-major (rows (a,alpha), cols (x,beta))
  T* Tw = bufA + size_t(N2) * LDT;   // T_c: N2 x N2 column-major

  // E_{L-1} = 1: every site is 1/sqrt(2) at [sigma][0][0].
  for (size_t e = tid; e < rowst; e += NT) {
    const size_t inner = e % site;
    const int a = int((inner % (CHI * CHI)) / CHI), b = int(inner % CHI);
    env[size_t(L - 1) * rowst + e] = (a == 0 && b == 0) ? T(0.70710678118654752440) : T(0);
  }
  double lambda = 0.5 * double(L) * 0.69314718055994530942;
  if (tid == 0) R.lognorm[L - 1] = lambda;

  for (int r = L - 1; r >= 1; --r) {
    const T* Ain = env + size_t(r) * rowst;
    T* Aout = env + size_t(r - 1) * rowst;
    const uint64_t* jh = R.Jh + size_t(r) * W;        // horizontal bonds of row r
    const uint64_t* jv = R.Jv + size_t(r - 1) * W;    // vertical bonds between rows r-1 and r
    long long log2acc = 0;

    // ---------------- left-to-right: R factors only ----------------
    // M_c = R_{c-1} At_c (rows (i,x), cols (b,ap)); R_c = R factor of M_c, rescaled by 2^-e_c.
    for (int c = 0; c < L - 1; ++c) {
      __syncthreads();
      for (int e = tid; e < int(site); e += NT) bufS[e] = Ain[size_t(c) * site + e];
      __syncthreads();
      T wv[2][2], wh[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int b = 0; b < 2; ++b) wv[x][b] = bond_weight<T>(jv, c, x, b, ep, em);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) wh[a][b] = (c > 0) ? bond_weight<T>(jh, c - 1, a, b, ep, em) : T(0);
      for (int o = tid; o < N2 * N2; o += NT) {
        const int i = o % N2;
        const int col = o / N2;
        const int b = col / CHI, ap = col % CHI;
        T d = 0;
        if (c == 0) {
          d = (i < CHI) ? bufS[(b * CHI + i) * CHI + ap] : T(0);
        } else {
          const T wa = wh[0][b], wb = wh[1][b];
#pragma unroll 8
          for (int al = 0; al < CHI; ++al) {
            const T p = bufR[al * LDT + i] * wa + bufR[(CHI + al) * LDT + i] * wb;
            d += p * bufS[(b * CHI + al) * CHI + ap];
          }
        }
        bufA[col * LDA + i * 2 + 0] = wv[0][b] * d;
        bufA[col * LDA + i * 2 + 1] = wv[1][b] * d;
      }
      __syncthreads();
      // Householder QR of M (MQ x N2); only R is kept, so reflectors are not stored.
      for (int j = 0; j < N2; ++j) {
        if (tid < WAVE) {
          T ss = 0;
          for (int i = j + 1 + tid; i < MQ; i += WAVE) {
            const T v = bufA[j * LDA + i];
            ss += v * v;
          }
          ss = wave_sum(ss);
          if (tid == 0) {
            const T alpha = bufA[j * LDA + j];
            T t = 0, beta = alpha, scal = 0;
            if (ss > T(0)) {
              beta = -copysign(sqrt(alpha * alpha + ss), alpha);
              t = (beta - alpha) / beta;
              scal = T(1) / (alpha - beta);
            }
            misc[0] = beta;
            misc[1] = scal;
            misc[3] = t;
          }
        }
        __syncthreads();
        const T t = misc[3], scal = misc[1];
        if (t != T(0)) {
          const int k = j + 1 + tid / 4;
          const int part = tid % 4;
          const bool act = (k < N2);
          T w = 0;
          if (act) {
            if (part == 0) w = bufA[k * LDA + j];
            for (int i = j + 1 + part; i < MQ; i += 4) w += bufA[j * LDA + i] * scal * bufA[k * LDA + i];
          }
          w += __shfl_xor(w, 1);
          w += __shfl_xor(w, 2);
          if (act) {
            const T tw = t * w;
            if (part == 0) bufA[k * LDA + j] -= tw;
            for (int i = j + 1 + part; i < MQ; i += 4) bufA[k * LDA + i] -= tw * bufA[j * LDA + i] * scal;
          }
        }
        __syncthreads();
        if (tid == 0) bufA[j * LDA + j] = misc[0];
      }
      __syncthreads();
      // carry R (upper triangle) with a power-of-two rescale; keep it for the second sweep
      T mx = 0;
      for (int o = tid; o < N2 * N2; o += NT) {
        const int i = o % N2, k = o / N2;
        if (i <= k) mx = fmax(mx, fabs(bufA[k * LDA + i]));
      }
      mx = block_max<NT>(mx, red);
      const int e = pow2_exponent(mx);
      log2acc += e;
      if (tid == 0) rexp[c] = e;
      T* rdst = rs + size_t(c) * N2 * N2;
      for (int o = tid; o < N2 * N2; o += NT) {
        const int i = o % N2, k = o / N2;
        const T v = (i <= k) ? T(ldexp(bufA[k * LDA + i], -e)) : T(0);
        bufR[k * LDT + i] = v;
        rdst[o] = v;
      }
    }

    // ---------------- right-to-left: truncation ----------------
    // Carried Xt (N2 x CHI, column-major in bufR) with X_{c+1} = R_c Xt.  For the last site the
    // right bond is summed, which is Xt[(b, 0)][0] = 1 for both b.
    __syncthreads();
    for (int o = tid; o < N2 * LDT; o += NT) bufR[o] = T(0);
    __syncthreads();
    if (tid == 0) { bufR[0 * LDT + 0] = T(1); bufR[0 * LDT + CHI] = T(1); }
    for (int c = L - 1; c >= 0; --c) {
      __syncthreads();
      for (int e = tid; e < int(site); e += NT) bufS[e] = Ain[size_t(c) * site + e];
      __syncthreads();
      T wv[2][2], wh[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int b = 0; b < 2; ++b) wv[x][b] = bond_weight<T>(jv, c, x, b, ep, em);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          wh[a][b] = (c > 0) ? bond_weight<T>(jh, c - 1, a, b, ep, em) : (a == 0 ? T(1) : T(0));
      // P_b = A_c[b] Xt_b (CHI x CHI each) into sc-free registers, then
      // Z[(a,al)][(x,be)] = sum_b wh(a,b) wv(x,b) P_b[al][be]
      for (int o = tid; o < CHI * CHI; o += NT) {
        const int al = o % CHI, be = o / CHI;
        T p0 = 0, p1 = 0;
#pragma unroll 8
        for (int ap = 0; ap < CHI; ++ap) {
          p0 += bufS[(0 * CHI + al) * CHI + ap] * bufR[be * LDT + ap];
          p1 += bufS[(1 * CHI + al) * CHI + ap] * bufR[be * LDT + CHI + ap];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int x = 0; x < 2; ++x)
            Zb[(x * CHI + be) * LDT + a * CHI + al] = wh[a][0] * wv[x][0] * p0 + wh[a][1] * wv[x][1] * p1;
      }
      __syncthreads();
      if (c == 0) {
        // site 0: the left bond is (a = 0, alpha = 0); A_0[x][0][be] = Z[(0,0)][(x,be)]
        T part = 0;
        for (int o = tid; o < 2 * CHI; o += NT) {
          const T d = Zb[o * LDT + 0];
          sc[o] = d;
          part += d * d;
        }
        const T nrm2 = block_sum<NT>(part, red);
        const T nrm = sqrt(nrm2);
        for (int o = tid; o < int(site); o += NT) {
          const int x = o / (CHI * CHI), al = (o / CHI) % CHI, be = o % CHI;
          Aout[o] = (al == 0 && nrm > T(0)) ? sc[x * CHI + be] / nrm : T(0);
        }
        lambda += double(log2acc) * 0.69314718055994530942 + log(double(nrm));
        if (tid == 0) R.lognorm[r - 1] = lambda;
        break;
      }
      // R_{c-1} into bufR (Xt is no longer needed), then T = R_{c-1} Z (upper triangular R)
      const T* rsrc = rs + size_t(c - 1) * N2 * N2;
      for (int o = tid; o < N2 * N2; o += NT) bufR[(o / N2) * LDT + (o % N2)] = rsrc[o];
      __syncthreads();
      for (int o = tid; o < N2 * N2; o += NT) {
        const int i = o % N2, col = o / N2;
        T d = 0;
        for (int a = i; a < N2; ++a) d += bufR[a * LDT + i] * Zb[col * LDT + a];
        Tw[col * LDT + i] = d;
      }
      __syncthreads();
      // column norms, Frobenius norm
      for (int k = tid; k < N2; k += NT) {
        T s2 = 0;
        for (int i = 0; i < N2; ++i) s2 += Tw[k * LDT + i] * Tw[k * LDT + i];
        cn2[k] = s2;
        perm[k] = k;
      }
      __syncthreads();
      T fro2 = 0;
      for (int k = 0; k < N2; ++k) fro2 += cn2[k];
      const T tolr2 = JacobiTol<T>::rank * JacobiTol<T>::rank * fro2;

      // QR with column pivoting; stops at the numerical rank
      int rank = N2;
      for (int j = 0; j < N2; ++j) {
        if (tid < WAVE) {
          T best = -1;
          int bi = j;
          for (int k = j + tid; k < N2; k += WAVE) {
            const T v = cn2[k];
            if (v > best) { best = v; bi = k; }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const T ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
          }
          if (tid == 0) { imisc[0] = bi; misc[2] = best; }
        }
        __syncthreads();
        if (!(misc[2] > tolr2)) { rank = j; break; }
        const int piv = imisc[0];
        if (piv != j) {
          for (int i = tid; i < N2; i += NT) {
            const T a = Tw[j * LDT + i];
            Tw[j * LDT + i] = Tw[piv * LDT + i];
            Tw[piv * LDT + i] = a;
          }
          if (tid == 0) {
            const T a = cn2[j]; cn2[j] = cn2[piv]; cn2[piv] = a;
            const int p = perm[j]; perm[j] = perm[piv]; perm[piv] = p;
          }
        }
        __syncthreads();
        if (tid < WAVE) {
          T ss = 0;
          for (int i = j + 1 + tid; i < N2; i += WAVE) {
            const T v = Tw[j * LDT + i];
            ss += v * v;
          }
          ss = wave_sum(ss);
          if (tid == 0) {
            const T alpha = Tw[j * LDT + j];
            T t = 0, beta = alpha, scal = 0;
            if (ss > T(0)) {
              beta = -copysign(sqrt(alpha * alpha + ss), alpha);
              t = (beta - alpha) / beta;
              scal = T(1) / (alpha - beta);
            }
            misc[0] = beta;
            misc[1] = scal;
            misc[3] = t;
          }
        }
        __syncthreads();
        {
          const T t = misc[3], scal = misc[1];
          const int k = j + 1 + tid / 4;
          const int part = tid % 4;
          const bool act = (k < N2);
          T w = 0;
          if (act && t != T(0)) {
            if (part == 0) w = Tw[k * LDT + j];
            for (int i = j + 1 + part; i < N2; i += 4) w += Tw[j * LDT + i] * scal * Tw[k * LDT + i];
          }
          w += __shfl_xor(w, 1);
          w += __shfl_xor(w, 2);
          T nn = 0;
          if (act) {
            const T tw = t * w;
            if (part == 0) Tw[k * LDT + j] -= tw;
            for (int i = j + 1 + part; i < N2; i += 4) {
              const T v = Tw[k * LDT + i] - tw * Tw[j * LDT + i] * scal;
              Tw[k * LDT + i] = v;
              nn += v * v;
            }
          }
          nn += __shfl_xor(nn, 1);
          nn += __shfl_xor(nn, 2);
          if (act && part == 0) cn2[k] = nn;
        }
        __syncthreads();
        if (tid == 0) Tw[j * LDT + j] = misc[0];
        __syncthreads();
      }

      // J = rows 0..rank-1 of R (row-major in bufR, ld LDT); one zero row if rank is odd
      const int nr = rank + (rank & 1);
      for (int o = tid; o < nr * N2; o += NT) {
        const int i = o / N2, k = o % N2;
        bufR[i * LDT + k] = (i < rank && k >= i) ? Tw[k * LDT + i] : T(0);
      }
      __syncthreads();

      // one-sided Jacobi on the rows of J, parallel round-robin ordering
      if (nr >= 2) {
        const T scale = sqrt(fro2);
        const T tol = JacobiTol<T>::rot * scale;
        const int g = tid / 8, l = tid % 8;
        const int npair = nr / 2;
        for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
          int rotated = 0;
          for (int rd = 0; rd < nr - 1; ++rd) {
            if (g < npair) {
              int p, q;
              if (g == 0) { p = nr - 1; q = rd; }
              else { p = (rd + g) % (nr - 1); q = (rd - g + nr - 1) % (nr - 1); }
              T xp[EPT], xq[EPT];
              T a = 0, b = 0, cc = 0;
#pragma unroll
              for (int e = 0; e < EPT; ++e) {
                const int k = l + 8 * e;
                xp[e] = (k < N2) ? bufR[p * LDT + k] : T(0);
                xq[e] = (k < N2) ? bufR[q * LDT + k] : T(0);
                a += xp[e] * xp[e];
                b += xq[e] * xq[e];
                cc += xp[e] * xq[e];
              }
#pragma unroll
              for (int off = 1; off < 8; off <<= 1) {
                a += __shfl_xor(a, off);
                b += __shfl_xor(b, off);
                cc += __shfl_xor(cc, off);
              }
              if (a > T(0) && b > T(0) && fabs(cc) > tol * sqrt(fmax(a, b))) {
                const T zeta = (b - a) / (T(2) * cc);
                T t;
                if (fabs(zeta) > T(1e15)) t = T(0.5) / zeta;
                else t = copysign(T(1), zeta) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
                const T cs = T(1) / sqrt(T(1) + t * t);
                const T sn = cs * t;
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                  const int k = l + 8 * e;
                  if (k < N2) {
                    bufR[p * LDT + k] = cs * xp[e] - sn * xq[e];
                    bufR[q * LDT + k] = sn * xp[e] + cs * xq[e];
                  }
                }
                rotated = 1;
              }
            }
            __syncthreads();
          }
          if (!__syncthreads_or(rotated)) break;
        }
      }
      // row norms and descending order
      for (int i = tid; i < N2; i += NT) {
        T s2 = 0;
        if (i < rank)
          for (int k = 0; k < N2; ++k) s2 += bufR[i * LDT + k] * bufR[i * LDT + k];
        sc[i] = s2;
      }
      __syncthreads();
      for (int i = tid; i < rank; i += NT) {
        int pos = 0;
        for (int j2 = 0; j2 < rank; ++j2) pos += (sc[j2] > sc[i]) || (sc[j2] == sc[i] && j2 < i);
        ord[pos] = i;
      }
      __syncthreads();
      const int kept = rank < CHI ? rank : CHI;
      // V rows (CHI x N2) in bufS: V[al][perm[kk]] = J[ord[al]][kk] / sigma
      for (int o = tid; o < CHI * N2; o += NT) {
        const int al = o / N2, kk = o % N2;
        T v = 0;
        if (al < kept) {
          const int row = ord[al];
          const T s2 = sc[row];
          if (s2 > T(0)) v = bufR[row * LDT + kk] / sqrt(s2);
        }
        bufS[al * N2 + perm[kk]] = v;
      }
      // the kept rows span the right subspace but small ones are orthogonal to the large ones
      // only up to rot * ||T|| / sigma: make them orthonormal (span unchanged)
      cholqr2_rows<T, CHI, NT>(bufS, N2, N2, kept, bufR, T(JacobiTol<T>::eta));
      // site c of E_{r-1}: B[x][al][be] = V[al][x*CHI + be]
      T* bout = Aout + size_t(c) * site;
      for (int o = tid; o < int(site); o += NT) {
        const int x = o / (CHI * CHI), al = (o / CHI) % CHI, be = o % CHI;
        bout[o] = bufS[al * N2 + x * CHI + be];
      }
      // Xt_{c} = 2^-e_{c-1} Z V^T (N2 x CHI) into bufR (column-major, ld LDT), rescaled
      const int ec = rexp[c - 1];
      T mx = 0;
      for (int o = tid; o < N2 * CHI; o += NT) {
        const int j = o % N2, al = o / N2;
        T d = 0;
#pragma unroll 8
        for (int col = 0; col < N2; ++col) d += Zb[col * LDT + j] * bufS[al * N2 + col];
        d = T(ldexp(d, -ec));
        bufR[al * LDT + j] = d;
        mx = fmax(mx, fabs(d));
      }
      mx = block_max<NT>(mx, red);
      const int e = pow2_exponent(mx);
      log2acc += e;
      for (int o = tid; o < N2 * CHI; o += NT) {
        const int j = o % N2, al = o / N2;
        bufR[al * LDT + j] = T(ldexp(bufR[al * LDT + j], -e));
      }
      // clear the rows of Xt beyond CHI columns (bufR columns CHI.. hold nothing needed)
    }
    __syncthreads();
  }

  // ---------------- ln Z_TN from the top row ----------------
  if (lnZ_out != nullptr) {
    __syncthreads();
    const T* A0 = env;   // row 0
    const uint64_t* jh0 = R.Jh;
    for (int o = tid; o < 2 * CHI; o += NT) sc[o] = A0[(o / CHI) * CHI * CHI + (o % CHI)];
    double logacc = 0;
    for (int c = 1; c < L; ++c) {
      __syncthreads();
      const T* A = A0 + size_t(c) * site;
      T mx = 0;
      T val = 0;
      const int o = tid;
      if (o < 2 * CHI) {
        const int sp = o / CHI, be = o % CHI;
        for (int s2 = 0; s2 < 2; ++s2) {
          const T w = bond_weight<T>(jh0, c - 1, s2, sp, ep, em);
          T dd = 0;
          for (int al = 0; al < CHI; ++al) dd += sc[s2 * CHI + al] * A[(sp * CHI + al) * CHI + be];
          val += w * dd;
        }
        mx = fabs(val);
      }
      mx = block_max<NT>(mx, red);
      const int e = pow2_exponent(mx);
      logacc += double(e) * 0.69314718055994530942;
      if (o < 2 * CHI) sc[o] = T(ldexp(val, -e));
    }
    __syncthreads();
    if (tid == 0) {
      const double s = double(sc[0]) + double(sc[CHI]);
      lnZ_out[blockIdx.x] = lambda + logacc + log(s);
    }
  }
}

template <typename T, int CHI>
hipError_t launch_env_build(const DevReal* d_reals, int n, double* d_lnZ, hipStream_t stream) {
  using S = EnvSmem<T, CHI>;
  static_assert(S::NT >= 4 * (S::N2 - 1), "four threads per trailing column");
  static_assert(2 * CHI <= S::NT, "");
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&env_build_kernel<T, CHI>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(S::bytes));
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((env_build_kernel<T, CHI>), dim3(n), dim3(S::NT), S::bytes, stream, d_reals,
                     d_lnZ);
  return hipGetLastError();
}

template <typename T>
size_t env_build_smem_bytes(int chi) {
  switch (chi) {
    case 2: return EnvSmem<T, 2>::bytes;
    case 4: return EnvSmem<T, 4>::bytes;
    case 8: return EnvSmem<T, 8>::bytes;
    case 16: return EnvSmem<T, 16>::bytes;
    case 32: return EnvSmem<T, 32>::bytes;
    default: return 0;
  }
}

hipError_t env_build(tnmc_precision prec, int chi, const DevReal* d_reals, int n, double* d_lnZ,
                     hipStream_t stream) {
  if (prec == TNMC_FP64) {
    switch (chi) {
      case 2: return launch_env_build<double, 2>(d_reals, n, d_lnZ, stream);
      case 4: return launch_env_build<double, 4>(d_reals, n, d_lnZ, stream);
      case 8: return launch_env_build<double, 8>(d_reals, n, d_lnZ, stream);
      case 16: return launch_env_build<double, 16>(d_reals, n, d_lnZ, stream);
      case 32: return launch_env_build<double, 32>(d_reals, n, d_lnZ, stream);
    }
  } else {
    switch (chi) {
      case 2: return launch_env_build<float, 2>(d_reals, n, d_lnZ, stream);
      case 4: return launch_env_build<float, 4>(d_reals, n, d_lnZ, stream);
      case 8: return launch_env_build<float, 8>(d_reals, n, d_lnZ, stream);
      case 16: return launch_env_build<float, 16>(d_reals, n, d_lnZ, stream);
      case 32: return launch_env_build<float, 32>(d_reals, n, d_lnZ, stream);
    }
  }
  return hipErrorInvalidValue;
}

size_t env_build_scratch_bytes(tnmc_precision prec, int chi, int L) {
  const size_t elem = (prec == TNMC_FP64) ? 8 : 4;
  return size_t(L) * 2 * chi * 2 * chi * elem;   // the carried R factor of every site
}

}  // namespace tnmc
