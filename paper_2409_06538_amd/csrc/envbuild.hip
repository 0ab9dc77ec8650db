// Boundary-MPS environment build (Sec. II B of arXiv:2409.06538): the row-transfer MPO applied
// to an MPS, then canonical SVD compression back to bond dimension CHI.
//
// One workgroup owns one realization and walks its rows r = L-1 .. 1 (E_{r-1} needs E_r).  The
// operator-applied site tensor is never stored:
//   At_c[(a,alpha), x, (b,alpha')] = wh(a,b) wv(x,b) A_c[b][alpha][alpha'],
// with wh, wv the Boltzmann weights (Eq. (10)) of the horizontal bond (c-1, c) of row r and of the
// vertical bond between rows r-1 and r at column c.  Per row:
//   left to right, c = 0 .. L-2: M_c = R_{c-1} At_c (rows (i, x), columns (b, alpha')), whose R
//     factor R_c (Householder) is kept, rescaled by 2^-e_c.  This is the QR sweep of the canonical
//     compression with Q_c never formed.
//   right to left, c = L-1 .. 1: with X_{c+1} = R_c Xt_{c+1} the matrix of the SVD step is
//     T_c = Q_c X_{c+1} = R_{c-1} Z_c,  Z_c[(a,alpha), (x,beta)] = sum_b wh wv (A_c[b] Xt_b)[alpha][beta];
//     its CHI leading right singular vectors V become site c of E_{r-1}, and
//     Xt_c = 2^-e_{c-1} Z_c V^T.  The SVD step is QR with column pivoting (stopping at the numerical
//     rank), one-sided Jacobi on the rows of the triangular factor, and a Gram-Schmidt pass that
//     makes the kept rows exactly orthonormal.
//   site 0 keeps the norm, which is divided out: lambda_{r-1} = lambda_r + (sum of exponents) ln 2
//     + ln ||A_0||.
// Every matrix is held in LDS; GEMM-shaped products use register tiles; the factorisations use one
// workgroup barrier per column.
#include <hip/hip_runtime.h>

#include <mutex>

#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace tnmc {

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<double> {
  // rotate a row pair while |c| > rot * ||T||_F * max(|row_p|, |row_q|)
  static constexpr double rot = 1e-14;
  // columns whose remaining norm is below rank * ||T||_F are dropped by the pivoted QR
  static constexpr double rank = 1e-15;
  // a kept row whose Gram-Schmidt residual norm^2 falls below eta is dependent
  static constexpr double eta = 1e-12;
};
template <>
struct JacobiTol<float> {
  static constexpr float rot = 2e-6f;
  static constexpr float rank = 3e-7f;
  static constexpr float eta = 1e-5f;
};

// Tolerances follow the storage precision of the environments.
template <typename E>
struct TolOf {
  using type = E;
};
template <>
struct TolOf<bf16_t> {
  using type = float;
};

constexpr int MAX_SWEEPS = 40;
// 32 threads per unit of CHI, at most 512 (8 waves, two per SIMD, so that LDS and barrier latency
// of one wave overlaps with the other's work while each keeps 256 registers).
// (the largest multiple of both 64 and 2 CHI not above 512 when 32 CHI exceeds 512: 384 at CHI = 48)
__host__ __device__ constexpr int env_gcd(int a, int b) { return b == 0 ? a : env_gcd(b, a % b); }
__host__ __device__ constexpr int env_threads(int chi) {
  return (32 * chi < 64) ? 64
         : (32 * chi <= 512) ? 32 * chi
         : 512 / (64 * 2 * chi / env_gcd(64, 2 * chi)) * (64 * 2 * chi / env_gcd(64, 2 * chi));
}
// threads per column in the Householder updates (a power of two; NT = TPC * 2 CHI)
__host__ __device__ constexpr int env_tpc(int chi) { return env_threads(chi) / (2 * chi); }
// threads per row pair in the Jacobi sweep and per row in the Gram-Schmidt pass
__host__ __device__ constexpr int env_tpp(int chi) {
  return (env_threads(chi) / chi < 2 * chi) ? env_threads(chi) / chi
                                            : ((2 * chi < 32) ? 2 * chi : 32);
}

// Left-sweep layout: M_c (MQ x N2) lives in registers.  Thread (g = tid / TPC, part = tid % TPC)
// owns rows [part * RPT, part * RPT + RPT) of column g (rows >= MQ are zero padding).
template <int CHI>
struct LeftCfg {
  static constexpr int N2 = 2 * CHI, MQ = 4 * CHI;
  static constexpr int NT = env_threads(CHI);
  static constexpr int TPC = NT / N2;
  static constexpr int RPT = (MQ + TPC - 1) / TPC;
  static constexpr int VLD = (TPC * RPT + 3) / 4 * 4;   // reflector buffer length
  static constexpr int LDAT = CHI + 4;                  // A_c^T rows [b][ap][al]
  static constexpr int LDRT = N2 + 4;                   // R~ rows [b][al][i]
  static constexpr size_t lds = size_t(2) * CHI * LDAT + size_t(2) * CHI * LDRT + 2 * VLD + 8;
};

template <typename T, int CHI>
struct EnvSmem {
  static constexpr int N2 = 2 * CHI;     // bond of the operator-applied MPS; SVD matrix side
  static constexpr int MQ = 4 * CHI;     // rows of M_c
  static constexpr int LDT = N2 + 4;     // column stride of T, R, Xt (column-major); row stride of J
  static constexpr int LDZ = N2 + 4;     // row stride of Z (row-major)
  static constexpr int LDG = CHI + 1;    // row stride of the Gram / Cholesky factors
  static constexpr int NT = env_threads(CHI);
  static constexpr int NW = NT / 64;
  static constexpr int TILE = 2;
  static constexpr size_t bufA_left = LeftCfg<CHI>::lds;
  static constexpr size_t bufA_right = size_t(N2) * LDZ + size_t(N2) * LDT;
  // + MQ + N2: rows read past the end of the last column (values masked) stay in bounds
  static constexpr size_t bufA = (bufA_left > bufA_right ? bufA_left : bufA_right) + MQ + N2;
  static constexpr size_t bufR = size_t(N2) * LDT;
  // site of E_r (row stride LDA_S) or V (row stride LDV) in bufS: the odd strides keep the rows
  // that one matrix-core operand load touches in distinct LDS banks
  static constexpr int LDA_S = CHI + 1;
  static constexpr int LDV = N2 + 1;
  static constexpr size_t bufS = (size_t(2) * CHI * LDA_S > size_t(CHI) * LDV)
                                     ? size_t(2) * CHI * LDA_S : size_t(CHI) * LDV;
  static constexpr size_t stage = size_t(2) * CHI * (CHI + 2);   // next site of E_r
  static constexpr size_t reals = bufA + bufR + bufS + stage + 4 * N2 + 2 * NW + 2 * NW + 8;
  // + 1024 exponents of the carried factors, + 2 x 1028 bytes of bond dimensions
  static constexpr size_t ints = 3 * N2 + 2 * NW + 8 + 1024 + 2 * 1028 / 4;
  static constexpr size_t bytes = reals * sizeof(T) + ints * sizeof(int);
};

template <typename T, typename P>
__device__ __forceinline__ T bond_weight(P row_bits, int c, int sa, int sb, T ep, T em) {
  // exp(beta J s_a s_b): J = -1 iff bit c is set; spin index 0 <-> +1, 1 <-> -1.
  const bool af = (row_bits[c >> 6] >> (c & 63)) & 1ull;
  const bool parallel = (sa == sb);
  return (parallel != af) ? ep : em;
}

// C (M x N) = A (M x K) B (K x N) in FP64 on 16x16x4 matrix-core tiles (M, N multiples of 16,
// K of 4).  Each wavefront takes whole 16 x 16 output tiles; lane (i, q) = (lane % 16, lane / 16)
// feeds A(i, k0 + q) and B(k0 + q, j) and receives rows q + 4 r of column i of its tile.
// fa(i, k) and fb(k, j) read the operands, fc(i, j, v) stores.
template <int M, int N, int K, int NT, typename FA, typename FB, typename FC>
__device__ __forceinline__ void mfma_gemm_f64(FA fa, FB fb, FC fc) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  static_assert(M % 16 == 0 && N % 16 == 0 && K % 16 == 0, "matrix-core tile shapes");
  constexpr int TM = M / 16, TN = N / 16, NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  for (int t = wv; t < TM * TN; t += NWV) {
    const int r0 = (t % TM) * 16, c0 = (t / TM) * 16;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = fa(r0 + i16, k0 + 4 * u + q);
        b[u] = fb(k0 + 4 * u + q, c0 + i16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) fc(r0 + q + 4 * r, c0 + i16, acc[r]);
  }
}

// C (M x N) = A (M x K) B (K x N) in FP32 on 16x16x4 matrix-core tiles (M, N multiples of 16,
// K of 16), over the first `tm` row tiles only (rows >= 16 tm are not written).  Lane
// (i, q) = (lane % 16, lane / 16) feeds A(i, k0 + q) and B(k0 + q, j) and receives rows 4 q + r of
// column i of its tile (the FP32 instruction orders its results unlike the FP64 one).
template <int M, int N, int K, int NT, typename FA, typename FB, typename FC>
__device__ __forceinline__ void mfma_gemm_f32(FA fa, FB fb, FC fc, int tm = M / 16) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  static_assert(M % 16 == 0 && N % 16 == 0 && K % 16 == 0, "matrix-core tile shapes");
  constexpr int TN = N / 16, NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  for (int t = wv; t < tm * TN; t += NWV) {
    const int r0 = (t % tm) * 16, c0 = (t / tm) * 16;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = fa(r0 + i16, k0 + 4 * u + q);
        b[u] = fb(k0 + 4 * u + q, c0 + i16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) fc(r0 + 4 * q + r, c0 + i16, acc[r]);
  }
}

// The same product over index blocks only: rows [mb BS, mb BS + 16 mt) for mb < MB, columns
// [nb BS, nb BS + 16 nt) for nb < NB, and the contraction over [kb BS, kb BS + 16 kt) for kb < KB
// (what lies outside is zero in the operands, or not needed in the result).
template <int NT, int BS, int MB, int NB, int KB, typename FA, typename FB, typename FC>
__device__ __forceinline__ void mfma_gemm_f32_blocks(FA fa, FB fb, FC fc, int mt, int nt, int kt) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  static_assert(BS % 16 == 0, "block starts on a tile boundary");
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  const int tiles_m = MB * mt, tiles_n = NB * nt;
  for (int t = wv; t < tiles_m * tiles_n; t += NWV) {
    const int tm = t % tiles_m, tn = t / tiles_m;
    const int r0 = (tm / mt) * BS + (tm % mt) * 16, c0 = (tn / nt) * BS + (tn % nt) * 16;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < KB; ++kb) {
      for (int kk = 0; kk < kt; ++kk) {
        const int k0 = kb * BS + kk * 16;
        float a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = fa(r0 + i16, k0 + 4 * u + q);
          b[u] = fb(k0 + 4 * u + q, c0 + i16);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) fc(r0 + 4 * q + r, c0 + i16, acc[r]);
  }
}

// BATCH independent products C_b = A_b B_b of the shapes above in one tile loop, so that all
// wavefronts share the tiles of all products.  fa(b, i, k), fb(b, k, j), fc(b, i, j, v).
template <int BATCH, int M, int N, int K, int NT, typename FA, typename FB, typename FC>
__device__ __forceinline__ void mfma_gemm_f64_batched(FA fa, FB fb, FC fc) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  static_assert(M % 16 == 0 && N % 16 == 0 && K % 16 == 0, "matrix-core tile shapes");
  constexpr int TM = M / 16, TN = N / 16, NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  for (int t = wv; t < BATCH * TM * TN; t += NWV) {
    const int bt = t / (TM * TN), tt = t % (TM * TN);
    const int r0 = (tt % TM) * 16, c0 = (tt / TM) * 16;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = fa(bt, r0 + i16, k0 + 4 * u + q);
        b[u] = fb(bt, k0 + 4 * u + q, c0 + i16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) fc(bt, r0 + q + 4 * r, c0 + i16, acc[r]);
  }
}

// Householder reflector parameters for a column with pivot entry a and sub-pivot norm^2 s:
// beta = -sign(a) sqrt(a^2 + s), tau = (beta - a) / beta, scal = 1 / (a - beta) (the scale that
// makes v_pivot = 1).  FP32 uses the hardware reciprocal square root and reciprocal (about 1 ulp
// each; the reflector stays orthogonal to working precision), FP64 the IEEE operations.
__device__ __forceinline__ void hh_params(double a, double s, double& beta, double& tau,
                                          double& scal) {
  beta = -copysign(sqrt(a * a + s), a);
  tau = (beta - a) / beta;
  scal = 1.0 / (a - beta);
}
__device__ __forceinline__ void hh_params(float a, float s, float& beta, float& tau,
                                          float& scal) {
  const float n2 = a * a + s;
  const float r = __builtin_amdgcn_rsqf(n2);
  const float nrm = n2 * r;
  beta = -copysign(nrm, a);
  tau = 1.0f + fabsf(a) * r;
  scal = copysign(__builtin_amdgcn_rcpf(fabsf(a) + nrm), a);
}

// One-sided Jacobi rotation of a row pair with norms^2 a, b and inner product cc (cc != 0):
// t = tan(theta) with the smaller-angle root, cs = 1 / sqrt(1 + t^2), sn = cs t.  cs and sn form
// an exact rotation to working precision whatever the rounding of t; FP32 uses hardware
// reciprocal and reciprocal square root.
__device__ __forceinline__ void jacobi_rot(double a, double b, double cc, double& cs, double& sn) {
  const double zeta = (b - a) / (2.0 * cc);
  double t;
  if (fabs(zeta) > 1e15) t = 0.5 / zeta;
  else t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  cs = 1.0 / sqrt(1.0 + t * t);
  sn = cs * t;
}
__device__ __forceinline__ void jacobi_rot(float a, float b, float cc, float& cs, float& sn) {
  const float zeta = (b - a) * __builtin_amdgcn_rcpf(2.0f * cc);
  float t;
  if (fabsf(zeta) > 1e15f) {
    t = 0.5f * __builtin_amdgcn_rcpf(zeta);
  } else {
    const float q = 1.0f + zeta * zeta;
    t = copysign(__builtin_amdgcn_rcpf(fabsf(zeta) + q * __builtin_amdgcn_rsqf(q)), zeta);
  }
  cs = __builtin_amdgcn_rsqf(1.0f + t * t);
  sn = cs * t;
}

// C(M x N) = A(M x KD) B(KD x N) with TM x TN register tiles per thread; M % TM == N % TN == 0.
// fa(i, k), fb(k, j) load operands, fc(i, j, v) stores a result.
template <int TM, int TN, int KD, int NT, typename T, typename FA, typename FB, typename FC>
__device__ __forceinline__ void gemm_tiles(int M, int N, FA fa, FB fb, FC fc) {
  const int tm = M / TM, tn = N / TN;
  for (int t = threadIdx.x; t < tm * tn; t += NT) {
    const int i0 = (t % tm) * TM, j0 = (t / tm) * TN;
    T acc[TM][TN];
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
      for (int s = 0; s < TN; ++s) acc[r][s] = T(0);
#pragma unroll 8
    for (int k = 0; k < KD; ++k) {
      T av[TM], bv[TN];
#pragma unroll
      for (int r = 0; r < TM; ++r) av[r] = fa(i0 + r, k);
#pragma unroll
      for (int s = 0; s < TN; ++s) bv[s] = fb(k, j0 + s);
#pragma unroll
      for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int s = 0; s < TN; ++s) acc[r][s] += av[r] * bv[s];
    }
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
      for (int s = 0; s < TN; ++s) fc(i0 + r, j0 + s, acc[r][s]);
  }
}

// Householder reflector from its owner group's registers m[], pivot row j (rows > j are zeroed
// by it): writes v (v_j = 1, zero above j) to vb, tau to taub, beta to *dslot.  Thread `part`
// of the group holds rows part + TPC t; only t < RL can be nonzero.
template <typename T, int TPC, int RPT, int RL>
__device__ __forceinline__ void make_reflector(const T (&m)[RPT], int j, int part, int MQ, T* vb,
                                               T* taub, T* dslot) {
  T sp[4] = {T(0), T(0), T(0), T(0)}, a = 0;
#pragma unroll
  for (int t = 0; t < RL; ++t) {
    const int rho = part + TPC * t;
    sp[t & 3] += (rho > j) ? m[t] * m[t] : T(0);
    a += (rho == j) ? m[t] : T(0);
  }
  T s = (sp[0] + sp[1]) + (sp[2] + sp[3]);
  s = group_sum<TPC>(s);
  a = group_sum<TPC>(a);
  T tau = 0, beta = a, scal = 0;
  if (s > T(0)) hh_params(a, s, beta, tau, scal);
#pragma unroll
  for (int t = 0; t < RL; ++t) {
    const int rho = part + TPC * t;
    vb[rho] = (rho > j && rho < MQ) ? m[t] * scal : (rho == j ? T(1) : T(0));
  }
  if (part == 0) {
    *taub = tau;
    *dslot = beta;
  }
}

// Live-column numbering of the register-resident M (column g = tid / TPC): livek[g] = the rank
// of column g among the nonzero columns (-1 for a zero column), *nlive = their count.  Columns
// outside the bonds of the environment are exactly zero, so the QR below runs over the live
// columns only.  Ends with a barrier.
template <typename T, int CHI>
__device__ __forceinline__ void number_live_columns(const T (&m)[LeftCfg<CHI>::RPT], int* flag,
                                                    int* livek, int* nlive) {
  using C = LeftCfg<CHI>;
  constexpr int N2 = C::N2, TPC = C::TPC, RPT = C::RPT;
  static_assert(N2 <= 2 * WAVE, "two ballots number every column");
  const int tid = threadIdx.x, g = tid / TPC, part = tid % TPC;
  T nz = 0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) nz += (m[t] != T(0)) ? T(1) : T(0);
  nz = group_sum<TPC>(nz);
  if (part == 0) flag[g] = nz > T(0);
  __syncthreads();
  if (tid < WAVE) {
    const bool f0 = tid < N2 && flag[tid];
    const bool f1 = tid + WAVE < N2 && flag[tid + WAVE];
    const unsigned long long b0 = __ballot(f0), b1 = __ballot(f1);
    const unsigned long long below = (tid == 0) ? 0ull : (~0ull >> (WAVE - tid));
    if (tid < N2) livek[tid] = f0 ? __popcll(b0 & below) : -1;
    if (tid + WAVE < N2) livek[tid + WAVE] = f1 ? __popcll(b0) + __popcll(b1 & below) : -1;
    if (tid == 0) *nlive = __popcll(b0) + __popcll(b1);
  }
  __syncthreads();
}

// R factor of the register-resident M (R-only Householder QR) over its live columns, one
// barrier per reflector: after applying reflector k, the owner of live column k + 1 publishes
// reflector k + 1 into the other half of the double buffer.  A group of TP threads owns a
// column; thread `part` of it holds rows part + TP t; rows >= TP RL are zero, and so are the rows
// >= kmax once a column has seen every reflector: kmax = min(live columns, nonzero rows)
// reflectors are needed.  A live column (live rank kg) ends with its diagonal entry (row kg) in
// *dslot and the rows above it in m[]; a column with kg >= kmax gets *dslot = 0, a zero column
// (kg < 0) is left alone.  The R rows are thus compact: rows >= kmax are zero.
template <typename T, int CHI, int RL, int TP>
__device__ void householder_regs(T (&m)[LeftCfg<CHI>::RPT], T* vbuf, T* taub, T* dslot, int kg,
                                 int kmax) {
  using C = LeftCfg<CHI>;
  constexpr int MQ = C::MQ, RPT = C::RPT, VLD = C::VLD;
  static_assert(RL <= RPT && TP * RL <= VLD, "live rows fit the reflector buffer");
  const int part = threadIdx.x % TP;
  if (kg >= kmax && part == 0) *dslot = T(0);
  if (kg == 0 && kmax > 0) make_reflector<T, TP, RPT, RL>(m, 0, part, MQ, vbuf, taub, dslot);
  __syncthreads();
  for (int k = 0; k < kmax; ++k) {
    const T* vj = vbuf + (k & 1) * VLD;
    const T tau = taub[k & 1];
    if (kg > k) {
      // long slices re-read the reflector for the update instead of holding it in registers
      constexpr bool HOLD = RL <= 32;
      T vv[HOLD ? RL : 1];
      T wp[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        const T x = vj[part + TP * t];
        if constexpr (HOLD) vv[t] = x;
        wp[t & 3] += x * m[t];
      }
      T w = (wp[0] + wp[1]) + (wp[2] + wp[3]);
      w = group_sum<TP>(w);
      const T tw = tau * w;
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        if constexpr (HOLD) m[t] -= tw * vv[t];
        else m[t] -= tw * vj[part + TP * t];
      }
      if (kg == k + 1 && k + 1 < kmax)
        make_reflector<T, TP, RPT, RL>(m, k + 1, part, MQ, vbuf + ((k + 1) & 1) * VLD,
                                       taub + ((k + 1) & 1), dslot);
    }
    __syncthreads();
  }
}

// Orthonormalises rows 0..k-1 of V (CHI x N2, row-major, ld LDVR) in place, a group of TPP threads
// per row; the rows start with unit norm, and a row whose residual norm^2 falls below eta lies in
// the span of the earlier rows to rounding.  One pass of modified Gram-Schmidt taking the rows two
// at a time, one barrier per pair: with rows a and c = a+1 as they stand at the start of the step,
// c' = c - (<c,a>/<a,a>) a, and every later row b subtracts its projections on a and c', formed
// from <b,a>, <b,c>, <a,a>, <c,a>, <c,c>.  Rows whose residual norm^2 falls below eta are set to
// zero; the rows are normalised at the end.  Only the 2 KW columns (x, be < KW), at x CHI + be,
// take part (the others are zero).
template <typename T, int CHI, int NT, int LDVR, int KW = CHI, int TPP = env_tpp(CHI)>
__device__ void mgs_pairs_rows(T* V, int k, T eta) {
  constexpr int N2 = 2 * KW, EPR = (N2 + TPP - 1) / TPP;
  static_assert(NT / TPP >= CHI, "a group of TPP threads for every row");
  auto col = [](int j) { return (j / KW) * CHI + j % KW; };
  const int grp = threadIdx.x / TPP, l = threadIdx.x % TPP;
  const bool mine = grp < k;
  // wavefronts that hold no row only keep the barriers
  const bool wave_live = (threadIdx.x / WAVE) * (WAVE / TPP) < k;
  T vb[EPR];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EPR; ++e) {
    const int j = l + TPP * e;
    vb[e] = (mine && j < N2) ? V[grp * LDVR + col(j)] : T(0);
  }
  for (int a = 0; a < k; a += 2) {
    const int c = a + 1;
    const bool pair = c < k;
    if (wave_live) {
      T va[EPR], vc[EPR];
      T naa = 0, nca = 0, ncc = 0, dba = 0, dbc = 0;
#pragma unroll
      for (int e = 0; e < EPR; ++e) {
        const int j = l + TPP * e;
        const int jj = col(j < N2 ? j : 0);
        const T ra = V[a * LDVR + jj], rc = V[(pair ? c : a) * LDVR + jj];
        va[e] = (j < N2) ? ra : T(0);
        vc[e] = (pair && j < N2) ? rc : T(0);
        naa += va[e] * va[e];
        nca += vc[e] * va[e];
        ncc += vc[e] * vc[e];
        dba += vb[e] * va[e];
        dbc += vb[e] * vc[e];
      }
      naa = group_sum<TPP>(naa);
      nca = group_sum<TPP>(nca);
      ncc = group_sum<TPP>(ncc);
      dba = group_sum<TPP>(dba);
      dbc = group_sum<TPP>(dbc);
      const bool aok = naa > eta;
      const T ria = aok ? fast_rcp(naa) : T(0);
      const T g = nca * ria;                  // c' = c - g a
      const T ncp = ncc - g * nca;            // <c', c'>
      const bool cok = pair && ncp > eta;
      if (mine && grp > c) {
        const T fa = dba * ria;
        const T fc = cok ? (dbc - g * dba) * fast_rcp(ncp) : T(0);
        const T ca = fa - fc * g;             // b -= fa a + fc c' = (fa - fc g) a + fc c
#pragma unroll
        for (int e = 0; e < EPR; ++e) {
          const int j = l + TPP * e;
          vb[e] -= ca * va[e] + fc * vc[e];
          if (j < N2) V[grp * LDVR + col(j)] = vb[e];
        }
      }
      if (mine && grp == c) {
#pragma unroll
        for (int e = 0; e < EPR; ++e) {
          const int j = l + TPP * e;
          vb[e] = cok ? vb[e] - g * va[e] : T(0);
          if (j < N2) V[grp * LDVR + col(j)] = vb[e];
        }
      }
      if (mine && grp == a && !aok) {
#pragma unroll
        for (int e = 0; e < EPR; ++e) vb[e] = T(0);
      }
    }
    __syncthreads();
  }
  if (wave_live) {
    T n2 = 0;
#pragma unroll
    for (int e = 0; e < EPR; ++e) n2 += vb[e] * vb[e];
    n2 = group_sum<TPP>(n2);
    const T f = (n2 > T(0)) ? T(1) / sqrt(n2) : T(0);
#pragma unroll
    for (int e = 0; e < EPR; ++e) {
      const int j = l + TPP * e;
      vb[e] *= f;
      if (mine && j < N2) V[grp * LDVR + col(j)] = vb[e];
    }
  }
  __syncthreads();
}

// T: arithmetic type; E: storage type of the environments.  GRAM selects the Gram form of both
// sweeps (FP64 arithmetic for FP32 / BF16 environments): the QR sweep carries G_c = R_c^T R_c,
// and the SVD step factors Z_c^T G_{c-1} Z_c = (R_{c-1} Z_c)^T (R_{c-1} Z_c) by pivoted Cholesky,
// whose factor is the R of the pivoted QR of R_{c-1} Z_c (same pivots, same rows up to sign).
template <typename T, typename E, int CHI, bool GRAM, bool FLD>
__global__ __launch_bounds__(env_threads(CHI)) void env_build_kernel(const DevReal* reals,
                                                                     double* lnZ_out) {
  using Tol = JacobiTol<typename TolOf<E>::type>;
  // FP64 products on matrix-core tiles where the shapes allow
  constexpr bool MF64 = std::is_same<T, double>::value && CHI % 16 == 0;
  constexpr bool MF32 = std::is_same<T, float>::value && CHI % 16 == 0;
  using S = EnvSmem<T, CHI>;
  constexpr int N2 = S::N2, MQ = S::MQ, LDT = S::LDT, LDZ = S::LDZ;
  constexpr int LDA_S = S::LDA_S, LDV = S::LDV;
  constexpr int NT = S::NT, NW = S::NW, TL = S::TILE;
  constexpr int TPP = env_tpp(CHI);   // threads per Jacobi row pair
  constexpr int TPC = env_tpc(CHI);   // threads per column in the QR updates
  constexpr int EPT = (N2 + TPP - 1) / TPP;   // elements per thread of a Jacobi row
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* bufA = reinterpret_cast<T*>(smem_raw);
  T* bufR = bufA + S::bufA;
  T* bufS = bufR + S::bufR;
  T* Astage = bufS + S::bufS;       // 2 CHI^2: next site of E_r
  T* diag = Astage + S::stage;      // N2
  T* sc = diag + N2;                // 2 N2 scalars scratch
  T* cnv = sc + 2 * N2;             // N2 (ss double buffer lives in its first 2 entries too)
  T* candv = cnv + N2;              // 2 x NW argmax candidates
  T* red = candv + 2 * NW;          // 2 x NW per-wave maxima (the left sweep alternates halves)
  T* misc = red + 2 * NW;           // 8
  int* perm = reinterpret_cast<int*>(misc + 8);   // N2 logical -> physical column
  int* ord = perm + N2;                           // N2
  int* unpk = ord + N2;                           // N2: 1 = column not picked as a pivot
  int* candi = unpk + N2;                         // 2 x NW
  int* imisc = candi + 2 * NW;                    // 8
  int* rexp = imisc + 8;                          // exponents of the carried R_c (L <= 1024)
  // bond dimensions of E_r (bdin) and of E_{r-1} (bdout, filled by the second sweep): entry c is
  // the bond between sites c-1 and c; entries 0 and L are 1
  unsigned char* bdin = reinterpret_cast<unsigned char*>(rexp + 1024);
  unsigned char* bdout = bdin + 1028;
  // Sites whose bonds are all at most KWS are processed on the KWS-wide part of every block
  // (the rest is zero): the same arithmetic on a quarter of the entries and an eighth of the
  // products.  The numerical-rank truncation keeps most bonds of the random-bond lattices well
  // below chi.
  constexpr int KWS = 16;
  constexpr bool ADAPT = GRAM && MF64 && CHI > KWS && CHI <= 2 * KWS;
  // perm[rank .. nk) = the columns < nk never picked as pivots (unpk[col] = 1), ascending; wave w ranks
  // columns 64 w .. 64 w + 63 by ballot, offset by the counts of the waves before it.
  auto rank_unpicked = [&](int rk, int nk) {
    constexpr int NWC = (2 * CHI + WAVE - 1) / WAVE;
    static_assert(NWC <= 8, "column-count slots");
    const int t = threadIdx.x, wi = t / WAVE, li = t % WAVE;
    const bool un = t < nk && unpk[t];
    const unsigned long long mask = __ballot(un);
    if (li == 0 && wi < NWC) imisc[wi] = __popcll(mask);
    __syncthreads();
    if (un) {
      int base = rk;
      for (int w = 0; w < wi; ++w) base += imisc[w];
      perm[base + __popcll(mask & ((1ull << li) - 1ull))] = t;
    }
    __syncthreads();
  };

  // The thread index is re-issued at the top of every site (an empty asm that the compiler must
  // assume redefines it), so addresses derived from it are recomputed per site instead of being
  // hoisted out of the site loops and held in registers across them.
  int tid = threadIdx.x;
  auto fresh_tid = [&]() { asm volatile("" : "+v"(tid)); };
  const DevReal R = reals[blockIdx.x];
  const int L = R.L;
  const int W = words_per_row(L);
  const T ep = T(exp(R.beta)), em = T(exp(-R.beta));
  gmem<E>* env = as_global(reinterpret_cast<E*>(R.env));
  gmem<T>* rs = as_global(reinterpret_cast<T*>(R.ws));   // L x N2 x N2 scratch: R_c column-major
  gmem<double>* lognorm = as_global(R.lognorm);
  const size_t site = size_t(2) * CHI * CHI;
  const size_t rowst = site * L;
  T* Zr = bufA;                                       // Z_c: N2 x N2 row-major, ld LDZ
  T* Tw = bufA + size_t(N2) * LDZ;                    // T_c: N2 x N2 column-major, ld LDT

  for (size_t e = tid; e < rowst; e += NT) {         // E_{L-1} = 1
    const size_t inner = e % site;
    const int a = int((inner % (CHI * CHI)) / CHI), b = int(inner % CHI);
    gst<E>(env, size_t(L - 1) * rowst + e,
           narrow<E>((a == 0 && b == 0) ? T(0.70710678118654752440) : T(0)));
  }
  double lambda = 0.5 * double(L) * 0.69314718055994530942;
  if (tid == 0) lognorm[L - 1] = lambda;
  for (int c = tid; c <= L; c += NT) {
    bdin[c] = 1;
    bdout[c] = 1;
    if (R.bonds != nullptr) R.bonds[size_t(L - 1) * (L + 1) + c] = 1;
  }

  for (int r = L - 1; r >= 1; --r) {
    const gmem<E>* Ain = env + size_t(r) * rowst;
    gmem<E>* Aout = env + size_t(r - 1) * rowst;
    const gmem<const uint64_t>* jh = as_global(R.Jh) + size_t(r) * W;      // horizontal bonds of row r
    const gmem<const uint64_t>* jv = as_global(R.Jv) + size_t(r - 1) * W;  // vertical bonds, rows r-1 and r
    long long log2acc = 0;

    if constexpr (GRAM) {
      // ---------------- left to right: Gram matrices ----------------
      // With At_c = wh(a,b) wv(x,b) A_c[b]:
      //   G_c[(b,.),(b',.)] = kx(b,b') A_c[b]^T P_bb' A_c[b'],  kx(b,b') = sum_x wv(x,b) wv(x,b'),
      //   P_bb' = sum_{a,a'} wh(a,b) wh(a',b') G_{c-1}[(a,.),(a',.)];  G_0 = kx A_0[b][0]^T A_0[b'][0].
      // G_c is rescaled by 4^-e_c (R_c by 2^-e_c) and kept for the second sweep.
      constexpr int LDC = CHI + 2;
      static_assert(4 * CHI * LDC <= N2 * LDT, "P and Q blocks fit a Gram buffer");
      static_assert(size_t(N2) * LDT + size_t(2) * CHI * LDC <= S::bufA, "left-sweep buffers");
      T* gX = bufA;                        // G_{c-1} (N2 x LDT), then Q
      T* gY = bufR;                        // P, then G_c
      T* As2 = bufA + size_t(N2) * LDT;    // A_c[b][al][ap], ld LDC (alternates with Astage)
      T* Anx = Astage;                     // site c+1 while site c is processed
      constexpr int tmb = CHI / TL;
      // Site c+1 of E_r is fetched while site c is processed and parked in As2 at its end.  The
      // rescale of G_c (per-wave maxima in red[]) is applied by the next site's P pass, which
      // also stores the rescaled G_c for the second sweep.
      constexpr int SPT = (2 * CHI * CHI + NT - 1) / NT;
      E lpf[SPT];
      int lcc = 0;   // the fetched site (its field weights are applied when it is parked)
      auto lfetch = [&](int cc) {
#pragma unroll
        for (int t = 0; t < SPT; ++t) {
          const int e = tid + NT * t;
          if ((2 * CHI * CHI) % NT == 0 || e < int(site)) lpf[t] = gld<E>(Ain, size_t(cc) * site + e);
        }
        lcc = cc;
      };
      auto lpark = [&]() {
        T lg0, lg1;
        site_field_t<FLD, T>(R, r, lcc, ep, em, lg0, lg1);
#pragma unroll
        for (int t = 0; t < SPT; ++t) {
          const int e = tid + NT * t;
          if ((2 * CHI * CHI) % NT == 0 || e < int(site)) {
            const int b = e / (CHI * CHI), al = (e / CHI) % CHI, ap = e % CHI;
            Anx[(b * CHI + al) * LDC + ap] = (b ? lg1 : lg0) * widen(lpf[t]);
          }
        }
      };
      // The per-wave maxima of G_cc are in half (cc & 1) of red[]: a site has no barrier after
      // its reads of the previous half, so a wave that finishes early writes the other one.
      auto take_exponent = [&](int cc) {   // exponent of G_cc from the per-wave maxima
        const T* rd = red + (cc & 1) * NW;
        T m = rd[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmax(m, rd[w]);
        const int e = (pow2_exponent(m) + 1) / 2;
        log2acc += e;
        if (tid == 0) rexp[cc] = e;
        return e;
      };
      __syncthreads();
      lfetch(0);
      lpark();
      {
        T* tmp = As2;
        As2 = Anx;
        Anx = tmp;
      }
      for (int c = 0; c < L - 1; ++c) {
        fresh_tid();
        __syncthreads();
        if (c + 1 < L - 1) lfetch(c + 1);
        // kx(b,b') = sum_x wv(x,b) wv(x,b') = ep^2 + em^2 if b == b', 2 ep em otherwise, whatever
        // the sign of the vertical coupling (kept as two scalars: a 2x2 table indexed by the
        // runtime b would be placed in scratch memory)
        const T kxd = ep * ep + em * em, kxo = T(2) * ep * em;
        T mx = 0;
        if (c == 0) {
          for (int o = tid; o < N2 * N2; o += NT) {
            const int i = o / N2, k = o % N2;
            const int b = i / CHI, ap = i % CHI, b2 = k / CHI, ap2 = k % CHI;
            const T f = (b == b2) ? kxd : kxo;
            const T g = f * As2[(b * CHI) * LDC + ap] * As2[(b2 * CHI) * LDC + ap2];
            gY[i * LDT + k] = g;
            mx = fmax(mx, fabs(g));
          }
        } else {
          const T gs = T(ldexp(T(1), -2 * take_exponent(c - 1)));
          gmem<T>* gdst = rs + size_t(c - 1) * N2 * N2;
          T wh2[2][2];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) wh2[a][b] = bond_weight<T>(jh, c - 1, a, b, ep, em);
          auto left_site = [&](auto kwc) {
            constexpr int KW = decltype(kwc)::value;
            if constexpr (MF64) {
              // One wavefront per (b, b', column block of 16): P_bb' is formed from G_{c-1} as the
              // operand of Q = P_bb' A_c[b'], and Q stays in the matrix-core accumulators, whose
              // rows (q + 4 r of each lane group) are the rows the B operand of
              // G_c = kx A_c[b]^T Q takes from each lane: no LDS round trip, no barrier.
              typedef double v4d __attribute__((ext_vector_type(4)));
              constexpr int TT = KW / 16;
              const int lane = tid & (WAVE - 1), wvi = tid / WAVE, i16 = lane & 15, qg = lane >> 4;
              // the rescaled G_{c-1} (zero outside its bonds) for the second sweep
              for (int o = tid; o < N2 * N2; o += NT) gdst[o] = gs * gX[(o / N2) * LDT + o % N2];
              if (wvi < 4 * TT) {
                const int blk = wvi / TT, jb = wvi % TT;
                const int b = blk >> 1, b2 = blk & 1;
                const T w0b = gs * (b ? wh2[0][1] : wh2[0][0]), w1b = gs * (b ? wh2[1][1] : wh2[1][0]);
                const T w0c = b2 ? wh2[0][1] : wh2[0][0], w1c = b2 ? wh2[1][1] : wh2[1][0];
                v4d q[TT];
#pragma unroll
                for (int ib = 0; ib < TT; ++ib) {
                  q[ib] = v4d{0.0, 0.0, 0.0, 0.0};
                  const int al = ib * 16 + i16;
#pragma unroll
                  for (int kb = 0; kb < TT; ++kb) {
                    double pa[4], ab[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                      const int al2 = kb * 16 + 4 * u + qg;
                      const T g00 = gX[al * LDT + al2], g01 = gX[al * LDT + CHI + al2];
                      const T g10 = gX[(CHI + al) * LDT + al2], g11 = gX[(CHI + al) * LDT + CHI + al2];
                      pa[u] = w0b * (w0c * g00 + w1c * g01) + w1b * (w0c * g10 + w1c * g11);
                      ab[u] = As2[(b2 * CHI + al2) * LDC + jb * 16 + i16];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                      q[ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[u], ab[u], q[ib], 0, 0, 0);
                  }
                }
                const T f = (b == b2) ? kxd : kxo;
#pragma unroll
                for (int ib2 = 0; ib2 < TT; ++ib2) {
                  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                  for (int kb = 0; kb < TT; ++kb) {
                    double at[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) at[u] = As2[(b * CHI + kb * 16 + 4 * u + qg) * LDC + ib2 * 16 + i16];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(at[u], q[kb][u], acc, 0, 0, 0);
                  }
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    const int i = ib2 * 16 + qg + 4 * r, j = jb * 16 + i16;
                    const T g = f * acc[r];
                    gY[(b * CHI + i) * LDT + b2 * CHI + j] = g;
                    mx = fmax(mx, fabs(g));
                  }
                }
              }
              if constexpr (KW < CHI) {
                // G_c is zero outside its bonds (at most KW): fill, so that a full-width next site
                // reads zeros there
                for (int o = tid; o < N2 * N2; o += NT) {
                  const int i = o / N2, k = o % N2;
                  if (i % CHI >= KW || k % CHI >= KW) gY[i * LDT + k] = T(0);
                }
              }
              if (c + 1 < L - 1) lpark();   // into the other buffer (As2 is the current site)
            } else {
              for (int o = tid; o < 4 * KW * KW; o += NT) {
                const int blk = o / (KW * KW), al = (o / KW) % KW, al2 = o % KW;
                const int b = blk >> 1, b2 = blk & 1;
                // (selects, not indexing with the runtime b: that would put the table in scratch)
                const T w0b = gs * (b ? wh2[0][1] : wh2[0][0]), w1b = gs * (b ? wh2[1][1] : wh2[1][0]);
                const T w0c = b2 ? wh2[0][1] : wh2[0][0], w1c = b2 ? wh2[1][1] : wh2[1][0];
                const T g00 = gX[al * LDT + al2], g01 = gX[al * LDT + CHI + al2];
                const T g10 = gX[(CHI + al) * LDT + al2], g11 = gX[(CHI + al) * LDT + CHI + al2];
                gY[(blk * CHI + al) * LDC + al2] =
                    w0b * (w0c * g00 + w1c * g01) + w1b * (w0c * g10 + w1c * g11);
                if constexpr (KW == CHI) {
                  if (blk == 0) {   // the rescaled G_{c-1}, once per entry, for the second sweep
                    gdst[al * N2 + al2] = gs * g00;
                    gdst[al * N2 + CHI + al2] = gs * g01;
                    gdst[(CHI + al) * N2 + al2] = gs * g10;
                    gdst[(CHI + al) * N2 + CHI + al2] = gs * g11;
                  }
                }
              }
              if constexpr (KW < CHI) {
                // the whole rescaled G_{c-1} (zero outside its bonds) for the second sweep
                for (int o = tid; o < N2 * N2; o += NT) gdst[o] = gs * gX[(o / N2) * LDT + o % N2];
              }
              __syncthreads();
              if (c + 1 < L - 1) lpark();   // into the other buffer: As2 is read until the end of site c
            // Q_bb' = P_bb' A_c[b'] (into gX)
            for (int t = tid; t < 4 * tmb * tmb; t += NT) {
              const int blk = t / (tmb * tmb), tt = t % (tmb * tmb);
              const int i0 = (tt % tmb) * TL, j0 = (tt / tmb) * TL, b2 = blk & 1;
              T acc[TL][TL];
  #pragma unroll
              for (int u = 0; u < TL; ++u)
  #pragma unroll
                for (int v = 0; v < TL; ++v) acc[u][v] = T(0);
  #pragma unroll 8
              for (int k = 0; k < CHI; ++k) {
                T av[TL], bv[TL];
  #pragma unroll
                for (int u = 0; u < TL; ++u) av[u] = gY[(blk * CHI + i0 + u) * LDC + k];
  #pragma unroll
                for (int v = 0; v < TL; ++v) bv[v] = As2[(b2 * CHI + k) * LDC + j0 + v];
  #pragma unroll
                for (int u = 0; u < TL; ++u)
  #pragma unroll
                  for (int v = 0; v < TL; ++v) acc[u][v] += av[u] * bv[v];
              }
  #pragma unroll
              for (int u = 0; u < TL; ++u)
  #pragma unroll
                for (int v = 0; v < TL; ++v) gX[(blk * CHI + i0 + u) * LDC + j0 + v] = acc[u][v];
            }
            __syncthreads();
            // G_c = kx A_c[b]^T Q_bb' (into gY)
            for (int t = tid; t < 4 * tmb * tmb; t += NT) {
              const int blk = t / (tmb * tmb), tt = t % (tmb * tmb);
              const int i0 = (tt % tmb) * TL, j0 = (tt / tmb) * TL, b = blk >> 1, b2 = blk & 1;
              T acc[TL][TL];
  #pragma unroll
              for (int u = 0; u < TL; ++u)
  #pragma unroll
                for (int v = 0; v < TL; ++v) acc[u][v] = T(0);
  #pragma unroll 8
              for (int k = 0; k < CHI; ++k) {
                T av[TL], bv[TL];
  #pragma unroll
                for (int u = 0; u < TL; ++u) av[u] = As2[(b * CHI + k) * LDC + i0 + u];
  #pragma unroll
                for (int v = 0; v < TL; ++v) bv[v] = gX[(blk * CHI + k) * LDC + j0 + v];
  #pragma unroll
                for (int u = 0; u < TL; ++u)
  #pragma unroll
                  for (int v = 0; v < TL; ++v) acc[u][v] += av[u] * bv[v];
              }
              const T f = (b == b2) ? kxd : kxo;
  #pragma unroll
              for (int u = 0; u < TL; ++u)
  #pragma unroll
                for (int v = 0; v < TL; ++v)
                {
                  const T g = f * acc[u][v];
                  gY[(b * CHI + i0 + u) * LDT + b2 * CHI + j0 + v] = g;
                  mx = fmax(mx, fabs(g));
                }
            }
                        }
          };
          if constexpr (ADAPT) {
            if (bdin[c] <= KWS && bdin[c + 1] <= KWS) left_site(std::integral_constant<int, KWS>{});
            else left_site(std::integral_constant<int, CHI>{});
          } else {
            left_site(std::integral_constant<int, CHI>{});
          }
        }
        if (c == 0 && L > 2) lpark();
        mx = wave_max(mx);
        if ((tid & (WAVE - 1)) == 0) red[(c & 1) * NW + tid / WAVE] = mx;
        T* tmp = gX;
        gX = gY;
        gY = tmp;
        tmp = As2;
        As2 = Anx;
        Anx = tmp;
      }
      // the last Gram matrix of the row: rescale and store
      __syncthreads();
      {
        const T gs = T(ldexp(T(1), -2 * take_exponent(L - 2)));
        gmem<T>* gdst = rs + size_t(L - 2) * N2 * N2;
        for (int o = tid; o < N2 * N2; o += NT) gdst[o] = gs * gX[(o / N2) * LDT + o % N2];
      }
    } else // ---------------- left to right: R factors ----------------
    {
      using C = LeftCfg<CHI>;
      constexpr int TPC = C::TPC, RPT = C::RPT, LDAT = C::LDAT, LDRT = C::LDRT;
      T* AsT = bufA;                                   // A_c^T: [b][ap][al], ld LDAT
      T* Rt = AsT + size_t(2) * CHI * LDAT;            // R~_b = sum_a wh(a,b) R_{c-1}[:, (a, .)]
      T* vbuf = Rt + size_t(2) * CHI * LDRT;           // 2 x VLD reflectors
      T* taub = vbuf + 2 * C::VLD;                     // 2 taus
      // rows per thread that can be nonzero: a quarter, half or all of RPT
      constexpr int RQ = RPT / 4 > 0 ? RPT / 4 : 1, RH = RPT / 2 > 0 ? RPT / 2 : 1;
      int kprev = 0;                                   // nonzero rows of R_{c-1}
      for (int c = 0; c < L - 1; ++c) {
        fresh_tid();
        __syncthreads();
        // only the block (al < bdin[c], ap < bdin[c+1]) of site c of E_r can be nonzero; the
        // rest of AsT is never read
        const int bl = bdin[c], br = bdin[c + 1], blk = bl * br;
        T fg0, fg1;   // the site's field weights
        site_field_t<FLD, T>(R, r, c, ep, em, fg0, fg1);
        for (int o = tid; o < 2 * blk; o += NT) {
          const int b = o >= blk ? 1 : 0, rem = o - b * blk;
          const int al = rem / br, ap = rem - al * br;
          AsT[(b * CHI + ap) * LDAT + al] =
              (b ? fg1 : fg0) * widen(gld<E>(Ain, size_t(c) * site + size_t(b) * CHI * CHI + al * CHI + ap));
        }
        if (c > 0) {
          T wh2[2][2];   // wh2[a][b]
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) wh2[a][b] = bond_weight<T>(jh, c - 1, a, b, ep, em);
          // only the columns (a, al < bdin[c]) of R_{c-1} can be nonzero
          const int nal = bdin[c];
          for (int o = tid; o < 2 * nal * N2; o += NT) {
            const int b = o / (nal * N2), al = (o / N2) % nal, i = o % N2;
            Rt[(b * CHI + al) * LDRT + i] =
                wh2[0][b] * bufR[al * LDT + i] + wh2[1][b] * bufR[(CHI + al) * LDT + i];
          }
        }
        __syncthreads();
        // M_c rows (i, x): at site 0, i is the left bond of E_r (dimension bdin[0] = 1); after
        // that, i runs over the nonzero rows of R_{c-1}
        const int nrows = (c == 0) ? 2 * int(bdin[0]) : 2 * kprev;
        const int alim = bl;
        T m[RPT];
        // One site with TP threads per column.  TP = TPC: every column has a group (column g =
        // tid / TPC), the zero ones are found by ballot.  TP = 2 TPC (right bond <= CHI / 2): the
        // CHI groups take the 2 br columns (b, alpha' < br) in order, so each thread holds half as
        // many rows; the other columns of R_c are written as zeros.
        auto site_qr = [&](auto rlc, auto tpc, T (&m)[RPT]) __attribute__((always_inline)) {
          constexpr int RL = decltype(rlc)::value, TP = decltype(tpc)::value;
          constexpr bool REMAP = TP != TPC;
          const int part = tid % TP, h = tid / TP;
          const int g = !REMAP ? h : (h < br ? h : (h < 2 * br ? CHI + h - br : -1));
          const int gb = g < 0 ? 0 : g / CHI, gap = g < 0 ? 0 : g % CHI;
          const bool colz = g < 0 || gap >= br;          // column outside the right bond: zero
          const T w0 = bond_weight<T>(jv, c, 0, gb, ep, em);
          const T w1 = bond_weight<T>(jv, c, 1, gb, ep, em);
          const T wx = (part & 1) ? w1 : w0;             // rows part + TP t all have x = part & 1
          const T* acol = AsT + (gb * CHI + gap) * LDAT;   // A[b][.][ap]
#pragma unroll
          for (int t = 0; t < RPT; ++t) m[t] = T(0);
          if (c == 0) {
#pragma unroll
            for (int t = 0; t < RL; ++t) {
              const int rho = part + TP * t, i = rho >> 1;
              m[t] = (rho < MQ && i < alim && !colz) ? wx * acol[i < alim ? i : 0] : T(0);
            }
          } else {
            const T* rb = Rt + size_t(gb) * CHI * LDRT + (part >> 1);
            // eight rows at a time over the bond, so that few loads are in flight
            constexpr int CH = RL < 8 ? RL : 8;
#pragma unroll
            for (int t0 = 0; t0 < RL; t0 += CH) {
              for (int al = 0; al < alim; ++al) {
                const T a = acol[al];
                const T* rr = rb + al * LDRT;
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                  const int t = t0 + u;
                  if (t < RL && part + TP * t < MQ) m[t] += rr[(TP / 2) * t] * a;
                }
              }
            }
#pragma unroll
            for (int t = 0; t < RL; ++t) m[t] = colz ? T(0) : m[t] * wx;
          }
          int kg, kmax;
          if constexpr (!REMAP) {
            number_live_columns<T, CHI>(m, perm, ord, imisc + 6);
            kg = ord[g];
            kmax = imisc[6] < nrows ? imisc[6] : nrows;
          } else {
            kg = g < 0 ? -1 : h;
            kmax = 2 * br < nrows ? 2 * br : nrows;
          }
          // a zero column keeps diag = 0 (in the remapped form every column outside the bond)
          if (!REMAP && kg < 0 && part == 0) diag[g] = T(0);
          if (REMAP && tid < N2 && (tid % CHI) >= br) diag[tid] = T(0);
          householder_regs<T, CHI, RL, TP>(m, vbuf, taub, diag + (g < 0 ? 0 : g), kg, kmax);
          // carry R with a power-of-two rescale; keep it for the second sweep
          T mx = 0;
#pragma unroll
          for (int t = 0; t < RL; ++t)
            if (part + TP * t < kg) mx = fmax(mx, fabs(m[t]));
          if (tid < N2) mx = fmax(mx, fabs(diag[tid]));
          mx = block_max<NT>(mx, red);
          const int e = pow2_exponent(mx);
          log2acc += e;
          // exponent and the number of nonzero rows of R_c (< 256), packed: 256 e + kmax
          if (tid == 0) rexp[c] = e * 256 + kmax;
          gmem<T>* rsite = rs + size_t(c) * N2 * N2;
          if (g >= 0) {
            const T dg = diag[g];
#pragma unroll
            for (int t = 0; t < RPT; ++t) {
              const int rho = part + TP * t;
              if (TP * t < N2 && rho < N2) {
                const T v = T(ldexp(rho < kg ? m[t] : (rho == kg ? dg : T(0)), -e));
                bufR[g * LDT + rho] = v;
                rsite[size_t(g) * N2 + rho] = v;
              }
            }
          }
          if constexpr (REMAP) {
            // the columns (b, alpha' >= br) of R_c are zero
            const int nz = CHI - br;
            for (int o = tid; o < 2 * nz * N2; o += NT) {
              const int col = (o / (nz * N2)) * CHI + br + (o / N2) % nz, rho = o % N2;
              bufR[col * LDT + rho] = T(0);
              rsite[size_t(col) * N2 + rho] = T(0);
            }
          }
          kprev = kmax;
        };
        bool done = false;
        if constexpr (RPT >= 16) {   // chi >= 32: enough rows per thread to halve
          constexpr int TP2 = 2 * TPC, R2 = RPT / 2, RQ2 = R2 / 4, RH2 = R2 / 2;
          if (2 * br <= CHI) {
            const int tl = (nrows + TP2 - 1) / TP2;
            if (tl <= RQ2) site_qr(std::integral_constant<int, RQ2>{}, std::integral_constant<int, TP2>{}, m);
            else if (tl <= RH2) site_qr(std::integral_constant<int, RH2>{}, std::integral_constant<int, TP2>{}, m);
            else site_qr(std::integral_constant<int, R2>{}, std::integral_constant<int, TP2>{}, m);
            done = true;
          }
        }
        if (!done) {
          const int tl = (nrows + TPC - 1) / TPC;
          if (tl <= RQ) site_qr(std::integral_constant<int, RQ>{}, std::integral_constant<int, TPC>{}, m);
          else if (tl <= RH) site_qr(std::integral_constant<int, RH>{}, std::integral_constant<int, TPC>{}, m);
          else site_qr(std::integral_constant<int, RPT>{}, std::integral_constant<int, TPC>{}, m);
        }
      }
    }

    // ---------------- right to left: truncation ----------------
    // Xt (N2 x CHI column-major in bufR); for the last site the right bond is summed over b,
    // i.e. Xt[(b, 0)][0] = 1 for both b.
    __syncthreads();
    for (int o = tid; o < N2 * LDT; o += NT) bufR[o] = T(0);
    __syncthreads();
    if (tid == 0) { bufR[0] = T(1); bufR[CHI] = T(1); }
    // Site c-1 of E_r is fetched while site c is processed: its loads are issued at the start
    // of site c and parked in LDS (Astage) once the products of site c have used bufS; in the Gram
    // form G_{c-1} is fetched at the start of site c into registers.
    constexpr int SPT = (2 * CHI * CHI + NT - 1) / NT;
    constexpr int GPT = GRAM ? (N2 * N2 + NT - 1) / NT : 1;
    E apf[SPT];
    T gpf[GPT];
    int acc_site = 0;   // the fetched site (its field weights are applied when it is parked)
    auto fetch_site = [&](int cc) {
#pragma unroll
      for (int t = 0; t < SPT; ++t) {
        const int e = tid + NT * t;
        if ((2 * CHI * CHI) % NT == 0 || e < int(site)) apf[t] = gld<E>(Ain, size_t(cc) * site + e);
      }
      acc_site = cc;
    };
    auto park_site = [&]() {
      T ag0, ag1;
      site_field_t<FLD, T>(R, r, acc_site, ep, em, ag0, ag1);
#pragma unroll
      for (int t = 0; t < SPT; ++t) {
        const int e = tid + NT * t;
        if ((2 * CHI * CHI) % NT == 0 || e < int(site))
          Astage[e] = (e >= CHI * CHI ? ag1 : ag0) * widen(apf[t]);
      }
    };
    fetch_site(L - 1);
    park_site();
    for (int c = L - 1; c >= 0; --c) {
      fresh_tid();
      __syncthreads();
      for (int e = tid; e < int(site); e += NT) bufS[(e / CHI) * LDA_S + e % CHI] = Astage[e];
      if (c > 0) fetch_site(c - 1);
      if constexpr (GRAM) {
        if (c > 0) {
          const gmem<T>* gsrc = rs + size_t(c - 1) * N2 * N2;
#pragma unroll
          for (int t = 0; t < GPT; ++t) {
            const int o = tid + NT * t;
            if ((N2 * N2) % NT == 0 || o < N2 * N2) gpf[t] = gsrc[o];
          }
        }
      }
      __syncthreads();
      T wv[2][2], wh[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int b = 0; b < 2; ++b) wv[x][b] = bond_weight<T>(jv, c, x, b, ep, em);
      // 2^-e rescale of Xt_{c+1} (from the maxima its product left in red[]), folded into wh
      T xsc = T(1);
      if (c < L - 1) {
        T m = red[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmax(m, red[w]);
        const int xe = pow2_exponent(m);
        log2acc += xe;
        xsc = T(ldexp(T(1), -xe));
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          wh[a][b] = xsc * ((c > 0) ? bond_weight<T>(jh, c - 1, a, b, ep, em) : (a == 0 ? T(1) : T(0)));
      // Sites whose bonds (both of site c of E_r, and the right bond of site c of E_{r-1}) are at
      // most KWS run on the KWS-wide part of every block.  Z, W, H and the Cholesky factor are
      // then stored compactly (index (s, al) at s KW + al); the site of E_{r-1}, V and Xt_c keep the
      // full layout, zero outside the bonds.  Returns true after site 0 (end of the row).
      auto right_site = [&](auto kwc) -> bool {
        constexpr int KW = decltype(kwc)::value, NK = 2 * KW;
        auto phys = [](int u) { return (u / KW) * CHI + u % KW; };
        // Z[(a,al)][(x,be)] = sum_b wh(a,b) wv(x,b) (A_c[b] Xt_b)[al][be]
        if constexpr (MF64) {
          // both products of an output tile on 16x16x4 FP64 matrix-core tiles, combined in registers
          typedef double v4d __attribute__((ext_vector_type(4)));
          constexpr int TT = KW / 16;
          const int lane = tid & 63, wvi = tid >> 6, i16 = lane & 15, qg = lane >> 4;
          for (int t = wvi; t < TT * TT; t += NW) {
            const int r0 = (t % TT) * 16, c0 = (t / TT) * 16;
            v4d p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
  #pragma unroll
            for (int k0 = 0; k0 < KW; k0 += 4) {
              const int k = k0 + qg;
              const double a0 = bufS[(r0 + i16) * LDA_S + k], a1 = bufS[(CHI + r0 + i16) * LDA_S + k];
              const double x0 = bufR[(c0 + i16) * LDT + k], x1 = bufR[(c0 + i16) * LDT + CHI + k];
              p0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0, p0, 0, 0, 0);
              p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1, p1, 0, 0, 0);
            }
  #pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int al = r0 + qg + 4 * rr, be = c0 + i16;
  #pragma unroll
              for (int a = 0; a < 2; ++a)
  #pragma unroll
                for (int x = 0; x < 2; ++x)
                  Zr[(a * KW + al) * LDZ + x * KW + be] =
                      wh[a][0] * wv[x][0] * p0[rr] + wh[a][1] * wv[x][1] * p1[rr];
            }
          }
        } else if constexpr (MF32) {
          // the same on 16x16x4 FP32 matrix-core tiles (results in rows 4 q + r)
          typedef float v4f __attribute__((ext_vector_type(4)));
          constexpr int TT = KW / 16;
          const int lane = tid & 63, wvi = tid >> 6, i16 = lane & 15, qg = lane >> 4;
          for (int t = wvi; t < TT * TT; t += NW) {
            const int r0 = (t % TT) * 16, c0 = (t / TT) * 16;
            v4f p0 = {0.f, 0.f, 0.f, 0.f}, p1 = {0.f, 0.f, 0.f, 0.f};
  #pragma unroll
            for (int k0 = 0; k0 < KW; k0 += 4) {
              const int k = k0 + qg;
              const float a0 = bufS[(r0 + i16) * LDA_S + k], a1 = bufS[(CHI + r0 + i16) * LDA_S + k];
              const float x0 = bufR[(c0 + i16) * LDT + k], x1 = bufR[(c0 + i16) * LDT + CHI + k];
              p0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, x0, p0, 0, 0, 0);
              p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, x1, p1, 0, 0, 0);
            }
  #pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int al = r0 + 4 * qg + rr, be = c0 + i16;
  #pragma unroll
              for (int a = 0; a < 2; ++a)
  #pragma unroll
                for (int x = 0; x < 2; ++x)
                  Zr[(a * KW + al) * LDZ + x * KW + be] =
                      wh[a][0] * wv[x][0] * p0[rr] + wh[a][1] * wv[x][1] * p1[rr];
            }
          }
        } else
        {
          constexpr int tm = CHI / TL;
          for (int t = tid; t < tm * tm; t += NT) {
            const int al0 = (t % tm) * TL, be0 = (t / tm) * TL;
            T p0[TL][TL], p1[TL][TL];
  #pragma unroll
            for (int u = 0; u < TL; ++u)
  #pragma unroll
              for (int v = 0; v < TL; ++v) { p0[u][v] = T(0); p1[u][v] = T(0); }
  #pragma unroll 8
            for (int ap = 0; ap < CHI; ++ap) {
              T a0[TL], a1[TL], x0[TL], x1[TL];
  #pragma unroll
              for (int u = 0; u < TL; ++u) {
                a0[u] = bufS[(al0 + u) * LDA_S + ap];
                a1[u] = bufS[(CHI + al0 + u) * LDA_S + ap];
                x0[u] = bufR[(be0 + u) * LDT + ap];
                x1[u] = bufR[(be0 + u) * LDT + CHI + ap];
              }
  #pragma unroll
              for (int u = 0; u < TL; ++u)
  #pragma unroll
                for (int v = 0; v < TL; ++v) {
                  p0[u][v] += a0[u] * x0[v];
                  p1[u][v] += a1[u] * x1[v];
                }
            }
  #pragma unroll
            for (int a = 0; a < 2; ++a)
  #pragma unroll
              for (int x = 0; x < 2; ++x) {
                const T f0 = wh[a][0] * wv[x][0], f1 = wh[a][1] * wv[x][1];
  #pragma unroll
                for (int u = 0; u < TL; ++u)
  #pragma unroll
                  for (int v = 0; v < TL; ++v)
                    Zr[(a * CHI + al0 + u) * LDZ + x * CHI + be0 + v] = f0 * p0[u][v] + f1 * p1[u][v];
              }
          }
        }
        __syncthreads();
        if (c > 0) park_site();   // bufS and Astage are not read again during site c
        if (c == 0) {
          // site 0: left bond (a = 0, alpha = 0): A_0[x][0][be] = Z[(0,0)][(x,be)]
          T part = 0;
          for (int o = tid; o < 2 * CHI; o += NT) {
            const T d = (o % CHI < KW) ? Zr[(o / CHI) * KW + o % CHI] : T(0);
            sc[o] = d;
            part += d * d;
          }
          const T nrm2 = block_sum<NT>(part, red);
          const T nrm = sqrt(nrm2);
          for (int o = tid; o < int(site); o += NT) {
            const int x = o / (CHI * CHI), al = (o / CHI) % CHI, be = o % CHI;
            gst<E>(Aout, o, narrow<E>((al == 0 && nrm > T(0)) ? sc[x * CHI + be] / nrm : T(0)));
          }
          lambda += double(log2acc) * 0.69314718055994530942 + log(double(nrm));
          if (tid == 0) lognorm[r - 1] = lambda;
          return true;
        }
        int rank = NK;
        T fro2 = 0;
        if constexpr (GRAM) {
          // H = Z^T G_{c-1} Z (row-major in bufR), via W = G_{c-1} Z (in Tw).  Rounding leaves H
          // slightly asymmetric; the factorisation reads its columns only.
  #pragma unroll
          for (int t = 0; t < GPT; ++t) {
            const int o = tid + NT * t;
            if ((N2 * N2) % NT == 0 || o < N2 * N2) bufR[(o / N2) * LDT + (o % N2)] = gpf[t];
          }
          __syncthreads();
          auto ga = [&](int i, int k) { return bufR[phys(i) * LDT + phys(k)]; };
          auto gb = [&](int k, int col) { return Zr[k * LDZ + col]; };
          auto gc = [&](int i, int col, T v) { Tw[i * LDT + col] = v; };
          auto ha = [&](int c1, int i) { return Zr[i * LDZ + c1]; };
          auto hb = [&](int i, int c2) { return Tw[i * LDT + c2]; };
          auto hc = [&](int c1, int c2, T v) { bufR[c1 * LDT + c2] = v; };
          if constexpr (MF64) mfma_gemm_f64<NK, NK, NK, NT>(ga, gb, gc);
          else gemm_tiles<TL, TL, N2, NT, T>(N2, N2, ga, gb, gc);
          __syncthreads();
          if constexpr (MF64) {
            // H is symmetric: the tiles on and above the diagonal, each mirrored below
            typedef double v4d __attribute__((ext_vector_type(4)));
            constexpr int TH = NK / 16, NTILE = TH * (TH + 1) / 2;
            const int lane = tid & 63, wvi = tid >> 6, i16 = lane & 15, qg = lane >> 4;
            for (int t = wvi; t < NTILE; t += NW) {
              int ti = 0, rem = t;
              while (rem >= TH - ti) { rem -= TH - ti; ++ti; }
              const int tj = ti + rem;
              const int r0 = ti * 16, c0 = tj * 16;
              v4d acc = {0.0, 0.0, 0.0, 0.0};
              for (int k0 = 0; k0 < NK; k0 += 16) {
                double a[4], b[4];
  #pragma unroll
                for (int u = 0; u < 4; ++u) {
                  a[u] = ha(r0 + i16, k0 + 4 * u + qg);
                  b[u] = hb(k0 + 4 * u + qg, c0 + i16);
                }
  #pragma unroll
                for (int u = 0; u < 4; ++u)
                  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
              }
  #pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const int i = r0 + qg + 4 * rr, j = c0 + i16;
                bufR[i * LDT + j] = acc[rr];
                if (ti != tj) bufR[j * LDT + i] = acc[rr];
              }
            }
          } else {
            gemm_tiles<TL, TL, N2, NT, T>(N2, N2, ha, hb, hc);
          }
          __syncthreads();
          // ---- pivoted Cholesky of H, stopping at the numerical rank: H[p, p] = L L^T ----
          // One wavefront, lane a = row a (2 CHI <= 64), so the loop needs no workgroup barrier.
          // Left-looking: with p_j the row of largest remaining diagonal d,
          //   L[a][j] = (H[a][p_j] - sum_{i<j} L[a][i] L[p_j][i]) / sqrt(d[p_j]),  d[a] -= L[a][j]^2;
          // row j of L^T (natural column order) goes to Tw.  The pivot comes from one unsigned wave
          // maximum over keys (float bits of d with the low 6 bits = 63 - row: larger d first, to
          // 2^-17 relative, ties to the smaller row); its exact d by readlane.  Within one wavefront
          // LDS operations complete in order, so the rows of L^T written at step i are visible to
          // every lane at later steps.
          static_assert(NK <= WAVE, "one wavefront holds every row");
          if (tid < WAVE) {
            const int a = tid;
            const bool live = a < NK;
            T d = live ? bufR[a * LDT + a] : T(0);
            const T f2 = wave_sum(live ? fmax(d, T(0)) : T(0));
            const T tol2 = T(Tol::rank) * T(Tol::rank) * f2;
            bool pkd = !live;
            int rk = NK;
            if constexpr (NK <= 32) {
              // Widths up to 16: lane a keeps its row of L in registers, and the pivot row's entries
              // come by readlane (wave-uniform lane), so no step waits on LDS for the dot product.
              T Lr[NK];
#pragma unroll
              for (int j = 0; j < NK; ++j) {
                const uint32_t key =
                    pkd ? 0u : ((__float_as_uint(float(fmax(d, T(0)))) & ~63u) | uint32_t(63 - a));
                const uint32_t bk = wave_max_u32(key);
                const int piv = 63 - int(bk & 63u);
                const T best = readlane_v(d, piv);
                if (bk == 0u || !(best > tol2)) {
                  rk = j;
                  break;
                }
                const T hap = bufR[a * LDT + piv];
                T inv = T(__builtin_amdgcn_rsq(double(best)));
                inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
                inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
                const T sq = best * inv;
                T dot = 0;
#pragma unroll
                for (int i = 0; i < j; ++i) dot += Lr[i] * readlane_v(Lr[i], piv);
                const bool arow = !pkd && a != piv;
                const T La = (a == piv) ? sq : (arow ? (hap - dot) * inv : T(0));
                Lr[j] = La;
                if (live) Tw[j * LDT + a] = La;
                d -= arow ? La * La : T(0);
                if (a == piv) pkd = true;
                if (a == 0) perm[j] = piv;
              }
            } else {
            // Wider: the first 16 columns of L stay in registers as above; later columns read the
            // earlier rows of L^T from LDS (16 register columns measured faster than 32, which
            // made the kernel spill).
            constexpr int NRG = 16;
            T Lr[NRG];
            bool stop = false;
#pragma unroll
            for (int j = 0; j < NRG; ++j) {
              const uint32_t key =
                  pkd ? 0u : ((__float_as_uint(float(fmax(d, T(0)))) & ~63u) | uint32_t(63 - a));
              const uint32_t bk = wave_max_u32(key);
              const int piv = 63 - int(bk & 63u);
              const T best = readlane_v(d, piv);
              if (bk == 0u || !(best > tol2)) {
                rk = j;
                stop = true;
                break;
              }
              const T hap = bufR[a * LDT + piv];
              T inv = T(__builtin_amdgcn_rsq(double(best)));
              inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
              inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
              const T sq = best * inv;
              T dot = 0;
#pragma unroll
              for (int i = 0; i < j; ++i) dot += Lr[i] * readlane_v(Lr[i], piv);
              const bool arow = !pkd && a != piv;
              const T La = (a == piv) ? sq : (arow ? (hap - dot) * inv : T(0));
              Lr[j] = La;
              if (live) Tw[j * LDT + a] = La;
              d -= arow ? La * La : T(0);
              if (a == piv) pkd = true;
              if (a == 0) perm[j] = piv;
            }
            if (!stop)
            for (int j = NRG; j < NK; ++j) {
              const uint32_t key =
                  pkd ? 0u : ((__float_as_uint(float(fmax(d, T(0)))) & ~63u) | uint32_t(63 - a));
              const uint32_t bk = wave_max_u32(key);
              const int piv = 63 - int(bk & 63u);
              const T best = readlane_v(d, piv);
              if (bk == 0u || !(best > tol2)) { rk = j; break; }
              // 1/sqrt(d) from the hardware estimate refined by two Newton steps
              T inv = T(__builtin_amdgcn_rsq(double(best)));
              inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
              inv = inv * (T(1.5) - T(0.5) * best * inv * inv);
              const T sq = best * inv;
              const T hap = bufR[a * LDT + piv];
              T dot = 0;
#pragma unroll
              for (int i = 0; i < NRG; ++i) dot += Lr[i] * readlane_v(Lr[i], piv);
              // four rows per round, loads issued together (rows past j are clamped and masked)
              for (int i0 = NRG; i0 < j; i0 += 4) {
                T x[4], y[4];
  #pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const int ii = (i0 + u < NK) ? i0 + u : NK - 1;
                  x[u] = Tw[ii * LDT + a];
                  y[u] = Tw[ii * LDT + piv];
                }
  #pragma unroll
                for (int u = 0; u < 4; ++u) dot += (i0 + u < j) ? x[u] * y[u] : T(0);
              }
              const bool arow = !pkd && a != piv;
              const T La = (a == piv) ? sq : (arow ? (hap - dot) * inv : T(0));
              if (live) Tw[j * LDT + a] = La;
              d -= arow ? La * La : T(0);
              if (a == piv) pkd = true;
              if (a == 0) perm[j] = piv;
            }
            }
            if (live) unpk[a] = pkd ? 0 : 1;
            if (a == 0) {
              imisc[7] = rk;
              misc[0] = f2;
            }
          }
          __syncthreads();
          rank = imisc[7];
          fro2 = misc[0];
          rank_unpicked(rank, NK);
          // J = rows 0..rank-1 of L^T in pivoted column order (row-major in bufR, ld LDT)
          const int nr = rank + (rank & 1);
          for (int o = tid; o < nr * NK; o += NT) {
            const int i = o / NK, kk = o % NK;
            bufR[i * LDT + kk] = (i < rank) ? Tw[i * LDT + perm[kk]] : T(0);
          }
          __syncthreads();
        } else {
          // R_{c-1} into bufR, then T = R_{c-1} Z.  Rows >= nrT of R_{c-1} are zero, and so
          // are those of T: the product and the pivoted QR below run over TPC RL2 >= nrT rows.
          const int nrT = rexp[c - 1] & 255;
          constexpr int RPT2 = (N2 + TPC - 1) / TPC;
          constexpr int R2Q = RPT2 / 4 > 0 ? RPT2 / 4 : 1, R2H = RPT2 / 2 > 0 ? RPT2 / 2 : 1;
          const int tl2 = (nrT + TPC - 1) / TPC;
          const int rl2 = (tl2 <= R2Q) ? R2Q : (tl2 <= R2H) ? R2H : RPT2;
          const int mrows = (TPC * rl2 < N2) ? TPC * rl2 : N2;
          const gmem<T>* rsrc = rs + size_t(c - 1) * N2 * N2;
          for (int o = tid; o < N2 * mrows; o += NT) {
            const int col = o / mrows, i = o % mrows;
            bufR[col * LDT + i] = rsrc[size_t(col) * N2 + i];
          }
          __syncthreads();
          auto ta = [&](int i, int a) { return bufR[a * LDT + i]; };
          auto tb = [&](int a, int col) { return Zr[a * LDZ + col]; };
          auto tc = [&](int i, int col, T v) { Tw[col * LDT + i] = v; };
          if constexpr (MF64) {
            mfma_gemm_f64<N2, N2, N2, NT>(ta, tb, tc);
          } else if constexpr (MF32) {
            // T is zero outside the columns (x, be < bdout[c+1]); the contraction runs over the
            // columns (a, al < bdin[c]) of R_{c-1}, the others being zero
            const int nbt = (bdout[c + 1] + 15) / 16, kbt = (bdin[c] + 15) / 16;
            mfma_gemm_f32_blocks<NT, CHI, 1, 2, 2>(ta, tb, tc, (mrows + 15) / 16, nbt, kbt);
            const int nz = CHI - 16 * nbt;
            for (int o = tid; o < 2 * nz * mrows; o += NT) {
              const int col = (o / (nz * mrows)) * CHI + 16 * nbt + (o / mrows) % nz;
              Tw[col * LDT + o % mrows] = T(0);
            }
          } else {
            gemm_tiles<TL, TL, N2, NT, T>((mrows + TL - 1) / TL * TL, N2, ta, tb, tc);
          }
          __syncthreads();

          // ---- QR with column pivoting, stopping at the numerical rank ----
          // Group g (TPC threads) owns physical column g; thread part keeps rows part + TPC t
          // (t < RL2) in registers and republishes them in Tw after each update, so that every
          // thread reads the next pivot column from LDS and forms its reflector itself (one
          // barrier per column).
          // TP = TPC: every physical column g = tid / TPC has a group.  TP = 2 TPC (right bond
          // bdo of the new site <= CHI / 2): the CHI groups take the 2 bdo columns (x, be < bdo)
          // of T in order (the others are zero and never pivots), so each thread holds half as
          // many rows.
          const int bdo = bdout[c + 1];
          int g = 0, part = 0;
          bool owner = false, active = false;
          auto qrcp = [&](auto rlc, auto tpc) __attribute__((always_inline)) {
            constexpr int RL2 = decltype(rlc)::value, TP = decltype(tpc)::value;
            part = tid % TP;
            const int h = tid / TP;
            g = (TP == TPC) ? h : (h < bdo ? h : (h < 2 * bdo ? CHI + h - bdo : N2));
            owner = g < N2;
            active = owner;
            T mc[RL2];
            T cn = 0;
            {
              T cp[4] = {T(0), T(0), T(0), T(0)};
    #pragma unroll
              for (int t = 0; t < RL2; ++t) {
                const int rho = part + TP * t;
                mc[t] = (owner && rho < N2) ? Tw[g * LDT + rho] : T(0);
                cp[t & 3] += mc[t] * mc[t];
              }
              cn = group_sum<TP>((cp[0] + cp[1]) + (cp[2] + cp[3]));
            }
            {
              T bv = owner ? cn : T(-1);
              int bi = owner ? g : N2;
              wave_argmax(bv, bi);
              if ((tid & (WAVE - 1)) == 0) { candv[tid / WAVE] = bv; candi[tid / WAVE] = bi; }
            }
            fro2 = block_sum<NT>((owner && part == 0) ? cn : T(0), red);
            const T tolr2 = T(Tol::rank) * T(Tol::rank) * fro2;
            rank = N2;
            for (int j = 0; j < N2; ++j) {
              const int buf = j & 1;
              // arg-max of the per-wave candidates (ties -> smaller column), without branches
              T cv[NW];
              int ci[NW];
    #pragma unroll
              for (int w = 0; w < NW; ++w) {
                cv[w] = candv[buf * NW + w];
                ci[w] = candi[buf * NW + w];
              }
              T best = cv[0];
              int piv = ci[0];
    #pragma unroll
              for (int w = 1; w < NW; ++w) {
                const bool better = (cv[w] > best) | ((cv[w] == best) & (ci[w] < piv));
                best = better ? cv[w] : best;
                piv = better ? ci[w] : piv;
              }
              if (!(best > tolr2)) { rank = j; break; }
              const T* pc = Tw + piv * LDT;
              const T alpha = pc[j];
              const T ss = fmax(best - alpha * alpha, T(0));
              T tau = 0, beta = alpha, scal = 0;
              if (ss > T(0)) hh_params(alpha, ss, beta, tau, scal);
              if (tid == 0) { diag[j] = beta; perm[j] = piv; }
              if (g == piv) active = false;
              T v[RL2];
              T wp[4] = {T(0), T(0), T(0), T(0)};
              // loads first and unconditional (a select on the loaded value would let the
              // compiler move each load under its own branch and wait for it there)
    #pragma unroll
              for (int t = 0; t < RL2; ++t) {
                const int rho = part + TP * t;
                v[t] = pc[(N2 % TP == 0 || rho < N2) ? rho : 0];
              }
    #pragma unroll
              for (int t = 0; t < RL2; ++t) {
                const int rho = part + TP * t;
                const T sg = (rho > j && rho < N2) ? scal : T(0);
                const T one = (rho == j) ? T(1) : T(0);
                v[t] = v[t] * sg + one;
                wp[t & 3] += v[t] * mc[t];
              }
              const T w = group_sum<TP>((wp[0] + wp[1]) + (wp[2] + wp[3]));
              T np[4] = {T(0), T(0), T(0), T(0)};
              if (active) {
                const T tw = tau * w;
    #pragma unroll
                for (int t = 0; t < RL2; ++t) {
                  const int rho = part + TP * t;
                  mc[t] -= tw * v[t];
                  np[t & 3] += (rho > j) ? mc[t] * mc[t] : T(0);
                  if (N2 % TP == 0 || rho < N2) Tw[g * LDT + rho] = mc[t];
                }
              }
              const T nn = group_sum<TP>((np[0] + np[1]) + (np[2] + np[3]));
              {
                T bv = active ? nn : T(-1);
                int bi = active ? g : N2;
                wave_argmax(bv, bi);
                if ((tid & (WAVE - 1)) == 0) {
                  candv[(buf ^ 1) * NW + tid / WAVE] = bv;
                  candi[(buf ^ 1) * NW + tid / WAVE] = bi;
                }
              }
              __syncthreads();
            }
          };
          bool done = false;
          if constexpr (RPT2 >= 8) {   // rows of T = TPC rl2 = 2 TPC (rl2 / 2)
            if (2 * bdo <= CHI) {
              using I2 = std::integral_constant<int, 2 * TPC>;
              if (rl2 == R2Q) qrcp(std::integral_constant<int, R2Q / 2>{}, I2{});
              else if (rl2 == R2H) qrcp(std::integral_constant<int, R2H / 2>{}, I2{});
              else qrcp(std::integral_constant<int, RPT2 / 2>{}, I2{});
              done = true;
            }
          }
          if (!done) {
            using I1 = std::integral_constant<int, TPC>;
            if (rl2 == R2Q) qrcp(std::integral_constant<int, R2Q>{}, I1{});
            else if (rl2 == R2H) qrcp(std::integral_constant<int, R2H>{}, I1{});
            else qrcp(std::integral_constant<int, RPT2>{}, I1{});
          }
          // columns never picked follow the pivots in ascending order (the zero columns that
          // have no group in the remapped form among them)
          if (owner && part == 0) unpk[g] = active ? 1 : 0;
          if (done && tid < N2 && (tid % CHI) >= bdo) unpk[tid] = 1;
          __syncthreads();
          rank_unpicked(rank, NK);
          // J = rows 0..rank-1 of R in pivoted column order (row-major in bufR, ld LDT)
          const int nr = rank + (rank & 1);
          for (int o = tid; o < nr * NK; o += NT) {
            const int i = o / NK, kk = o % NK;
            T val = T(0);
            if (i < rank) val = (kk > i) ? Tw[perm[kk] * LDT + i] : (kk == i ? diag[i] : T(0));
            bufR[i * LDT + kk] = val;
          }
          __syncthreads();
        }
        const int nr = rank + (rank & 1);

        // ---- one-sided Jacobi on the rows of J, parallel round-robin ordering ----
        // Needed only when the numerical rank exceeds CHI: otherwise every direction is kept, and
        // the span of the rows of J (what site c of E_{r-1} depends on) is already final.
        if (KW == CHI && nr >= 2 && rank > CHI) {
          const T tol = T(Tol::rot) * sqrt(fro2);
          const int gj = tid / TPP, l = tid % TPP;
          const int npair = nr / 2;
          for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
            int rotated = 0;
            for (int rd = 0; rd < nr - 1; ++rd) {
              if (gj < npair) {
                int p, q;
                if (gj == 0) { p = nr - 1; q = rd; }
                else { p = (rd + gj) % (nr - 1); q = (rd - gj + nr - 1) % (nr - 1); }
                T xp[EPT], xq[EPT];
                T a = 0, b = 0, cc = 0;
  #pragma unroll
                for (int e = 0; e < EPT; ++e) {
                  const int k = l + TPP * e;
                  const int kc = (N2 % TPP == 0 || k < N2) ? k : 0;   // in bounds; masked below
                  xp[e] = bufR[p * LDT + kc];
                  xq[e] = bufR[q * LDT + kc];
                }
  #pragma unroll
                for (int e = 0; e < EPT; ++e) {
                  const T mk = (N2 % TPP == 0 || l + TPP * e < N2) ? T(1) : T(0);
                  xp[e] *= mk;
                  xq[e] *= mk;
                  a += xp[e] * xp[e];
                  b += xq[e] * xq[e];
                  cc += xp[e] * xq[e];
                }
                a = group_sum<TPP>(a);
                b = group_sum<TPP>(b);
                cc = group_sum<TPP>(cc);
                if (a > T(0) && b > T(0) && cc * cc > tol * tol * fmax(a, b)) {
                  T cs, sn;
                  jacobi_rot(a, b, cc, cs, sn);
  #pragma unroll
                  for (int e = 0; e < EPT; ++e) {
                    const int k = l + TPP * e;
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
        // ---- row norms, descending order, kept rows (normalised) into V ----
        {
          const int gj = tid / TPP, l = tid % TPP;
          for (int i0 = 0; i0 < N2; i0 += NT / TPP) {
            const int i = i0 + gj;
            T s2 = 0;
  #pragma unroll
            for (int e = 0; e < EPT; ++e) {
              const int k = l + TPP * e;
              const T x = (i < rank && k < NK) ? bufR[i * LDT + k] : T(0);
              s2 += x * x;
            }
            s2 = group_sum<TPP>(s2);
            if (l == 0 && i < N2) sc[i] = s2;
          }
        }
        __syncthreads();
        for (int i = tid; i < rank; i += NT) {
          int pos = i;
          if (rank > CHI) {   // only the CHI largest are kept; otherwise any order will do
            pos = 0;
            for (int j2 = 0; j2 < rank; ++j2) pos += (sc[j2] > sc[i]) || (sc[j2] == sc[i] && j2 < i);
          }
          ord[pos] = i;
        }
        __syncthreads();
        const int kept = rank < CHI ? rank : CHI;
        if (tid == 0) bdout[c] = static_cast<unsigned char>(kept);
        for (int o = tid; o < CHI * NK; o += NT) {
          const int al = o / NK, kk = o % NK;
          T val = 0;
          if (al < kept) {
            const int row = ord[al];
            const T s2 = sc[row];
            if (s2 > T(0)) val = bufR[row * LDT + kk] / sqrt(s2);
          }
          bufS[al * LDV + phys(perm[kk])] = val;
        }
        if constexpr (KW < CHI) {   // the columns (x, be >= KW) of V are zero
          constexpr int NZ = 2 * (CHI - KW);
          for (int o = tid; o < CHI * NZ; o += NT) {
            const int al = o / NZ, z = o % NZ;
            bufS[al * LDV + (z / (CHI - KW)) * CHI + KW + z % (CHI - KW)] = T(0);
          }
        }
        // small kept rows are orthogonal to the large ones only up to rot ||T|| / sigma: make the
        // kept rows orthonormal (span unchanged)
        // One pass suffices in the Gram form: the rows come from a pivoted Cholesky factor whose
        // conditioning is bounded by the FP32 rank tolerance, so FP64 Gram-Schmidt leaves them
        // orthonormal to ~1e-10; the QR form (FP64 environments, and FP32 arithmetic at
        // chi = 48) takes a second pass.
        if constexpr (GRAM) mgs_pairs_rows<T, CHI, NT, LDV, KW, (KW <= 16 ? 8 : TPP)>(bufS, kept, T(Tol::eta));
        else {
          // two passes, the rows taken two at a time (one barrier per pair), over the columns
          // (x, be < bdout[c+1]) only: the right bond of the new site bounds its nonzero columns
          const int bdr = bdout[c + 1];
          constexpr int KW1 = CHI > 16 ? 16 : CHI, KW2 = CHI > 24 ? 24 : CHI;
          const int kwm = bdr <= KW1 ? KW1 : bdr <= KW2 ? KW2 : CHI;
          for (int pass = 0; pass < 2; ++pass) {
            if (kwm == KW1) mgs_pairs_rows<T, CHI, NT, LDV, KW1>(bufS, kept, T(Tol::eta));
            else if (kwm == KW2) mgs_pairs_rows<T, CHI, NT, LDV, KW2>(bufS, kept, T(Tol::eta));
            else mgs_pairs_rows<T, CHI, NT, LDV>(bufS, kept, T(Tol::eta));
          }
        }
        gmem<E>* bout = Aout + size_t(c) * site;   // site c of E_{r-1}: B[x][al][be] = V[al][x*CHI + be]
        for (int o = tid; o < int(site); o += NT) {
          const int x = o / (CHI * CHI), al = (o / CHI) % CHI, be = o % CHI;
          gst<E>(bout, o, narrow<E>(bufS[al * LDV + x * CHI + be]));
        }
        // Xt_c = 2^-e_{c-1} Z V^T (N2 x CHI, column-major in bufR), then a power-of-two rescale
        const int ec = GRAM ? rexp[c - 1] : (rexp[c - 1] >> 8);
        T mx = 0;
        {
          auto xa = [&](int j, int col) { return Zr[j * LDZ + col]; };
          auto xb = [&](int col, int al) { return bufS[al * LDV + phys(col)]; };
          auto xc = [&](int j, int al, T val) {
            const T d = T(ldexp(val, -ec));
            bufR[al * LDT + phys(j)] = d;
            mx = fmax(mx, fabs(d));
          };
          if constexpr (KW < CHI) {   // the rows (a, al >= KW) of Xt_c are zero
            constexpr int NZ = 2 * (CHI - KW);
            for (int o = tid; o < CHI * NZ; o += NT) {
              const int al = o / NZ, z = o % NZ;
              bufR[al * LDT + (z / (CHI - KW)) * CHI + KW + z % (CHI - KW)] = T(0);
            }
          }
          if constexpr (MF64) {
            mfma_gemm_f64<NK, CHI, NK, NT>(xa, xb, xc);
          } else if constexpr (MF32) {
            // only the rows (a, al < bdin[c]) of Z, the kept rows of V and their columns
            // (x, be < bdout[c+1]) can be nonzero; the rest of Xt_c is written as zeros
            const int mtx = (bdin[c] + 15) / 16, ntx = (kept + 15) / 16;
            const int ktx = (bdout[c + 1] + 15) / 16;
            mfma_gemm_f32_blocks<NT, CHI, 2, 1, 2>(xa, xb, xc, mtx, ntx, ktx);
            for (int o = tid; o < CHI * N2; o += NT) {
              const int al = o / N2, j = o % N2;
              if (al >= 16 * ntx || j % CHI >= 16 * mtx) bufR[al * LDT + j] = T(0);
            }
          } else {
            gemm_tiles<TL, TL, N2, NT, T>(N2, CHI, xa, xb, xc);
          }
        }
        // the power-of-two rescale of Xt_c is applied to Z_{c-1} (per-wave maxima in red[])
        mx = wave_max(mx);
        if ((tid & (WAVE - 1)) == 0) red[tid / WAVE] = mx;
        return false;
      };
      bool row_done;
      if constexpr (ADAPT) {
        if (bdin[c] <= KWS && bdin[c + 1] <= KWS && bdout[c + 1] <= KWS)
          row_done = right_site(std::integral_constant<int, KWS>{});
        else
          row_done = right_site(std::integral_constant<int, CHI>{});
      } else {
        row_done = right_site(std::integral_constant<int, CHI>{});
      }
      if (row_done) break;
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

  // a non-finite log-norm of any row propagates into the last one (lambda_0)
  if (tid == 0 && R.status != nullptr && !isfinite(lambda)) atomicOr(R.status, TNMC_ST_LOGNORM);

  // ---------------- ln Z_TN from the top row ----------------
  if (lnZ_out != nullptr) {
    __syncthreads();
    const gmem<E>* A0 = env;   // row 0
    const gmem<const uint64_t>* jh0 = as_global(R.Jh);
    // (row 0's fields, if any, weight each site of E_0 by exp(beta h s))
    {
      T g0, g1;
      site_field_t<FLD, T>(R, 0, 0, ep, em, g0, g1);
      for (int o = tid; o < 2 * CHI; o += NT)
        sc[o] = (o >= CHI ? g1 : g0) * widen(gld<E>(A0, (o / CHI) * CHI * CHI + (o % CHI)));
    }
    double logacc = 0;
    for (int c = 1; c < L; ++c) {
      __syncthreads();
      const gmem<E>* A = A0 + size_t(c) * site;
      T mx = 0, val = 0;
      if (tid < 2 * CHI) {
        const int sp = tid / CHI, be = tid % CHI;
        T g0, g1;
        site_field_t<FLD, T>(R, 0, c, ep, em, g0, g1);
        for (int s2 = 0; s2 < 2; ++s2) {
          const T w = bond_weight<T>(jh0, c - 1, s2, sp, ep, em);
          T dd = 0;
          for (int al = 0; al < CHI; ++al) dd += sc[s2 * CHI + al] * widen(gld<E>(A, (sp * CHI + al) * CHI + be));
          val += w * dd;
        }
        val *= sp ? g1 : g0;
        mx = fabs(val);
      }
      mx = block_max<NT>(mx, red);
      const int e = pow2_exponent(mx);
      logacc += double(e) * 0.69314718055994530942;
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

template <typename T, typename E, int CHI, bool GRAM, bool FLD>
hipError_t launch_env_build(const DevReal* d_reals, int n, double* d_lnZ, hipStream_t stream) {
  using S = EnvSmem<T, CHI>;
  static_assert(S::NT == env_tpc(CHI) * S::N2, "one group of TPC threads per column");
  static_assert(env_tpp(CHI) * CHI <= S::NT && env_tpp(CHI) <= 64, "Jacobi pair groups");
  static_assert(2 * CHI <= S::NT, "");
  static_assert(S::NT % 64 == 0, "");
  static_assert(LeftCfg<CHI>::lds <= S::bufA, "left-sweep buffers fit in bufA");
  static_assert(LeftCfg<CHI>::TPC * LeftCfg<CHI>::RPT >= LeftCfg<CHI>::MQ, "rows covered");
  // Raise the dynamic-LDS limit once per device (not on every call, so that calls captured
  // into a HIP graph enqueue nothing but the launch).
  constexpr int MAX_DEVICES = 64;
  static std::once_flag once[MAX_DEVICES];
  static hipError_t attr[MAX_DEVICES];
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::call_once(once[dev], [dev] {
    attr[dev] = hipFuncSetAttribute(reinterpret_cast<const void*>(&env_build_kernel<T, E, CHI, GRAM, FLD>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(S::bytes));
  });
  if (attr[dev] != hipSuccess) return attr[dev];
  hipLaunchKernelGGL((env_build_kernel<T, E, CHI, GRAM, FLD>), dim3(n), dim3(S::NT), S::bytes, stream, d_reals,
                     d_lnZ);
  return hipGetLastError();
}

hipError_t env_build(tnmc_precision prec, int chi, bool fields, const DevReal* d_reals, int n,
                     double* d_lnZ, hipStream_t stream) {
#define TNMC_ENV_CASE(TY, EY, C, G)                                                       \
  case C:                                                                                 \
    return fields ? launch_env_build<TY, EY, C, G, true>(d_reals, n, d_lnZ, stream)       \
                  : launch_env_build<TY, EY, C, G, false>(d_reals, n, d_lnZ, stream);
#define TNMC_ENV_CHIS(TY, EY, G) \
  TNMC_ENV_CASE(TY, EY, 2, G) TNMC_ENV_CASE(TY, EY, 4, G) TNMC_ENV_CASE(TY, EY, 8, G) \
  TNMC_ENV_CASE(TY, EY, 16, G) TNMC_ENV_CASE(TY, EY, 32, G)
  // FP64 environments: Householder / pivoted-QR form in FP64.  FP32 and BF16 environments: Gram
  // form in FP64 arithmetic, results rounded to the storage type; at chi = 48 (where FP64 Gram
  // matrices do not fit the LDS) the QR form in FP32.
  if (prec == TNMC_FP64) {
    switch (chi) { TNMC_ENV_CHIS(double, double, false) }
  } else if (prec == TNMC_FP32) {
    switch (chi) {
      TNMC_ENV_CHIS(double, float, true)
      TNMC_ENV_CASE(float, float, 48, false)
      case 64: return env_build_big(prec, chi, false, fields, d_reals, n, d_lnZ, stream);
    }
  } else if (prec == TNMC_BF16) {
    switch (chi) {
      TNMC_ENV_CHIS(double, bf16_t, true)
      TNMC_ENV_CASE(float, bf16_t, 48, false)
      case 64: return env_build_big(prec, chi, false, fields, d_reals, n, d_lnZ, stream);
    }
  }
#undef TNMC_ENV_CHIS
#undef TNMC_ENV_CASE
  return hipErrorInvalidValue;
}

size_t env_build_scratch_bytes(tnmc_precision prec, int chi, int L) {
  // the LDS forms keep FP64: the carried R factor or Gram matrix of every site; the Gram form
  // with global scratch (chi = 64, or chosen) its own layout; the larger of the two
  const size_t lds_form = size_t(L) * 2 * chi * 2 * chi * sizeof(double);
  if (!env_build_big_ok(prec, chi)) return lds_form;
  const size_t big = env_build_big_scratch_bytes(prec, chi, L);
  return big > lds_form ? big : lds_form;
}

}  // namespace tnmc
