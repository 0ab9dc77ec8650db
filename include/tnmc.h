/*
 * tnmc.h -- C ABI of the MI355X tensor-network Monte Carlo (TNMC) hot path for the 2D +-J
 * random-bond Ising model (RBIM).
 *
 * Paper: T. Chen, E. Guo, W. Zhang, P. Zhang, Y. Deng, "Tensor network Monte Carlo simulations
 * for the two-dimensional random bond Ising model", arXiv:2409.06538.
 *
 * Problem (Sec. II, Sec. III A): an L x L square lattice with free boundaries, couplings
 * J_ij = +-1 on nearest-neighbour bonds, i.i.d. with P(J = -1) = p, energy
 * E(s) = -sum J_ij s_i s_j (Eq. (10)), Boltzmann weight exp(-beta E) (Eq. (1)).  TNMC contracts the
 * tensor network of Z (Eq. (2)) with bond dimension truncated to chi (Sec. II B), samples
 * whole-lattice proposals from the approximate conditionals q(s_i | s_<i) (Eqs. (4)-(6)) and
 * removes the truncation bias with the Metropolis filter (Eq. (3)).
 *
 * Conventions shared by every entry point
 *  - Rows r = 0..L-1 top to bottom, columns c = 0..L-1 left to right.  W(L) = ceil(L / 64).
 *  - Bit-packed +-1 values: bit (c % 64) of word (c / 64) is 1 iff the value is -1; padding bits
 *    are 0.  Couplings: Jh has L rows x W(L) words (bit c of row r is the bond (r,c)-(r,c+1),
 *    c < L-1); Jv has L-1 rows x W(L) words (bit c of row r is the bond (r,c)-(r+1,c)).
 *    Spins: one configuration is Lmax rows x W(Lmax) words, where Lmax is the largest L of the
 *    batch (rows and bits beyond a realization's own L are 0).
 *  - Pointers named d_* are DEVICE pointers owned by the caller; host arrays (tnmc_instance
 *    tables, seeds) are read during the call only.  The library allocates no device memory: every
 *    buffer, including the workspace, comes from the caller (sizes from the *_bytes queries).
 *  - Every call enqueues work on `stream` and returns without synchronising.  Argument errors are
 *    detected on the host and returned synchronously (nothing is enqueued then).  Launch failures
 *    return TNMC_EHIP.  No exception crosses this interface.
 *  - Results are a pure function of (inputs, seeds, counters, precision): re-running is
 *    bit-identical.  Random draws use Philox4x64-10 (Salmon et al., SC'11): draw i of the stream
 *    keyed (k0, k1) with counter words (c1, c2, c3) is word (i & 3) of the block at counter
 *    (i >> 2, c1, c2, c3), turned into u = (w >> 11) * 2^-53 in [0, 1).
 *  - Concurrent calls that share a workspace race; use one workspace per stream.
 *  - Every call enqueues kernel launches only (host tables and seeds travel as kernel
 *    arguments; no copies from host memory, no memsets), so a sequence of calls can be captured
 *    into a HIP graph and replayed: each replay uses the host values of the capture and the
 *    device buffers they name.  The first call of each (precision, chi) on a device should be
 *    made outside a capture (it raises the kernel's LDS limit once).
 */
#ifndef TNMC_H
#define TNMC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNMC_OK = 0,
  TNMC_EINVAL = -1,   /* bad argument (sizes, null pointers, unsupported chi or L) */
  TNMC_ENOMEM = -2,   /* workspace smaller than tnmc_workspace_bytes */
  TNMC_EHIP = -3,     /* a HIP call or kernel launch failed */
  TNMC_ENUMERIC = -4, /* tnmc_status_check: a realization's status word holds a fault bit */
  TNMC_ESTATE = -5    /* chain state inconsistent with the call */
} tnmc_status;

/* Storage precision of the environments.  What each mode computes in:
 *   TNMC_FP64  environments stored in FP64; build (Householder / pivoted QR) and sampler in FP64.
 *   TNMC_FP32  environments stored in FP32.  Build: at chi <= 32 the Gram form in FP64
 *              arithmetic (FP64 matrix-core products), each site rounded to FP32 when stored; at
 *              chi = 48 the QR form in FP32 arithmetic (FP32 matrix-core products).  Sampler:
 *              FP32 arithmetic (FP32 matrix-core tiles for chi a multiple of 16).
 *   TNMC_BF16  environments stored as bfloat16 (round to nearest even from the build's result of
 *              each site); build arithmetic as for TNMC_FP32; the sampler widens each staged site
 *              to FP32 and computes in FP32.
 * The stored, rounded tensors are the environments that later rows and the sampler use.  The
 * running log-normalisation of the environments, log q(s), energies' Boltzmann factors and the
 * acceptance ratio are FP64 in every mode.  Lower precision can only lower the acceptance rate:
 * the Metropolis step keeps the chain exact whatever q is (Eq. (3)). */
typedef enum { TNMC_FP64 = 0, TNMC_FP32 = 1, TNMC_BF16 = 2 } tnmc_precision;

/* One disorder realization.  An array of these (host memory) describes a batch. */
typedef struct {
  int32_t L;          /* lattice side, 2 <= L <= 1024 */
  int32_t pad_;
  double beta;        /* inverse temperature, > 0 (Nishimori line: ln((1-p)/p) / 2, Sec. III A) */
  uint64_t id;        /* realization id: third counter word of its proposal and accept streams */
  uint64_t* d_Jh;     /* L x W(L) words (written by tnmc_make_couplings, else caller-filled) */
  uint64_t* d_Jv;     /* (L-1) x W(L) words */
  void* d_env;        /* tnmc_env_bytes(L, chi, prec) bytes: written by tnmc_build_env */
  double* d_lognorm;  /* L doubles: lambda_r = ln ||E_r||_2, written by tnmc_build_env */
  uint32_t* d_status; /* one status word (TNMC_ST_* bits, OR-ed in by the kernels), or NULL */
  uint8_t* d_bonds;   /* L x (L + 1) bytes, or NULL: entry [r][c] bounds the bond between sites
                         c-1 and c of E_r (no stored entry of E_r beyond it is nonzero; entries
                         c = 0 and c = L are 1).  Written by tnmc_build_env; read by tnmc_propose
                         and tnmc_logq at chi = 64 to load only the nonzero block of each site
                         (the results are the same without it; NULL: whole sites are loaded). */
  int8_t* d_field;    /* L x L bytes (row-major, entry r * L + c), or NULL: integer site fields
                         h, -4 <= h <= 4, for a lattice that is a block of a larger system whose
                         other spins are held fixed (Sec. I: the block may be part of the
                         system; Sec. IV: the frozen lines act as external fields).  Site (r, c)
                         then carries the extra weight exp(beta h s), i.e. E(s) gains
                         -sum h s: tnmc_build_env (every form), tnmc_propose, tnmc_logq and
                         tnmc_energy all use it.  Written by tnmc_pbc_block, else by the caller. */
} tnmc_instance;

/* Bits of a realization's status word.  Kernels only set bits; the caller clears the word (any
 * device write of 0) and reads it with tnmc_status_check.  Fault bits: */
#define TNMC_ST_LOGNORM 0x1u   /* tnmc_build_env: a log-norm lambda_r or ln Z_TN is not finite */
#define TNMC_ST_WEIGHT 0x2u    /* tnmc_propose / tnmc_logq: a conditional weight Z_c(y) is NaN or
                                  infinite (p+ fell back to 1/2 there) */
#define TNMC_ST_LOGQ 0x4u      /* tnmc_propose / tnmc_logq: a log q(s) is not finite */
#define TNMC_ST_DELTA 0x8u     /* tnmc_accept: an acceptance exponent Delta is not finite */
#define TNMC_ST_FAULTS (TNMC_ST_LOGNORM | TNMC_ST_WEIGHT | TNMC_ST_LOGQ | TNMC_ST_DELTA)
/* Not a fault (the reading for vanishing weights after truncation): both conditional weights of
 * a site were <= 0 and p+ = 1/2 was used. */
#define TNMC_ST_FALLBACK 0x10u

/* Number of observable accumulators per realization (see tnmc_accept). */
#define TNMC_OBS_COUNT 9

/* Supported bond dimensions: chi in {2, 4, 8, 16, 32} for every precision, and chi = 48 for
 * TNMC_FP32 and TNMC_BF16; L in [2, 1024].  Returns 1 if supported, else 0. */
int tnmc_chi_supported(int32_t chi, tnmc_precision prec);

/* Bytes of one realization's environments: L rows x L sites x 2 x chi x chi elements of the
 * storage type (8, 4 or 2 bytes), layout
 * [r][c][sigma][alpha][beta] (sigma 0 <-> +1), zero-padded where the bond is smaller than chi. */
size_t tnmc_env_bytes(int32_t L, int32_t chi, tnmc_precision prec);

/* Workspace bytes needed by every entry point below for this batch (the maximum over the
 * calls, so one buffer serves them all; it holds the device copy of the instance table and the
 * per-call scratch).  K = proposals per
 * realization per call.  Returns 0 on invalid arguments. */
size_t tnmc_workspace_bytes(const tnmc_instance* inst, int32_t n, int32_t chi, int32_t K,
                            tnmc_precision prec);

/* a1 -- couplings (Sec. III A): bond k of realization i is antiferromagnetic iff
 * u_k < p, u_k = draw k of the stream keyed (seeds[i], 0) with counter words (0, 0, 0); the
 * L(L-1) horizontal bonds come first in row-major order (k = r(L-1) + c), then the vertical
 * bonds (k = L(L-1) + rL + c).  Writes d_Jh and d_Jv of every instance.  0 <= p <= 1. */
tnmc_status tnmc_make_couplings(const tnmc_instance* inst, int32_t n, const uint64_t* seeds,
                                double p, void* d_workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* a2 + a3 -- environments (Sec. II B).  For every realization: E_{L-1} = 1; for r = L-1..1,
 * E_{r-1} = compress_chi(T_r E_r) where T_r applies the row's Boltzmann matrices (Eq. (10)):
 * (T_r f)(x) = sum_y prod_c exp(beta Jv[r-1][c] x_c y_c) prod_c exp(beta Jh[r][c] y_c y_{c+1}) f(y).
 * compress_chi is the canonical SVD compression (left-orthonormalise by QR, then truncate
 * right to left keeping the chi largest singular values at every bond).  Each E_r is stored as a
 * unit-norm MPS in d_env (sites 1..L-1 right-orthonormal) with d_lognorm[r] = ln ||E_r||_2.
 * d_lnZ (n doubles, device, may be NULL) receives ln Z_TN = lambda_0 + ln sum_x H_0(x) E_0(x)/||E_0||.
 * The workspace must hold tnmc_workspace_bytes.  A non-finite lambda_r or ln Z_TN sets
 * TNMC_ST_LOGNORM in the realization's status word. */
tnmc_status tnmc_build_env(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                           void* d_workspace, size_t workspace_bytes, double* d_lnZ,
                           hipStream_t stream);

/* The same environments by a chosen form of the build.  TNMC_FORM_DEFAULT is tnmc_build_env.
 * TNMC_FORM_GRAM_L2 is the Gram form of the canonical compression with the per-site matrices in
 * the workspace (L2-resident) instead of LDS -- the form tnmc_build_env uses at chi = 64 --
 * available for TNMC_FP32 (FP64 arithmetic) and TNMC_BF16 (FP32 arithmetic, with a coarser
 * numerical-rank cut) environments at chi = 8, 16, 32, 48, 64.  Same arguments, layout and errors
 * as tnmc_build_env (TNMC_EINVAL for a form that does not exist at this chi and precision); the
 * two forms are the same compression, so their results agree to rounding and rank cut. */
#define TNMC_FORM_DEFAULT 0
#define TNMC_FORM_GRAM_L2 1
/* TNMC_FORM_ZIPUP: a different compression, the zip-up (Stoudenmire and White, New J. Phys. 12,
 * 055026 (2010); a contraction variant of Sec. II B): per row one sweep of SVD truncations over
 * the operator-applied MPS, without the orthonormalising sweep, right to left for the first row
 * applied and then alternating so that each sweep runs away from the orthogonality centre the
 * previous one left.  Cheaper than the canonical compression (no Gram matrices, half the
 * products) and less accurate (each cut keeps the leading directions of the swept block, not
 * the state's Schmidt directions), so it lowers the acceptance; the stored environments
 * alternate between right- and left-orthonormal sites, which the sampler does not depend on.
 * Same precisions and chi as TNMC_FORM_GRAM_L2. */
#define TNMC_FORM_ZIPUP 2
tnmc_status tnmc_build_env_form(const tnmc_instance* inst, int32_t n, int32_t chi,
                                tnmc_precision prec, int32_t form, void* d_workspace,
                                size_t workspace_bytes, double* d_lnZ, hipStream_t stream);

/* tnmc_build_env for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same environments, log-norms and
 * ln Z_TN, with no workspace argument.  The descriptor table and the build scratch of the batch
 * live in a fixed device array inside the library, TNMC_STATIC_SCRATCH_BYTES per device, held
 * until the process ends; the call allocates nothing.  A batch whose descriptor table plus build
 * scratch (the tnmc_build_env part of tnmc_workspace_bytes) exceeds that size returns
 * TNMC_ENOMEM before anything is enqueued.  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams, other threads) race and must be ordered by
 * the caller.  The first call on each device should be made outside a graph capture (it looks
 * up the array's device address and raises the kernel's LDS limit once). */
#define TNMC_STATIC_SCRATCH_BYTES (64u << 20)
tnmc_status tnmc_build_env_static(const tnmc_instance* inst, int32_t n, int32_t chi,
                                  tnmc_precision prec, double* d_lnZ, hipStream_t stream);

/* a4 + a5 -- K whole-lattice proposals per realization (Sec. II A-B, Eqs. (4)-(6)), sampled row
 * by row and, within a row, column by column from the cached environments: right partial sums
 * R_c(y) = sum_y' w_c(y,y') phi_{c+1}(y') A^{(c+1)}[y'] R_{c+1}(y') and a left running vector;
 * Z_c(y) = [w_{c-1}(s_{c-1},y)] phi_c(y) l A^{(c)}[y] R_c(y), phi_c(y) = exp(beta Jv[r-1][c] s[r-1][c] y),
 * w_c(y,y') = exp(beta Jh[r][c] y y'), and phi_c(y) also carries exp(beta h[r][c] y) where the
 * realization has fields (row 0 included; d_E then includes -sum h s).  Negative Z_c(y) count as 0; p+ = Z_c(+)/(Z_c(+)+Z_c(-))
 * (1/2 if the sum is 0 or not finite), clamped to [1e-12, 1-1e-12]; s = +1 iff u < p+ with u
 * = draw c of the stream keyed (seed, 1) with counter words (r, first_proposal + k, id).
 * Outputs per (realization i, proposal k): d_spins [n][K][Lmax][W(Lmax)] words, d_logq [n][K]
 * (FP64 sum of ln p+ or ln(1-p+), formed as the logarithm of the product of the conditionals with
 * its binary exponent kept apart), d_E [n][K] int32 exact energy (a5: E = 2U - N_B, U the number
 * of unsatisfied bonds).  d_fallbacks (n uint32, device, may be NULL) counts sites where p+ fell
 * back to 1/2 (accumulated, not reset).  Status word bits: TNMC_ST_WEIGHT where a weight was not
 * finite, TNMC_ST_FALLBACK where both weights were <= 0, TNMC_ST_LOGQ for a non-finite log q. */
tnmc_status tnmc_propose(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                         int32_t K, uint64_t seed, uint64_t first_proposal, void* d_workspace,
                         size_t workspace_bytes, uint64_t* d_spins, double* d_logq, int32_t* d_E,
                         uint32_t* d_fallbacks, hipStream_t stream);

/* Autotuner of the proposal kernel's launch shape: wavefronts per workgroup (16 proposals each
 * with matrix-core tiles, chi a multiple of 16; one thread per proposal otherwise).  Every shape
 * gives bit-identical outputs (each proposal's arithmetic does not depend on its workgroup); the
 * shape sets how many workgroups share each staged environment site and how many fill the chip.
 * The library keeps a tuning table keyed by (chi, prec, Lmax, n, K) that tnmc_propose and
 * tnmc_logq consult; without an entry they use the default (8 wavefronts for Lmax <= 64 when
 * the grid covers every CU, else 4). */

/* The candidate shapes at this chi: writes up to 4 values to waves (may be NULL), returns how
 * many. */
int32_t tnmc_propose_candidates(int32_t chi, int32_t* waves);

/* Set (waves = a candidate) or erase (waves = 0) the table entry of a batch shape. */
tnmc_status tnmc_tune_set(int32_t chi, tnmc_precision prec, int32_t Lmax, int32_t n, int32_t K,
                          int32_t waves);

/* The shape tnmc_propose uses for this batch shape (the table entry or the default); 0 on invalid
 * arguments. */
int32_t tnmc_tune_get(int32_t chi, tnmc_precision prec, int32_t Lmax, int32_t n, int32_t K);

/* Time every candidate on this batch (one untimed launch, then `reps` launches between two HIP
 * events on `stream`, proposals first_proposal = 0 with `seed`), store the fastest in the tuning
 * table and in *h_best_waves (host, may be NULL); h_ms (host, may be NULL) receives the mean
 * milliseconds per launch of each candidate in the order of tnmc_propose_candidates.  Arguments
 * as for tnmc_propose (d_fallbacks is not used); the outputs of the last timed launch are left
 * in d_spins, d_logq, d_E.  Synchronises the stream; not for use under graph capture. */
tnmc_status tnmc_autotune_propose(const tnmc_instance* inst, int32_t n, int32_t chi,
                                  tnmc_precision prec, int32_t K, uint64_t seed,
                                  void* d_workspace, size_t workspace_bytes, uint64_t* d_spins,
                                  double* d_logq, int32_t* d_E, int32_t reps,
                                  int32_t* h_best_waves, float* h_ms, hipStream_t stream);

/* log q(s) of given configurations (the same conditionals as tnmc_propose, with the spins read
 * from d_spins instead of drawn): d_spins [n][K][Lmax][W(Lmax)], d_logq [n][K]. */
tnmc_status tnmc_logq(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                      int32_t K, const uint64_t* d_spins, void* d_workspace,
                      size_t workspace_bytes, double* d_logq, hipStream_t stream);

/* a5 -- exact integer energies E(s) = -sum J_ij s_i s_j (Eq. (10)), minus sum h s where the
 * realization has fields, of d_spins [n][K][Lmax][W] into d_E [n][K]. */
tnmc_status tnmc_energy(const tnmc_instance* inst, int32_t n, int32_t K, const uint64_t* d_spins,
                        int32_t* d_E, void* d_workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* a6 -- independence Metropolis chains (Eq. (3) with g(s'|s) = q(s'), Appendix A).  Each
 * realization runs n_chain chains; chain j consumes proposals k = j*K/n_chain .. (j+1)*K/n_chain-1
 * in order (K % n_chain == 0).  Per step: Delta = (-beta E' - log q') - (-beta E - log q); accept
 * iff Delta >= 0 or u < exp(Delta), u = draw (first_step + t) of the stream keyed (seed, 2) with
 * counter words (j, id, 0), t the step index within the chain; a chain whose d_chain_init byte is
 * 0 takes its first proposal unconditionally (not counted as accepted) and sets the byte to 1.
 * Chain state [n][n_chain]: d_chain_spins (Lmax x W words each), d_chain_E, d_chain_logq,
 * d_chain_init -- read and updated.  Outputs: d_accepted [n][K] (1 = accepted), d_current [n][K]
 * int32 (proposal index the chain holds after that step, -1 = a configuration from before this
 * call).  If d_accum != NULL, the observables of Sec. III C of every chain after every step are
 * added to d_accum [n][TNMC_OBS_COUNT]: count, sum E, sum E^2, sum m^2, sum m^4, sum m_edge^2,
 * sum q, sum q^2, sum q^4 (q = overlap of chains 0 and 1, when n_chain >= 2; m_edge over the
 * sites L/4 .. 3L/4-1 of each edge, divided by 2L).  A non-finite Delta sets TNMC_ST_DELTA in the
 * realization's status word (the proposal is then rejected: the comparisons are false). */
tnmc_status tnmc_accept(const tnmc_instance* inst, int32_t n, int32_t n_chain, int32_t K,
                        const uint64_t* d_prop_spins, const double* d_prop_logq,
                        const int32_t* d_prop_E, uint64_t seed, uint64_t first_step,
                        uint64_t* d_chain_spins, int32_t* d_chain_E, double* d_chain_logq,
                        uint8_t* d_chain_init, uint8_t* d_accepted, int32_t* d_current,
                        double* d_accum, void* d_workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* Observables of the current chain states (one sample per chain), added to d_accum
 * [n][TNMC_OBS_COUNT] with the layout of tnmc_accept. */
tnmc_status tnmc_observables(const tnmc_instance* inst, int32_t n, int32_t n_chain,
                             const uint64_t* d_chain_spins, const int32_t* d_chain_E,
                             double* d_accum, void* d_workspace, size_t workspace_bytes,
                             hipStream_t stream);

/* f1 -- disorder averages of the sampled quantities (Sec. III C) over n realizations of one
 * lattice side L at inverse temperature beta, from their d_accum rows [n][TNMC_OBS_COUNT] (as
 * filled by tnmc_accept / tnmc_observables with n_chain chains per realization).  The thermal
 * average < > of realization i is its sum over its sample count (count / n_chain for the overlap,
 * formed once per step from chains 0 and 1); [ ] is the mean over the n realizations.  Writes
 * d_out[TNMC_AVG_COUNT] (device): [<E>], [<E^2>], [<m^2>], [<m^4>], [<m_edge^2>], [<q>], [<q^2>],
 * [<q^4>], [<q^2>^2], the Binder ratio Q_q = [<q^4>] / [<q^2>^2] (Eq. (15)), the overlap
 * susceptibility chi_q = (L^2 / T) ([<q^2>] - [<q>]^2) (Eq. (16)) and the edge susceptibility
 * chi_edge = L [<m_edge^2>] (Sec. III C).  The overlap entries need n_chain >= 2 (else they are 0
 * and Q_q is not a number).  Mixed-L batches average each L's rows separately. */
#define TNMC_AVG_COUNT 12
tnmc_status tnmc_disorder_average(const double* d_accum, int32_t n, int32_t L, double beta,
                                  int32_t n_chain, double* d_out, hipStream_t stream);

/* Numeric status of a batch: waits until `stream` has finished, then reads the status word of
 * every realization (0 where d_status is NULL) into h_words (n words, host memory, may be NULL).
 * Returns TNMC_ENUMERIC if any word holds a fault bit (TNMC_ST_FAULTS), TNMC_OK otherwise,
 * TNMC_EHIP if a HIP call fails.  It synchronises, so it cannot be captured into a HIP graph;
 * the words are not cleared. */
tnmc_status tnmc_status_check(const tnmc_instance* inst, int32_t n, uint32_t* h_words,
                              hipStream_t stream);

/* f4 -- periodic boundaries by a frozen line pair (Sec. IV).  A torus of side L (3 <= L <= 1024)
 * with couplings on its 2 L^2 bonds and one chain's configuration.  Each step freezes row r0 and
 * column c0; the other (L-1) x (L-1) spins form an open block whose site (a, b) is torus site
 * ((r0 + 1 + a) mod L, (c0 + 1 + b) mod L), with the frozen spins acting as fields on its
 * boundary.  A step is: tnmc_pbc_block, tnmc_build_env / tnmc_propose on the block (fields
 * included), tnmc_logq and tnmc_energy of the current block state into the chain state
 * (d_chain_init = 1), tnmc_accept with one chain per block, tnmc_pbc_merge. */
typedef struct {
  int32_t L;           /* torus side, 3 <= L <= 1024 */
  int32_t r0, c0;      /* frozen row and column of this step, 0 <= r0, c0 < L */
  int32_t pad_;
  const uint64_t* d_Jh;  /* L x W(L) words: bit c of row r is the bond (r,c)-(r,(c+1) mod L) */
  const uint64_t* d_Jv;  /* L x W(L) words: bit c of row r is the bond (r,c)-((r+1) mod L,c) */
  uint64_t* d_spins;     /* L x W(L) words: the chain's configuration (read; written by merge) */
} tnmc_torus;

/* Workspace bytes of tnmc_pbc_block / tnmc_pbc_merge for n tori. */
size_t tnmc_pbc_workspace_bytes(int32_t n);

/* The open block of each torus tor[i] (blk[i].L must be tor[i].L - 1): writes blk[i].d_Jh and
 * d_Jv (the block's bonds, the layout of tnmc_instance), blk[i].d_field (L_b x L_b fields: the sum
 * of J s_f over the frozen neighbours f of each block site) and the block's configuration into
 * d_block_spins [n][Lmax][W(Lmax)] (Lmax = largest blk[i].L; the layout of one chain's state). */
tnmc_status tnmc_pbc_block(const tnmc_torus* tor, const tnmc_instance* blk, int32_t n,
                           uint64_t* d_block_spins, void* d_workspace, size_t workspace_bytes,
                           hipStream_t stream);

/* Writes the block configurations d_block_spins [n][Lmax][W(Lmax)] back into tor[i].d_spins (the
 * frozen row and column kept) and, if d_E_torus != NULL, the torus energy -sum over the 2 L^2
 * bonds of J s s into d_E_torus [n]. */
tnmc_status tnmc_pbc_merge(const tnmc_torus* tor, const tnmc_instance* blk, int32_t n,
                           const uint64_t* d_block_spins, int32_t* d_E_torus, void* d_workspace,
                           size_t workspace_bytes, hipStream_t stream);

const char* tnmc_status_string(tnmc_status s);

#ifdef __cplusplus
}
#endif
#endif /* TNMC_H */
