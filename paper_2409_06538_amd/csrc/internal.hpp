// Host/device interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tnmc.h"

namespace tnmc {

// Device-side descriptor of one realization (built by the C ABI layer in the workspace).
struct DevReal {
  int L;
  int slot;   // index of this realization in the caller's batch (the table may be reordered)
  double beta;
  uint64_t id;
  const uint64_t* Jh;
  const uint64_t* Jv;
  void* env;
  double* lognorm;
  void* ws;   // this realization's slice of the workspace (call-specific use)
  uint32_t* status;   // numeric status word (TNMC_ST_* bits) or nullptr
  uint8_t* bonds;     // L x (L + 1) bond dimensions of the stored environments, or nullptr
  const int8_t* field;   // L x L integer site fields, or nullptr
};

// Device-side descriptor of one torus (periodic lattice) and its frozen lines.
struct DevTorus {
  int L, r0, c0, pad;
  const uint64_t* Jh;
  const uint64_t* Jv;
  uint64_t* spins;
};

// exp(beta h s) of an integer site field h for s = +1 (g0) and s = -1 (g1), from ep = e^beta and
// em = e^-beta (|h| <= 4 multiplications)
template <typename T>
__device__ __forceinline__ void field_weights(int h, T ep, T em, T& g0, T& g1) {
  const T u = h > 0 ? ep : em, v = h > 0 ? em : ep;
  T a = T(1), b = T(1);
  for (int k = 0, m = h < 0 ? -h : h; k < m; ++k) {
    a *= u;
    b *= v;
  }
  g0 = a;
  g1 = b;
}

// The weights of site (r, c) of a realization (1 without a field).
template <typename T>
__device__ __forceinline__ void site_field(const DevReal& R, int r, int c, T ep, T em, T& g0, T& g1) {
  g0 = T(1);
  g1 = T(1);
  if (R.field != nullptr) {
    const int h = R.field[size_t(r) * R.L + c];
    if (h != 0) field_weights<T>(h, ep, em, g0, g1);
  }
}

// The same, compiled away (weights 1) where the batch has no fields.
template <bool FLD, typename T>
__device__ __forceinline__ void site_field_t(const DevReal& R, int r, int c, T ep, T em, T& g0,
                                             T& g1) {
  if constexpr (FLD) {
    site_field<T>(R, r, c, ep, em, g0, g1);
  } else {
    g0 = T(1);
    g1 = T(1);
  }
}

hipError_t couplings_launch(const DevReal* d_reals, int n, const uint64_t* d_seeds, double p,
                            int Lmax, hipStream_t stream);

// fields: some realization of the batch has site fields (the kernels then read them)
hipError_t env_build(tnmc_precision prec, int chi, bool fields, const DevReal* d_reals, int n,
                     double* d_lnZ, hipStream_t stream);
size_t env_build_scratch_bytes(tnmc_precision prec, int chi, int L);
// The Gram form with global scratch (envbuild_big.hip): the build of chi = 64 (FP32 and BF16
// environments), and a selectable form at chi = 8 .. 48
int env_build_big_ok(tnmc_precision prec, int chi);
hipError_t env_build_big(tnmc_precision prec, int chi, bool zipup, bool fields,
                         const DevReal* d_reals, int n, double* d_lnZ, hipStream_t stream);
size_t env_build_big_scratch_bytes(tnmc_precision prec, int chi, int L);

// waves: wavefronts per workgroup of the proposal kernel (propose_waves_ok), 0 = default
hipError_t propose(tnmc_precision prec, int chi, const DevReal* d_reals, int n, int K, int Lmax,
                   uint64_t seed, uint64_t first, const uint64_t* d_teacher, uint64_t* d_spins,
                   double* d_logq, int32_t* d_E, uint32_t* d_fallbacks, int waves,
                   hipStream_t stream);
int propose_default_waves(int chi, int n, int K, int Lmax);
int propose_waves_ok(int chi, int waves);
size_t propose_scratch_bytes(tnmc_precision prec, int chi, int L, int K);

hipError_t energy_launch(const DevReal* d_reals, int n, int K, int Lmax, const uint64_t* d_spins,
                         int32_t* d_E, hipStream_t stream);
// adds -sum h s to d_E [n][K] for the realizations with fields
hipError_t field_energy_launch(const DevReal* d_reals, int n, int K, int Lmax,
                               const uint64_t* d_spins, int32_t* d_E, hipStream_t stream);

// Lmax: the largest block side (the row count of one block configuration in d_block_spins)
hipError_t pbc_block_launch(const DevTorus* d_tor, const DevReal* d_blk, int n, int Lmax,
                            uint64_t* d_block_spins, hipStream_t stream);
hipError_t pbc_merge_launch(const DevTorus* d_tor, int n, int Lmax, const uint64_t* d_block_spins,
                            int32_t* d_E_torus, hipStream_t stream);

hipError_t accept_launch(const DevReal* d_reals, int n, int n_chain, int K, int Lmax,
                         const uint64_t* d_prop_spins, const double* d_prop_logq,
                         const int32_t* d_prop_E, uint64_t seed, uint64_t first_step,
                         uint64_t* d_chain_spins, int32_t* d_chain_E, double* d_chain_logq,
                         uint8_t* d_chain_init, uint8_t* d_accepted, int32_t* d_current,
                         double* d_accum, int32_t* d_ws_oldE, int32_t* d_ws_final,
                         hipStream_t stream);

hipError_t observables_launch(const DevReal* d_reals, int n, int n_chain, int Lmax,
                              const uint64_t* d_chain_spins, const int32_t* d_chain_E,
                              double* d_accum, hipStream_t stream);

hipError_t disorder_average_launch(const double* d_accum, int n, int L, double beta, int n_chain,
                                   double* d_out, hipStream_t stream);

}  // namespace tnmc
