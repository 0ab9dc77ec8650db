// C ABI of the TNMC hot path (declared in include/tnmc.h): argument validation, workspace
// layout and kernel launches.  No exception crosses this layer; no device memory is allocated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "tnmc.h"

using namespace tnmc;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
// bytes of one stored environment element
inline size_t elem_bytes(tnmc_precision p) { return p == TNMC_FP64 ? 8 : (p == TNMC_FP32 ? 4 : 2); }

bool prec_ok(tnmc_precision p) { return p == TNMC_FP64 || p == TNMC_FP32 || p == TNMC_BF16; }
// chi = 48 and 64 exist for FP32 and BF16 environments only
bool chi_ok(int32_t chi, tnmc_precision p) {
  return chi == 2 || chi == 4 || chi == 8 || chi == 16 || chi == 32 ||
         ((chi == 48 || chi == 64) && p != TNMC_FP64);
}

// Basic per-instance checks; returns Lmax or -1.
int check_instances(const tnmc_instance* inst, int32_t n, bool need_env, bool need_J) {
  if (inst == nullptr || n < 1) return -1;
  int Lmax = 0;
  for (int i = 0; i < n; ++i) {
    const tnmc_instance& s = inst[i];
    if (s.L < 2 || s.L > 1024) return -1;
    if (!(s.beta > 0.0) || !std::isfinite(s.beta)) return -1;
    if (need_J && (s.d_Jh == nullptr || s.d_Jv == nullptr)) return -1;
    if (need_env && (s.d_env == nullptr || s.d_lognorm == nullptr)) return -1;
    Lmax = std::max(Lmax, int(s.L));
  }
  return Lmax;
}

size_t desc_bytes(int32_t n) { return align_up(size_t(n) * sizeof(DevReal)); }

size_t build_region(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision p) {
  size_t b = 0;
  for (int i = 0; i < n; ++i) b += align_up(env_build_scratch_bytes(p, chi, inst[i].L));
  return b;
}

size_t propose_region(const tnmc_instance* inst, int32_t n, int32_t chi, int32_t K,
                      tnmc_precision p) {
  size_t b = 0;
  for (int i = 0; i < n; ++i) b += align_up(propose_scratch_bytes(p, chi, inst[i].L, K));
  return b;
}

size_t accept_region(int32_t n, int32_t K) { return 2 * align_up(size_t(n) * K * sizeof(int32_t)); }

enum class Use { build, propose, none };

// Host data (the descriptor table, the coupling seeds) reaches the device as kernel arguments,
// not as a copy from pageable host memory: a kernel node of a captured HIP graph keeps its
// argument values, so a sequence of calls captured into a graph replays correctly.
constexpr int ARG_WORDS = 384;   // 3 KiB per launch, inside the 4 KiB kernel-argument block
struct ArgWords {
  uint64_t w[ARG_WORDS];
};

__global__ void __launch_bounds__(128) store_words_kernel(ArgWords a, uint64_t* dst, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = a.w[i];
}

hipError_t store_words(const uint64_t* src, size_t count, uint64_t* dst, hipStream_t stream) {
  for (size_t o = 0; o < count; o += ARG_WORDS) {
    ArgWords a;
    const size_t c = std::min<size_t>(ARG_WORDS, count - o);
    std::memcpy(a.w, src + o, c * sizeof(uint64_t));
    hipLaunchKernelGGL(store_words_kernel, dim3(1), dim3(128), 0, stream, a, dst + o, int(c));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Build the device descriptor table in the workspace; per-realization slices for `use`.  For the
// build and the proposals (workgroups whose runtime grows as L^2) the table lists the
// realizations by decreasing L, so that the longest workgroups are dispatched first; `slot`
// keeps each one's index in the caller's batch, which indexes every output.
hipError_t upload_desc(const tnmc_instance* inst, int32_t n, int32_t chi, int32_t K,
                       tnmc_precision p, Use use, void* ws, hipStream_t stream) {
  static_assert(sizeof(DevReal) % sizeof(uint64_t) == 0, "descriptor is whole words");
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  if (use == Use::build || use == Use::propose)
    std::stable_sort(order.begin(), order.end(),
                     [inst](int a, int b) { return inst[a].L > inst[b].L; });
  std::vector<DevReal> h(n);
  char* base = static_cast<char*>(ws) + desc_bytes(n);
  size_t off = 0;
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    DevReal& d = h[k];
    d.L = inst[i].L;
    d.slot = i;
    d.beta = inst[i].beta;
    d.id = inst[i].id;
    d.Jh = inst[i].d_Jh;
    d.Jv = inst[i].d_Jv;
    d.env = inst[i].d_env;
    d.lognorm = inst[i].d_lognorm;
    d.ws = base + off;
    d.status = inst[i].d_status;
    d.bonds = inst[i].d_bonds;
    d.field = inst[i].d_field;
    if (use == Use::build) off += align_up(env_build_scratch_bytes(p, chi, inst[i].L));
    else if (use == Use::propose) off += align_up(propose_scratch_bytes(p, chi, inst[i].L, K));
  }
  return store_words(reinterpret_cast<const uint64_t*>(h.data()),
                     sizeof(DevReal) * n / sizeof(uint64_t), static_cast<uint64_t*>(ws), stream);
}

inline tnmc_status hip_status(hipError_t e) { return e == hipSuccess ? TNMC_OK : TNMC_EHIP; }

// Scratch of tnmc_build_env_static: the descriptor table and the build scratch of its batch,
// in a file-scope device array (one copy per device, held until the process ends).  Host code
// never passes `scratch` itself to a kernel or a copy: it passes the device address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
static_assert(TNMC_STATIC_SCRATCH_BYTES % 256 == 0, "whole 256-byte blocks");
__device__ __align__(256) unsigned char scratch[TNMC_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::once_flag scratch_once[MAX_DEVICES];
void* scratch_ptr[MAX_DEVICES];
hipError_t scratch_err[MAX_DEVICES];

// Device address of this device's scratch array (looked up on the first call on each device,
// with that device current).
hipError_t static_scratch(void** out) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::call_once(scratch_once[dev], [dev] {
    scratch_err[dev] = hipGetSymbolAddress(&scratch_ptr[dev], HIP_SYMBOL(scratch));
    if (scratch_err[dev] == hipSuccess && scratch_ptr[dev] == nullptr)
      scratch_err[dev] = hipErrorInvalidSymbol;
  });
  if (scratch_err[dev] != hipSuccess) return scratch_err[dev];
  *out = scratch_ptr[dev];
  return hipSuccess;
}

// Tuning table of the proposal kernel's launch shape (wavefronts per workgroup), filled by
// tnmc_autotune_propose or tnmc_tune_set and read by every proposal launch.
using TuneKey = std::tuple<int, int, int, int, int>;   // chi, precision, Lmax, n, K
std::mutex tune_mu;
std::map<TuneKey, int> tune_table;

int tuned_waves(int chi, tnmc_precision prec, int Lmax, int n, int K) {
  std::lock_guard<std::mutex> g(tune_mu);
  auto it = tune_table.find(TuneKey(chi, int(prec), Lmax, n, K));
  return it == tune_table.end() ? 0 : it->second;
}

bool any_field(const tnmc_instance* inst, int32_t n) {
  for (int i = 0; i < n; ++i)
    if (inst[i].d_field != nullptr) return true;
  return false;
}

size_t torus_desc_bytes(int32_t n) { return align_up(size_t(n) * sizeof(DevTorus)); }

// Checks of a batch of tori and their blocks; returns the largest block side or -1.
int check_tori(const tnmc_torus* tor, const tnmc_instance* blk, int32_t n, bool need_block) {
  if (tor == nullptr || blk == nullptr || n < 1) return -1;
  int Lmax = 0;
  for (int i = 0; i < n; ++i) {
    const tnmc_torus& t = tor[i];
    if (t.L < 3 || t.L > 1024 || t.r0 < 0 || t.r0 >= t.L || t.c0 < 0 || t.c0 >= t.L) return -1;
    if (t.d_Jh == nullptr || t.d_Jv == nullptr || t.d_spins == nullptr) return -1;
    if (blk[i].L != t.L - 1) return -1;
    if (need_block && (blk[i].d_Jh == nullptr || blk[i].d_Jv == nullptr || blk[i].d_field == nullptr))
      return -1;
    Lmax = std::max(Lmax, int(blk[i].L));
  }
  return Lmax;
}

// The torus table in the workspace after the realization table.
hipError_t upload_tori(const tnmc_torus* tor, int32_t n, void* ws, hipStream_t stream) {
  static_assert(sizeof(DevTorus) % sizeof(uint64_t) == 0, "descriptor is whole words");
  std::vector<DevTorus> h(n);
  for (int i = 0; i < n; ++i) {
    h[i].L = tor[i].L;
    h[i].r0 = tor[i].r0;
    h[i].c0 = tor[i].c0;
    h[i].pad = 0;
    h[i].Jh = tor[i].d_Jh;
    h[i].Jv = tor[i].d_Jv;
    h[i].spins = tor[i].d_spins;
  }
  return store_words(reinterpret_cast<const uint64_t*>(h.data()),
                     sizeof(DevTorus) * n / sizeof(uint64_t),
                     reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + desc_bytes(n)), stream);
}

int batch_lmax(const tnmc_instance* inst, int32_t n) {
  int Lmax = 0;
  for (int i = 0; i < n; ++i) Lmax = std::max(Lmax, int(inst[i].L));
  return Lmax;
}

}  // namespace

extern "C" {

int tnmc_chi_supported(int32_t chi, tnmc_precision prec) { return prec_ok(prec) && chi_ok(chi, prec); }

size_t tnmc_env_bytes(int32_t L, int32_t chi, tnmc_precision prec) {
  if (L < 2 || L > 1024 || !prec_ok(prec) || !chi_ok(chi, prec)) return 0;
  return size_t(L) * L * 2 * chi * chi * elem_bytes(prec);
}

size_t tnmc_workspace_bytes(const tnmc_instance* inst, int32_t n, int32_t chi, int32_t K,
                            tnmc_precision prec) {
  if (check_instances(inst, n, false, false) < 0 || !prec_ok(prec) || !chi_ok(chi, prec) || K < 1)
    return 0;
  const size_t r = std::max({build_region(inst, n, chi, prec), propose_region(inst, n, chi, K, prec),
                             accept_region(n, K), align_up(sizeof(uint64_t) * n)});
  return desc_bytes(n) + r;
}

tnmc_status tnmc_make_couplings(const tnmc_instance* inst, int32_t n, const uint64_t* seeds,
                                double p, void* d_workspace, size_t workspace_bytes,
                                hipStream_t stream) {
  const int Lmax = check_instances(inst, n, false, true);
  if (Lmax < 0 || seeds == nullptr || !(p >= 0.0 && p <= 1.0) || d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + align_up(sizeof(uint64_t) * n)) return TNMC_ENOMEM;
  char* d = static_cast<char*>(d_workspace);
  hipError_t e = upload_desc(inst, n, 4, 1, TNMC_FP32, Use::none, d, stream);
  if (e == hipSuccess)
    e = store_words(seeds, size_t(n), reinterpret_cast<uint64_t*>(d + desc_bytes(n)), stream);
  if (e == hipSuccess)
    e = couplings_launch(reinterpret_cast<const DevReal*>(d), n,
                         reinterpret_cast<const uint64_t*>(d + desc_bytes(n)), p, Lmax, stream);
  return hip_status(e);
}

tnmc_status tnmc_build_env(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                           void* d_workspace, size_t workspace_bytes, double* d_lnZ,
                           hipStream_t stream) {
  if (check_instances(inst, n, true, true) < 0 || !prec_ok(prec) || !chi_ok(chi, prec) ||
      d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + build_region(inst, n, chi, prec)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(inst, n, chi, 1, prec, Use::build, d_workspace, stream);
  if (e != hipSuccess) return TNMC_EHIP;
  return hip_status(env_build(prec, chi, any_field(inst, n),
                              static_cast<const DevReal*>(d_workspace), n, d_lnZ, stream));
}

tnmc_status tnmc_build_env_form(const tnmc_instance* inst, int32_t n, int32_t chi,
                                tnmc_precision prec, int32_t form, void* d_workspace,
                                size_t workspace_bytes, double* d_lnZ, hipStream_t stream) {
  if (form == TNMC_FORM_DEFAULT)
    return tnmc_build_env(inst, n, chi, prec, d_workspace, workspace_bytes, d_lnZ, stream);
  if ((form != TNMC_FORM_GRAM_L2 && form != TNMC_FORM_ZIPUP) ||
      check_instances(inst, n, true, true) < 0 || !env_build_big_ok(prec, chi) ||
      d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + build_region(inst, n, chi, prec)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(inst, n, chi, 1, prec, Use::build, d_workspace, stream);
  if (e != hipSuccess) return TNMC_EHIP;
  return hip_status(env_build_big(prec, chi, form == TNMC_FORM_ZIPUP, any_field(inst, n),
                                  static_cast<const DevReal*>(d_workspace), n, d_lnZ, stream));
}

tnmc_status tnmc_build_env_static(const tnmc_instance* inst, int32_t n, int32_t chi,
                                  tnmc_precision prec, double* d_lnZ, hipStream_t stream) {
  if (check_instances(inst, n, true, true) < 0 || !prec_ok(prec) || !chi_ok(chi, prec))
    return TNMC_EINVAL;
  // checked before any HIP call: a batch beyond the fixed array is refused
  if (desc_bytes(n) + build_region(inst, n, chi, prec) > TNMC_STATIC_SCRATCH_BYTES)
    return TNMC_ENOMEM;
  void* ws = nullptr;
  if (static_scratch(&ws) != hipSuccess) return TNMC_EHIP;
  hipError_t e = upload_desc(inst, n, chi, 1, prec, Use::build, ws, stream);
  if (e != hipSuccess) return TNMC_EHIP;
  return hip_status(env_build(prec, chi, any_field(inst, n), static_cast<const DevReal*>(ws), n,
                              d_lnZ, stream));
}

// waves > 0 forces a launch shape; otherwise the tuning table's entry or the default
static tnmc_status propose_common(const tnmc_instance* inst, int32_t n, int32_t chi,
                                  tnmc_precision prec, int32_t K, uint64_t seed,
                                  uint64_t first_proposal, const uint64_t* d_teacher,
                                  void* d_workspace, size_t workspace_bytes, uint64_t* d_spins,
                                  double* d_logq, int32_t* d_E, uint32_t* d_fallbacks,
                                  hipStream_t stream, int waves = 0) {
  const int Lmax = check_instances(inst, n, true, true);
  if (Lmax < 0 || !prec_ok(prec) || !chi_ok(chi, prec) || K < 1 || d_workspace == nullptr ||
      d_logq == nullptr)
    return TNMC_EINVAL;
  if (d_teacher == nullptr && (d_spins == nullptr || d_E == nullptr)) return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + propose_region(inst, n, chi, K, prec)) return TNMC_ENOMEM;
  if (waves <= 0) waves = tuned_waves(chi, prec, Lmax, n, K);
  hipError_t e = upload_desc(inst, n, chi, K, prec, Use::propose, d_workspace, stream);
  if (e != hipSuccess) return TNMC_EHIP;
  e = propose(prec, chi, static_cast<const DevReal*>(d_workspace), n, K, Lmax, seed,
              first_proposal, d_teacher, d_spins, d_logq, d_E, d_fallbacks, waves, stream);
  if (e == hipSuccess && d_teacher == nullptr && any_field(inst, n))
    e = field_energy_launch(static_cast<const DevReal*>(d_workspace), n, K, Lmax, d_spins, d_E,
                            stream);
  return hip_status(e);
}

int32_t tnmc_propose_candidates(int32_t chi, int32_t* waves) {
  int32_t m = 0;
  for (int w : {1, 2, 4, 8})
    if (propose_waves_ok(chi, w)) {
      if (waves != nullptr) waves[m] = w;
      ++m;
    }
  return m;
}

tnmc_status tnmc_tune_set(int32_t chi, tnmc_precision prec, int32_t Lmax, int32_t n, int32_t K,
                          int32_t waves) {
  if (!prec_ok(prec) || !chi_ok(chi, prec) || Lmax < 2 || Lmax > 1024 || n < 1 || K < 1)
    return TNMC_EINVAL;
  if (waves != 0 && !propose_waves_ok(chi, waves)) return TNMC_EINVAL;
  std::lock_guard<std::mutex> g(tune_mu);
  const TuneKey key(chi, int(prec), Lmax, n, K);
  if (waves == 0) tune_table.erase(key);
  else tune_table[key] = waves;
  return TNMC_OK;
}

int32_t tnmc_tune_get(int32_t chi, tnmc_precision prec, int32_t Lmax, int32_t n, int32_t K) {
  if (!prec_ok(prec) || !chi_ok(chi, prec) || Lmax < 2 || Lmax > 1024 || n < 1 || K < 1) return 0;
  const int w = tuned_waves(chi, prec, Lmax, n, K);
  return w > 0 ? w : propose_default_waves(chi, n, K, Lmax);
}

tnmc_status tnmc_autotune_propose(const tnmc_instance* inst, int32_t n, int32_t chi,
                                  tnmc_precision prec, int32_t K, uint64_t seed,
                                  void* d_workspace, size_t workspace_bytes, uint64_t* d_spins,
                                  double* d_logq, int32_t* d_E, int32_t reps,
                                  int32_t* h_best_waves, float* h_ms, hipStream_t stream) {
  if (check_instances(inst, n, true, true) < 0 || !prec_ok(prec) || !chi_ok(chi, prec) || K < 1 ||
      reps < 1 || d_spins == nullptr || d_logq == nullptr || d_E == nullptr)
    return TNMC_EINVAL;
  if (d_workspace == nullptr) return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + propose_region(inst, n, chi, K, prec)) return TNMC_ENOMEM;
  int32_t cand[4];
  const int m = tnmc_propose_candidates(chi, cand);
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return TNMC_EHIP;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return TNMC_EHIP;
  }
  tnmc_status st = TNMC_OK;
  int best = 0;
  float best_ms = 0.f;
  for (int j = 0; j < m && st == TNMC_OK; ++j) {
    // one untimed launch, then reps timed ones (the same proposals every time)
    st = propose_common(inst, n, chi, prec, K, seed, 0, nullptr, d_workspace, workspace_bytes,
                        d_spins, d_logq, d_E, nullptr, stream, cand[j]);
    if (st == TNMC_OK && hipEventRecord(ev[0], stream) != hipSuccess) st = TNMC_EHIP;
    for (int t = 0; t < reps && st == TNMC_OK; ++t)
      st = propose_common(inst, n, chi, prec, K, seed, 0, nullptr, d_workspace, workspace_bytes,
                          d_spins, d_logq, d_E, nullptr, stream, cand[j]);
    float ms = 0.f;
    if (st == TNMC_OK && (hipEventRecord(ev[1], stream) != hipSuccess ||
                          hipEventSynchronize(ev[1]) != hipSuccess ||
                          hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
      st = TNMC_EHIP;
    if (st != TNMC_OK) break;
    ms /= float(reps);
    if (h_ms != nullptr) h_ms[j] = ms;
    if (best == 0 || ms < best_ms) {
      best = cand[j];
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st != TNMC_OK) return st;
  st = tnmc_tune_set(chi, prec, batch_lmax(inst, n), n, K, best);
  if (h_best_waves != nullptr) *h_best_waves = best;
  return st;
}

tnmc_status tnmc_propose(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                         int32_t K, uint64_t seed, uint64_t first_proposal, void* d_workspace,
                         size_t workspace_bytes, uint64_t* d_spins, double* d_logq, int32_t* d_E,
                         uint32_t* d_fallbacks, hipStream_t stream) {
  if (d_spins == nullptr || d_E == nullptr) return TNMC_EINVAL;
  return propose_common(inst, n, chi, prec, K, seed, first_proposal, nullptr, d_workspace,
                        workspace_bytes, d_spins, d_logq, d_E, d_fallbacks, stream);
}

tnmc_status tnmc_logq(const tnmc_instance* inst, int32_t n, int32_t chi, tnmc_precision prec,
                      int32_t K, const uint64_t* d_spins, void* d_workspace,
                      size_t workspace_bytes, double* d_logq, hipStream_t stream) {
  if (d_spins == nullptr) return TNMC_EINVAL;
  return propose_common(inst, n, chi, prec, K, 0, 0, d_spins, d_workspace, workspace_bytes,
                        nullptr, d_logq, nullptr, nullptr, stream);
}

tnmc_status tnmc_energy(const tnmc_instance* inst, int32_t n, int32_t K, const uint64_t* d_spins,
                        int32_t* d_E, void* d_workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  const int Lmax = check_instances(inst, n, false, true);
  if (Lmax < 0 || K < 1 || d_spins == nullptr || d_E == nullptr || d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(inst, n, 4, 1, TNMC_FP32, Use::none, d_workspace, stream);
  if (e == hipSuccess)
    e = energy_launch(static_cast<const DevReal*>(d_workspace), n, K, Lmax, d_spins, d_E, stream);
  if (e == hipSuccess && any_field(inst, n))
    e = field_energy_launch(static_cast<const DevReal*>(d_workspace), n, K, Lmax, d_spins, d_E,
                            stream);
  return hip_status(e);
}

tnmc_status tnmc_accept(const tnmc_instance* inst, int32_t n, int32_t n_chain, int32_t K,
                        const uint64_t* d_prop_spins, const double* d_prop_logq,
                        const int32_t* d_prop_E, uint64_t seed, uint64_t first_step,
                        uint64_t* d_chain_spins, int32_t* d_chain_E, double* d_chain_logq,
                        uint8_t* d_chain_init, uint8_t* d_accepted, int32_t* d_current,
                        double* d_accum, void* d_workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  const int Lmax = check_instances(inst, n, false, false);
  if (Lmax < 0 || n_chain < 1 || K < n_chain || K % n_chain != 0 || d_prop_spins == nullptr ||
      d_prop_logq == nullptr || d_prop_E == nullptr || d_chain_spins == nullptr ||
      d_chain_E == nullptr || d_chain_logq == nullptr || d_chain_init == nullptr ||
      d_accepted == nullptr || d_current == nullptr || d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n) + accept_region(n, K)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(inst, n, 4, K, TNMC_FP32, Use::none, d_workspace, stream);
  if (e != hipSuccess) return TNMC_EHIP;
  char* base = static_cast<char*>(d_workspace) + desc_bytes(n);
  int32_t* oldE = reinterpret_cast<int32_t*>(base);
  int32_t* fin = reinterpret_cast<int32_t*>(base + align_up(size_t(n) * K * sizeof(int32_t)));
  return hip_status(accept_launch(static_cast<const DevReal*>(d_workspace), n, n_chain, K, Lmax,
                                  d_prop_spins, d_prop_logq, d_prop_E, seed, first_step,
                                  d_chain_spins, d_chain_E, d_chain_logq, d_chain_init,
                                  d_accepted, d_current, d_accum, oldE, fin, stream));
}

tnmc_status tnmc_observables(const tnmc_instance* inst, int32_t n, int32_t n_chain,
                             const uint64_t* d_chain_spins, const int32_t* d_chain_E,
                             double* d_accum, void* d_workspace, size_t workspace_bytes,
                             hipStream_t stream) {
  const int Lmax = check_instances(inst, n, false, false);
  if (Lmax < 0 || n_chain < 1 || d_chain_spins == nullptr || d_chain_E == nullptr ||
      d_accum == nullptr || d_workspace == nullptr)
    return TNMC_EINVAL;
  if (workspace_bytes < desc_bytes(n)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(inst, n, 4, 1, TNMC_FP32, Use::none, d_workspace, stream);
  if (e == hipSuccess)
    e = observables_launch(static_cast<const DevReal*>(d_workspace), n, n_chain, Lmax,
                           d_chain_spins, d_chain_E, d_accum, stream);
  return hip_status(e);
}

tnmc_status tnmc_disorder_average(const double* d_accum, int32_t n, int32_t L, double beta,
                                  int32_t n_chain, double* d_out, hipStream_t stream) {
  if (d_accum == nullptr || d_out == nullptr || n < 1 || L < 2 || L > 1024 || n_chain < 1 ||
      !(beta > 0.0) || !std::isfinite(beta))
    return TNMC_EINVAL;
  return hip_status(disorder_average_launch(d_accum, n, L, beta, n_chain, d_out, stream));
}

tnmc_status tnmc_status_check(const tnmc_instance* inst, int32_t n, uint32_t* h_words,
                              hipStream_t stream) {
  if (inst == nullptr || n < 1) return TNMC_EINVAL;
  std::vector<uint32_t> w(size_t(n), 0u);
  for (int i = 0; i < n; ++i)
    if (inst[i].d_status != nullptr &&
        hipMemcpyAsync(&w[i], inst[i].d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, stream) !=
            hipSuccess)
      return TNMC_EHIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return TNMC_EHIP;
  bool fault = false;
  for (int i = 0; i < n; ++i) {
    if (h_words != nullptr) h_words[i] = w[i];
    fault = fault || (w[i] & TNMC_ST_FAULTS) != 0;
  }
  return fault ? TNMC_ENUMERIC : TNMC_OK;
}

size_t tnmc_pbc_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  return desc_bytes(n) + torus_desc_bytes(n);
}

tnmc_status tnmc_pbc_block(const tnmc_torus* tor, const tnmc_instance* blk, int32_t n,
                           uint64_t* d_block_spins, void* d_workspace, size_t workspace_bytes,
                           hipStream_t stream) {
  const int Lmax = check_tori(tor, blk, n, true);
  if (Lmax < 0 || d_block_spins == nullptr || d_workspace == nullptr) return TNMC_EINVAL;
  if (workspace_bytes < tnmc_pbc_workspace_bytes(n)) return TNMC_ENOMEM;
  hipError_t e = upload_desc(blk, n, 4, 1, TNMC_FP32, Use::none, d_workspace, stream);
  if (e == hipSuccess) e = upload_tori(tor, n, d_workspace, stream);
  if (e == hipSuccess)
    e = pbc_block_launch(reinterpret_cast<const DevTorus*>(static_cast<char*>(d_workspace) +
                                                           desc_bytes(n)),
                         static_cast<const DevReal*>(d_workspace), n, Lmax, d_block_spins, stream);
  return hip_status(e);
}

tnmc_status tnmc_pbc_merge(const tnmc_torus* tor, const tnmc_instance* blk, int32_t n,
                           const uint64_t* d_block_spins, int32_t* d_E_torus, void* d_workspace,
                           size_t workspace_bytes, hipStream_t stream) {
  const int Lmax = check_tori(tor, blk, n, false);
  if (Lmax < 0 || d_block_spins == nullptr || d_workspace == nullptr) return TNMC_EINVAL;
  if (workspace_bytes < tnmc_pbc_workspace_bytes(n)) return TNMC_ENOMEM;
  hipError_t e = upload_tori(tor, n, d_workspace, stream);
  if (e == hipSuccess)
    e = pbc_merge_launch(reinterpret_cast<const DevTorus*>(static_cast<char*>(d_workspace) +
                                                           desc_bytes(n)),
                         n, Lmax, d_block_spins, d_E_torus, stream);
  return hip_status(e);
}

const char* tnmc_status_string(tnmc_status s) {
  switch (s) {
    case TNMC_OK: return "ok";
    case TNMC_EINVAL: return "invalid argument";
    case TNMC_ENOMEM: return "workspace too small";
    case TNMC_EHIP: return "HIP call or kernel launch failed";
    case TNMC_ENUMERIC: return "non-finite values (see the realization status words)";
    case TNMC_ESTATE: return "inconsistent chain state";
  }
  return "unknown status";
}

}  // extern "C"
