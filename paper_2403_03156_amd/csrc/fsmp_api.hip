// fsmp_api.hip -- host runtime of libfsmp.so: the C ABI of include/fsmp.h.
//
// Builds the SER and overlap tables in FP64 on the host, validates every call,
// stages per-waveform metadata through pinned memory, groups chains by PE capacity
// and enqueues the prologue, chain and posterior kernels on the caller's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fsmp_internal.h"

using namespace fsmp;

namespace {

const char *kVersion = "fsmp-mi355x 0.1 (gfx950)";
std::string g_create_error = "no error";

// ---- the allocation-free variant of fsmp_sample (fsmp_sample_noalloc)
// Its device workspace: one array per GPU in the code object, held until the process ends.
// Host code must not use the array's name as a device address: it takes the address
// hipGetSymbolAddress gives on each device (scratch_address), once per device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
// its host-side per-waveform arrays, for batches of up to these sizes
constexpr int64_t kNoAllocMaxWave = 65536, kNoAllocMaxChains = 262144;
struct NoAllocHost {
  int32_t kmx[kNoAllocMaxWave], gr[2 * kNoAllocMaxWave], order[kNoAllocMaxChains];
  double t0i[kNoAllocMaxWave];
  uint64_t wid[kNoAllocMaxWave];
  int64_t mfo[kNoAllocMaxWave + 1], ws[kNoAllocMaxWave];
};
NoAllocHost g_na;
std::mutex g_na_mutex;  // one allocation-free call at a time in the process (they share g_na)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (which must be `device`)
hipError_t scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ex-Gaussian density (Sec. 3): Gaussian N(mu, sigma^2) convolved with Exp(mean tau)
double exg(double t, double mu, double sigma, double tau) {
  const double a = sigma * sigma / tau;
  return std::exp((2.0 * mu + a - 2.0 * t) / (2.0 * tau)) * std::erfc((mu + a - t) / (std::sqrt(2.0) * sigma)) /
         (2.0 * tau);
}

double gauss(double t, double mu, double sigma) {
  const double u = (t - mu) / sigma;
  return std::exp(-0.5 * u * u) / (sigma * std::sqrt(2.0 * M_PI));
}

// Mode of the ex-Gaussian: its derivative is (g - f) / tau with g the Gaussian
// density, so the mode is the single sign change of g - f; bisection.
double exg_mode(double mu, double sigma, double tau) {
  double lo = mu - 10.0 * sigma, hi = mu + 10.0 * sigma + 10.0 * tau;
  for (int it = 0; it < 300; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (gauss(mid, mu, sigma) - exg(mid, mu, sigma, tau) > 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

struct Tables {
  int LV = 0, M = 0, sub = 0;
  std::vector<double> vtab, ovl;
};

bool build_tables(const fsmp_ser &ser, int sub, Tables &t, std::string &err) {
  const double tm = exg_mode(ser.mu, ser.sigma, ser.tau);
  const double fm = exg(tm, ser.mu, ser.sigma, ser.tau);
  if (!(fm > 0.0) || !std::isfinite(fm)) {
    err = "SER: density not positive at its mode";
    return false;
  }
  int LV = ser.support;
  if (LV == 0) {
    LV = 0;
    for (int L = 16; L <= 8192; L += 16)
      if ((double)L > tm && exg((double)L, ser.mu, ser.sigma, ser.tau) / fm < 1e-6) {
        LV = L;
        break;
      }
    if (LV == 0) {
      err = "SER: automatic support exceeds 8192 samples";
      return false;
    }
  }
  if (LV < 1 || LV > 512) {
    err = "SER: support must be 1..512 samples";
    return false;
  }
  t.LV = LV;
  t.sub = sub;
  t.M = sub * LV;
  t.vtab.assign(t.M, 0.0);
  for (int m = 0; m < t.M; ++m) t.vtab[m] = ser.amplitude * exg((double)m / sub, ser.mu, ser.sigma, ser.tau) / fm;
  // stationary overlaps: O[p][d] = sum_n V(n - p/sub) V(n - (p + d)/sub), d >= 0
  t.ovl.assign((size_t)sub * t.M, 0.0);
  for (int p = 0; p < sub; ++p)
    for (int d = 0; d < t.M; ++d) {
      double s = 0.0;
      const int g2 = p + d;
      const int n0 = (g2 + sub - 1) / sub;       // first sample of the later column
      const int n1 = (p + t.M - 1) / sub;        // last sample of the earlier column
      for (int n = n0; n <= n1; ++n) s += t.vtab[sub * n - p] * t.vtab[sub * n - g2];
      t.ovl[(size_t)p * t.M + d] = s;
    }
  return true;
}

template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  hipError_t ensure(size_t want) {
    if (want <= n && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    size_t cap = std::max<size_t>(want, 1);
    hipError_t e = hipMalloc((void **)&p, cap * sizeof(T));
    if (e == hipSuccess) n = cap;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct PinBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, std::max<size_t>(want, 64), hipHostMallocDefault);
    if (e == hipSuccess) bytes = std::max<size_t>(want, 64);
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

}  // namespace

struct fsmp_ctx {
  int device = 0;
  fsmp_ser ser{};
  fsmp_intensity phi{};
  fsmp_config cfg{};
  Tables tab;
  ModelDev md{};
  double *d_vtab = nullptr, *d_ovl = nullptr;
  // workspace
  DevBuf<int64_t> woff, mfoff;
  DevBuf<double> lam, t0init, mf;
  DevBuf<int32_t> kmax, grange, chains;
  DevBuf<uint64_t> wid;
  DevBuf<int32_t> wsteps;  // per-waveform sweeps (fsmp_batch.n_steps)
  DevBuf<int32_t> zinit;   // initial PE lists (fsmp_batch.z_init) and their chain offsets
  DevBuf<int64_t> zinit_off;
  DevBuf<int64_t> lwoff;    // fsmp_lucy: offsets, kmax, the unit-sum SER kernel
  DevBuf<int32_t> lkmax;
  DevBuf<double> lkern;
  DevBuf<int64_t> poff;    // fsmp_posterior: the batch offsets of the occupancy rows
  DevBuf<double> plam;     // fsmp_posterior: lambda0 per waveform for lambda-hat
  DevBuf<uint32_t> wflags;
  DevBuf<double> lane_d;
  DevBuf<int32_t> lane_i;
  DevBuf<double> draw_scr;  // charge draws: KCAP (KCAP + 1) FP64 words per chain
  DevBuf<double> ptab;      // light-curve partial-sum factors (ModelDev::ptab)
  // per PE capacity (kCaps), FSMP_DESIGN_*: 0 = lane group per chain, H in LDS
  // (capacities up to 64); 1 = one lane per chain, state in device memory; 2 = lane group
  // per chain, H in device memory.  Defaults from the batched 100k-waveform measurement:
  // one lane per chain wins at capacity 16 (few PEs, the serial work shared by 64 chains),
  // the device-memory groups everywhere above.
  int design[kNumCaps] = {1, 2, 2, 2, 2, 2, 2, 2};
  PinBuf stage;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  bool timing = false;
  bool serial = false;  // the autotuner's trials: the buckets one after the other on the call's stream
  // per PE capacity the autotuner's trial time (ms) of the design it chose, and that design
  // (-1: none); fsmp_sample takes them as the buckets' costs when it deals them to streams
  double tuned_ms[kNumCaps] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int tuned_design[kNumCaps] = {-1, -1, -1, -1, -1, -1, -1, -1};
  hipStream_t capture = nullptr;  // set while fsmp_graph_create captures the kernels
  hipGraph_t captured = nullptr;
  std::vector<fsmp_timing> timings;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_events;
  std::vector<hipEvent_t> evpool;
  // capacity buckets run concurrently: on the caller's stream and on side streams forked
  // from and joined back into it with events
  hipStream_t side[kNumCaps] = {};
  hipEvent_t fork = nullptr, join[kNumCaps] = {};
  // this device's copy of the allocation-free variant's scratch array (null if its address
  // could not be taken)
  unsigned char *scratch = nullptr;
  std::string err = "no error";
};

namespace {

fsmp_status fail(fsmp_ctx *c, fsmp_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return s;
}

bool finite(double v) { return std::isfinite(v); }

// whether a kernel design exists for a PE capacity under this model (LDS footprint),
// precision and charge law: the FP32 form and the mixture law run only in the lane groups
// with G^-1 in device memory (the FP32 form without capacity 48, which it runs at 64); one
// lane per chain exists at capacities 16 and 32 (FP64); the wide device-memory groups from
// capacity 32 up (FP64, single charge law)
bool design_available(const fsmp_ctx *c, int kcap, int design) {
  const bool fp32 = c->cfg.precision == FSMP_FP32_REFRESH;
  const bool mcp = c->cfg.n_mix > 0;
  switch (design) {
    case FSMP_DESIGN_GROUP: return !fp32 && !mcp && chain_kcap_supported(kcap, c->tab.M, c->cfg.grid_sub);
    case FSMP_DESIGN_LANE: return !fp32 && !mcp && (kcap == 16 || kcap == 32);
    case FSMP_DESIGN_GROUP_DEVMEM: return chain_dm_supported(kcap, c->tab.M, c->cfg.grid_sub, fp32, mcp);
    case FSMP_DESIGN_GROUP_DEVMEM_WIDE:
      return !mcp && chain_dm_supported(kcap, c->tab.M, c->cfg.grid_sub, fp32, false, true);
    default: return false;
  }
}

// the design a bucket runs in: the context's choice where it exists, else the lane groups
// with G^-1 in device memory
int effective_design(const fsmp_ctx *c, int kcap, int design) {
  if (design_available(c, kcap, design)) return design;
  return FSMP_DESIGN_GROUP_DEVMEM;
}

fsmp_status validate_model(const fsmp_ser *ser, const fsmp_intensity *phi, const fsmp_config *cfg, std::string &m) {
  char b[256];
  if (!ser || !phi || !cfg) return m = "null model pointer", FSMP_EINVAL;
  if (!finite(ser->mu) || !(ser->sigma > 0) || !(ser->tau > 0) || !finite(ser->sigma) || !finite(ser->tau))
    return m = "SER: need finite mu, sigma > 0, tau > 0", FSMP_EINVAL;
  if (!finite(ser->amplitude) || ser->amplitude < 0) return m = "SER: amplitude must be finite and >= 0", FSMP_EINVAL;
  if (ser->support < 0 || ser->support > 512) return m = "SER: support must be 0 (auto) or 1..512", FSMP_EINVAL;
  if (phi->kind != FSMP_PHI_EXP && phi->kind != FSMP_PHI_BIEXP) return m = "phi: unknown kind", FSMP_EINVAL;
  if (!(phi->tau_decay > 0) || !finite(phi->tau_decay)) return m = "phi: tau_decay must be > 0", FSMP_EINVAL;
  if (phi->kind == FSMP_PHI_BIEXP && (!(phi->tau_rise > 0) || !finite(phi->tau_rise)))
    return m = "phi: BIEXP needs tau_rise > 0", FSMP_EINVAL;
  if (!finite(phi->t0_min) || !finite(phi->t0_max) || phi->t0_min > phi->t0_max)
    return m = "phi: need finite t0_min <= t0_max", FSMP_EINVAL;
  if (!(cfg->sigma_eps > 0) || !finite(cfg->sigma_eps)) return m = "config: sigma_eps must be > 0", FSMP_EINVAL;
  if (!(cfg->sigma_q > 0) || !finite(cfg->sigma_q) || !finite(cfg->mu_q))
    return m = "config: need finite mu_q and sigma_q > 0", FSMP_EINVAL;
  if (cfg->grid_sub < 1 || cfg->grid_sub > 16) return m = "config: grid_sub must be 1..16", FSMP_EINVAL;
  if (!(cfg->jump_J > 0) || !(cfg->jump_J < 0.5)) return m = "config: jump_J must be in (0, 1/2)", FSMP_EINVAL;
  if (!(cfg->t0_step_sd > 0) || !(cfg->shift_sd > 0) || !finite(cfg->t0_step_sd) || !finite(cfg->shift_sd))
    return m = "config: step sizes must be > 0", FSMP_EINVAL;
  if (cfg->k_max < 1 || cfg->k_max > 192) return m = "config: k_max must be 1..192", FSMP_EINVAL;
  if (cfg->n_steps < 0 || cfg->n_chains < 1 || cfg->burn_in < 0 || cfg->burn_in > cfg->n_steps) {
    snprintf(b, sizeof b, "config: need n_steps >= 0, n_chains >= 1, 0 <= burn_in <= n_steps (got %d %d %d)",
             cfg->n_steps, cfg->n_chains, cfg->burn_in);
    return m = b, FSMP_EINVAL;
  }
  if ((cfg->record_flags & FSMP_REC_TRACE) && cfg->thin < 1) return m = "config: trace needs thin >= 1", FSMP_EINVAL;
  if ((cfg->record_flags & FSMP_REC_CHARGE) && cfg->thin < 1) return m = "config: charge draws need thin >= 1", FSMP_EINVAL;
  if (cfg->record_flags & ~(uint32_t)(FSMP_REC_TRACE | FSMP_REC_LOG | FSMP_REC_CHARGE))
    return m = "config: unknown record flag", FSMP_EINVAL;
  if (cfg->precision != FSMP_FP64 && cfg->precision != FSMP_FP32_REFRESH) return m = "config: unknown precision", FSMP_EINVAL;
  if (cfg->refresh_M < 0) return m = "config: refresh_M must be >= 0", FSMP_EINVAL;
  if (cfg->n_mix < 0 || cfg->n_mix > 8) return m = "config: n_mix must be 0..8", FSMP_EINVAL;
  if (cfg->n_mix > 0) {
    double wsum = 0.0;
    for (int e = 0; e < cfg->n_mix; ++e) {
      if (!(cfg->mix_weight[e] > 0) || !finite(cfg->mix_weight[e]) || !finite(cfg->mix_mu[e]) ||
          !(cfg->mix_sigma[e] > 0) || !finite(cfg->mix_sigma[e]))
        return m = "config: mixture components need weight > 0, finite mu and sigma > 0", FSMP_EINVAL;
      wsum += cfg->mix_weight[e];
    }
    if (std::fabs(wsum - 1.0) > 1e-9) return m = "config: mixture weights must sum to 1", FSMP_EINVAL;
    if (cfg->precision != FSMP_FP64) return m = "config: the mixture charge law runs in FP64 only", FSMP_ENOTSUP;
  }
  return FSMP_OK;
}

void fill_model(fsmp_ctx *c) {
  ModelDev &md = c->md;
  const fsmp_config &cf = c->cfg;
  md.s = cf.sigma_eps * cf.sigma_eps;
  md.inv_s = 1.0 / md.s;
  md.rho = md.s / (cf.sigma_q * cf.sigma_q);
  md.log_rho = std::log(md.rho);
  md.m = cf.mu_q;
  md.rhom = md.rho * cf.mu_q;
  md.rhom2 = md.rho * cf.mu_q * cf.mu_q;
  // mixture: weights accumulated in index order (the component draw compares a uniform with
  // these partial sums), and the per-component ridge terms
  md.n_mix = cf.n_mix;
  double cdf = 0.0;
  for (int e = 0; e < 8; ++e) {
    if (e < cf.n_mix) {
      cdf += cf.mix_weight[e];
      const double rho = md.s / (cf.mix_sigma[e] * cf.mix_sigma[e]);
      md.mix_cdf[e] = cdf;
      md.mix_rho[e] = rho;
      md.mix_lrho[e] = std::log(rho);
      md.mix_rhom[e] = rho * cf.mix_mu[e];
      md.mix_rhom2[e] = rho * cf.mix_mu[e] * cf.mix_mu[e];
    } else {
      md.mix_cdf[e] = md.mix_rho[e] = md.mix_lrho[e] = md.mix_rhom[e] = md.mix_rhom2[e] = 0.0;
    }
  }
  md.sub = c->tab.sub;
  md.LV = c->tab.LV;
  md.M = c->tab.M;
  md.dt = 1.0 / cf.grid_sub;
  md.kind = c->phi.kind;
  const double t2 = c->phi.tau_decay;
  md.inv_tau2 = 1.0 / t2;
  md.log_tau2 = std::log(t2);
  md.den2 = -std::expm1(-md.dt / t2);
  if (md.kind == FSMP_PHI_BIEXP) {
    const double t1 = c->phi.tau_rise;
    const double t12 = 1.0 / (1.0 / t1 + 1.0 / t2);
    md.inv_tau1 = 1.0 / t1;
    md.inv_tau12 = 1.0 / t12;
    md.C = (t1 + t2) / (t2 * t2);
    md.logC = std::log(md.C);
    md.den12 = -std::expm1(-md.dt / t12);
  } else {
    md.inv_tau1 = 0.0;
    md.inv_tau12 = 0.0;
    md.C = 1.0 / t2;
    md.logC = -md.log_tau2;
    md.den12 = 1.0;
  }
  md.sub_shift = -1;
  for (int k = 0; k < 31; ++k)
    if ((1 << k) == md.sub) md.sub_shift = k;
  md.t0_min = c->phi.t0_min;
  md.t0_max = c->phi.t0_max;
  md.t0_sd = cf.t0_step_sd;
  md.shift_sd = cf.shift_sd;
  md.J = cf.jump_J;
  md.logJ = std::log(cf.jump_J);
}

// Table of 1 - e^{-k dt / tau} (tau2, then tau12; 0 for EXP) for k = 0 .. n - 1, n >= need:
// the count-dependent factors of the light curve's partial sums.  Grown (never shrunk) when
// a batch has a longer solution space; earlier launches of this context are waited for
// before the old table is released.
hipError_t ensure_ptab(fsmp_ctx *c, int64_t need) {
  if (c->md.ptab && c->md.ptab_n >= need) return hipSuccess;
  const int64_t n = std::max<int64_t>(need, 4 * 4096 + 1);
  std::vector<double> h(2 * (size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    const double kdt = (double)k * c->md.dt;
    h[2 * k] = -std::expm1(-kdt * c->md.inv_tau2) / c->md.den2;
    h[2 * k + 1] = c->md.kind == FSMP_PHI_EXP ? 0.0 : -std::expm1(-kdt * c->md.inv_tau12) / c->md.den12;
  }
  (void)hipDeviceSynchronize();
  c->ptab.release();
  hipError_t e = c->ptab.ensure(2 * (size_t)n);
  if (e == hipSuccess) e = hipMemcpy(c->ptab.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    c->md.ptab = nullptr;
    c->md.ptab_n = 0;
    return e;
  }
  c->md.ptab = c->ptab.p;
  c->md.ptab_n = n;
  return hipSuccess;
}

hipEvent_t pool_event(fsmp_ctx *c, size_t i) {
  while (c->evpool.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->evpool.push_back(e);
  }
  return c->evpool[i];
}

}  // namespace

extern "C" {

const char *fsmp_version(void) { return kVersion; }

const char *fsmp_last_error(const fsmp_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

fsmp_status fsmp_create(fsmp_ctx **out, const fsmp_ser *ser, const fsmp_intensity *phi, const fsmp_config *cfg,
                        int device) {
  if (!out) return fail(nullptr, FSMP_EINVAL, "out is NULL");
  *out = nullptr;
  std::string m;
  fsmp_status s = validate_model(ser, phi, cfg, m);
  if (s != FSMP_OK) return fail(nullptr, s, "%s", m.c_str());
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(nullptr, FSMP_EDEVICE, "no HIP device");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, FSMP_EDEVICE, "device %d out of range (%d devices)", device, ndev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, FSMP_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, FSMP_EDEVICE, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
  fsmp_ctx *c = new fsmp_ctx();
  c->device = device;
  c->ser = *ser;
  c->phi = *phi;
  c->cfg = *cfg;
  if (!build_tables(c->ser, cfg->grid_sub, c->tab, m)) {
    delete c;
    return fail(nullptr, FSMP_EINVAL, "%s", m.c_str());
  }
  fill_model(c);
  for (int q = 0; q < kNumCaps; ++q)
    if (!design_available(c, kCaps[q], c->design[q])) c->design[q] = FSMP_DESIGN_GROUP_DEVMEM;
  if (const char *d = std::getenv("FSMP_CHAIN_DESIGN")) {
    // tuning override: one letter per capacity in kCaps order, g (lane group, H in LDS),
    // l (lane), d (lane group, H in device memory), w (its wide groups); a design that does
    // not exist for a capacity leaves its default
    const size_t L = std::strlen(d);
    for (int q = 0; q < kNumCaps && q < (int)L; ++q) {
      const int want = d[q] == 'g' ? FSMP_DESIGN_GROUP : d[q] == 'l' ? FSMP_DESIGN_LANE
                       : d[q] == 'd' ? FSMP_DESIGN_GROUP_DEVMEM : d[q] == 'w' ? FSMP_DESIGN_GROUP_DEVMEM_WIDE : -1;
      if (want >= 0 && design_available(c, kCaps[q], want)) c->design[q] = want;
    }
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(device);
  hipError_t e = hipMalloc((void **)&c->d_vtab, sizeof(double) * c->tab.M);
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_ovl, sizeof(double) * c->tab.ovl.size());
  if (e == hipSuccess) e = hipMemcpy(c->d_vtab, c->tab.vtab.data(), sizeof(double) * c->tab.M, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_ovl, c->tab.ovl.data(), sizeof(double) * c->tab.ovl.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming);
  if (e == hipSuccess) e = ensure_ptab(c, 0);
  if (e == hipSuccess) {
    // set-up of the allocation-free variant: the device address of its scratch array
    void *sp = nullptr;
    if (scratch_address(device, &sp) == hipSuccess) c->scratch = (unsigned char *)sp;
    (void)hipGetLastError();
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    fsmp_destroy(c);
    return fail(nullptr, FSMP_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return FSMP_OK;
}

void fsmp_destroy(fsmp_ctx *c) {
  if (!c) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  if (c->stage_done) {
    (void)hipEventSynchronize(c->stage_done);
    (void)hipEventDestroy(c->stage_done);
  }
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  for (int q = 0; q < kNumCaps; ++q) {
    if (c->side[q]) {
      (void)hipStreamSynchronize(c->side[q]);
      (void)hipStreamDestroy(c->side[q]);
    }
    if (c->join[q]) (void)hipEventDestroy(c->join[q]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->d_vtab) (void)hipFree(c->d_vtab);
  if (c->d_ovl) (void)hipFree(c->d_ovl);
  c->woff.release();
  c->poff.release();
  c->zinit.release();
  c->zinit_off.release();
  c->lwoff.release();
  c->lkmax.release();
  c->lkern.release();
  c->plam.release();
  c->mfoff.release();
  c->lam.release();
  c->t0init.release();
  c->mf.release();
  c->kmax.release();
  c->grange.release();
  c->chains.release();
  c->wid.release();
  c->wflags.release();
  c->lane_d.release();
  c->draw_scr.release();
  c->ptab.release();
  c->lane_i.release();
  c->stage.release();
  (void)hipSetDevice(prev);
  delete c;
}

size_t fsmp_workspace_bytes(const fsmp_ctx *c, const fsmp_batch *b) {
  if (!c || !b || b->n_wave < 0 || (b->n_wave > 0 && !b->offsets)) return 0;
  const int64_t n = b->n_wave;
  const fsmp_config &cf = c->cfg;
  const bool fp32 = cf.precision == FSMP_FP32_REFRESH;
  const int sub = cf.grid_sub;
  int64_t cnt[kNumCaps] = {0};
  size_t grid = 0;
  int64_t tmax = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = b->offsets[i + 1] - b->offsets[i];
    const int64_t lo = b->g_range ? b->g_range[2 * i] : 0, hi = b->g_range ? b->g_range[2 * i + 1] : sub * L - 1;
    const int64_t T = hi >= lo ? hi - lo + 1 : 0;
    grid += (size_t)T;
    tmax = std::max(tmax, T);
    int kc = chain_kcap_for(b->kmax ? b->kmax[i] : cf.k_max);
    if (fp32 && kc == 48) kc = 64;
    for (int q = 0; q < kNumCaps; ++q)
      if (kCaps[q] == kc) cnt[q] += cf.n_chains;
  }
  // batch metadata, chain lists, matched filter over T
  size_t bytes = (size_t)(n + 1) * 16 + (size_t)n * (8 + 8 + 4 + 8 + 8 + 4 + 4) + (size_t)n * cf.n_chains * 4 + grid * 8;
  // chain state of each bucket in its design; charge-draw scratch; partial-sum table
  for (int q = 0; q < kNumCaps; ++q) {
    if (!cnt[q]) continue;
    const int dz = effective_design(c, kCaps[q], c->design[q]);
    if (dz == FSMP_DESIGN_LANE)
      bytes += lane_ws_doubles(kCaps[q], cnt[q]) * 8 + lane_ws_ints(kCaps[q], cnt[q]) * 4;
    else if (dz == FSMP_DESIGN_GROUP_DEVMEM || dz == FSMP_DESIGN_GROUP_DEVMEM_WIDE)
      bytes += group_dm_ws_doubles(kCaps[q], cnt[q], fp32, dz == FSMP_DESIGN_GROUP_DEVMEM_WIDE) * 8;
    if (cf.record_flags & FSMP_REC_CHARGE) bytes += (size_t)((cnt[q] + 63) / 64 * 64) * kCaps[q] * (kCaps[q] + 1) * 8;
  }
  bytes += (size_t)std::max<int64_t>(tmax + 1, 4 * 4096 + 1) * 16;
  if (b->z_init_offsets && n > 0)
    bytes += (size_t)(n * cf.n_chains + 1) * 8 + (size_t)b->z_init_offsets[n * cf.n_chains] * 4;
  return bytes;
}

fsmp_status fsmp_set_timing(fsmp_ctx *c, int32_t enable) {
  if (!c) return FSMP_EINVAL;
  c->timing = enable != 0;
  return FSMP_OK;
}

int32_t fsmp_last_timings(const fsmp_ctx *cc, fsmp_timing *out, int32_t cap) {
  if (!cc) return 0;
  fsmp_ctx *c = const_cast<fsmp_ctx *>(cc);
  for (size_t i = 0; i < c->timings.size() && i < c->timing_events.size(); ++i) {
    auto &pr = c->timing_events[i];
    if (!pr.first || !pr.second) continue;
    if (hipEventSynchronize(pr.second) != hipSuccess) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) c->timings[i].ms = ms;
  }
  const int32_t n = (int32_t)c->timings.size();
  for (int32_t i = 0; i < n && i < cap && out; ++i) out[i] = c->timings[i];
  return n;
}

}  // extern "C"

namespace {

// fsmp_sample, or with `force` set fsmp_replay: the chains follow the recorded proposals
// and the lane-group kernels with G^-1 in device memory write delta-nu / log-alpha
fsmp_status sample_impl(fsmp_ctx *c, const fsmp_batch *b, const fsmp_samples *o, void *hip_stream,
                        const fsmp_logrec *force, double *rdnu, double *rla, bool noalloc = false) {
  if (!c) return FSMP_EINVAL;
  if (!b || !o) return fail(c, FSMP_EINVAL, "null batch or output");
  const fsmp_config &cf = c->cfg;
  if (force && cf.precision != FSMP_FP64) return fail(c, FSMP_ENOTSUP, "replay runs the FP64 form only");
  if (force && cf.n_mix > 0) return fail(c, FSMP_ENOTSUP, "replay runs the single-normal charge law only");
  if (b && b->z_init_offsets && cf.n_mix > 0)
    return fail(c, FSMP_ENOTSUP, "start lists are not offered with the mixture charge law");
  const int64_t n = b->n_wave;
  if (n < 0) return fail(c, FSMP_EINVAL, "n_wave < 0");
  if (n > 0 && (!b->wave || !b->offsets || !b->lambda)) return fail(c, FSMP_EINVAL, "wave, offsets and lambda are required");
  if (n > 0 && (!o->n_pe || !o->t0 || !o->z || !o->charge || !o->acc || !o->nhist || !o->counts || !o->status))
    return fail(c, FSMP_EINVAL, "an output buffer is NULL");
  if ((cf.record_flags & FSMP_REC_LOG) && !o->log) return fail(c, FSMP_EINVAL, "FSMP_REC_LOG set but log is NULL");
  if ((cf.record_flags & FSMP_REC_TRACE) && !o->trace) return fail(c, FSMP_EINVAL, "FSMP_REC_TRACE set but trace is NULL");
  if (n > 0 && b->n_steps && !o->rec_steps)
    return fail(c, FSMP_EINVAL, "per-waveform n_steps needs fsmp_samples.rec_steps");
  if ((cf.record_flags & FSMP_REC_CHARGE) && (!o->qdraw || !o->zdraw))
    return fail(c, FSMP_EINVAL, "FSMP_REC_CHARGE set but qdraw or zdraw is NULL");
  if (n > 0 && b->offsets[0] != 0) return fail(c, FSMP_EINVAL, "offsets[0] must be 0");
  const int sub = cf.grid_sub;
  if (n * (int64_t)cf.n_chains > INT32_MAX) return fail(c, FSMP_EINVAL, "too many chains");
  // ---- per-waveform metadata: in vectors, or (the allocation-free variant) in the
  // file-scope host arrays of its largest batch
  std::vector<int32_t> v_kmx, v_gr, v_order;
  std::vector<double> v_t0i;
  std::vector<uint64_t> v_wid;
  std::vector<int64_t> v_mfo, v_ws;
  int32_t *kmx, *gr, *order;
  double *t0i;
  uint64_t *wid;
  int64_t *mfo, *wsorted;
  if (noalloc) {
    if (n > kNoAllocMaxWave || n * (int64_t)cf.n_chains > kNoAllocMaxChains)
      return fail(c, FSMP_EINVAL, "fsmp_sample_noalloc takes at most %lld waveforms and %lld chains (got %lld, %lld)",
                  (long long)kNoAllocMaxWave, (long long)kNoAllocMaxChains, (long long)n,
                  (long long)(n * cf.n_chains));
    kmx = g_na.kmx;
    gr = g_na.gr;
    order = g_na.order;
    t0i = g_na.t0i;
    wid = g_na.wid;
    mfo = g_na.mfo;
    wsorted = g_na.ws;
  } else {
    v_kmx.resize(n);
    v_gr.resize(2 * n);
    v_order.resize((size_t)n * cf.n_chains);
    v_t0i.resize(n);
    v_wid.resize(n);
    v_mfo.resize(n + 1);
    v_ws.resize(n);
    kmx = v_kmx.data();
    gr = v_gr.data();
    order = v_order.data();
    t0i = v_t0i.data();
    wid = v_wid.data();
    mfo = v_mfo.data();
    wsorted = v_ws.data();
  }
  mfo[0] = 0;
  int kmax_all = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = b->offsets[i + 1] - b->offsets[i];
    if (L < 1 || L > 65536) return fail(c, FSMP_EINVAL, "waveform %lld: window of %lld samples (need 1..65536)", (long long)i, (long long)L);
    const double lm = b->lambda[i];
    if (!std::isfinite(lm) || lm < 0) return fail(c, FSMP_EINVAL, "waveform %lld: lambda must be finite and >= 0", (long long)i);
    const int km = b->kmax ? b->kmax[i] : cf.k_max;
    if (km < 1 || km > 192) return fail(c, FSMP_EINVAL, "waveform %lld: kmax %d outside 1..192", (long long)i, km);
    if (km > o->kz) return fail(c, FSMP_EINVAL, "waveform %lld: kmax %d exceeds the output row length kz %d", (long long)i, km, o->kz);
    kmx[i] = km;
    kmax_all = std::max(kmax_all, km);
    if (b->n_steps && (b->n_steps[i] < 1 || b->n_steps[i] > cf.n_steps))
      return fail(c, FSMP_EINVAL, "waveform %lld: n_steps %d outside 1..%d", (long long)i, b->n_steps[i], cf.n_steps);
    int lo = 0, hi = (int)(sub * L - 1);
    if (b->g_range) {
      lo = b->g_range[2 * i];
      hi = b->g_range[2 * i + 1];
      if (lo <= hi && (lo < 0 || hi > sub * L - 1))
        return fail(c, FSMP_EINVAL, "waveform %lld: g_range [%d, %d] outside [0, %lld]", (long long)i, lo, hi, (long long)(sub * L - 1));
    }
    gr[2 * i] = lo;
    gr[2 * i + 1] = hi;
    const double t0 = b->t0_init ? b->t0_init[i] : 0.5 * (c->phi.t0_min + c->phi.t0_max);
    if (!(t0 >= c->phi.t0_min && t0 <= c->phi.t0_max)) return fail(c, FSMP_EINVAL, "waveform %lld: t0_init outside the prior", (long long)i);
    t0i[i] = t0;
    wid[i] = b->wave_id ? b->wave_id[i] : (uint64_t)i;
    mfo[i + 1] = mfo[i] + (lo <= hi ? (int64_t)(hi - lo + 1) : 0);
  }
  // initial PE lists: per chain at most kmax PEs, each inside T where phi(t - t0_init) > 0
  int64_t n_init = 0;
  if (b->z_init_offsets && n > 0) {
    const int64_t nc = n * cf.n_chains;
    if (b->z_init_offsets[0] != 0) return fail(c, FSMP_EINVAL, "z_init_offsets[0] must be 0");
    if (b->z_init_offsets[nc] > 0 && !b->z_init) return fail(c, FSMP_EINVAL, "z_init is NULL");
    for (int64_t ci = 0; ci < nc; ++ci) {
      const int64_t i = ci / cf.n_chains, o0 = b->z_init_offsets[ci], o1 = b->z_init_offsets[ci + 1];
      if (o1 < o0 || o1 - o0 > kmx[i])
        return fail(c, FSMP_EINVAL, "chain %lld: initial list of %lld PEs (need 0..kmax %d)", (long long)ci,
                    (long long)(o1 - o0), kmx[i]);
      if (o1 > o0 && !(b->lambda[i] > 0.0))
        return fail(c, FSMP_EINVAL, "chain %lld: an initial PE list needs lambda > 0", (long long)ci);
      for (int64_t k = o0; k < o1; ++k) {
        const int32_t g = b->z_init[k];
        const double x = g * (1.0 / sub) - t0i[i];
        const bool pos = c->phi.kind == FSMP_PHI_BIEXP ? x > 0.0 : x >= 0.0;
        if (g < gr[2 * i] || g > gr[2 * i + 1] || !pos)
          return fail(c, FSMP_EINVAL, "chain %lld: initial PE at grid point %d outside T or before t0", (long long)ci, g);
      }
    }
    n_init = b->z_init_offsets[nc];
  }
  // the occupancy counts of one grid point stay below n_chains * recorded sweeps * kmax
  if (o->occ && (int64_t)cf.n_chains * (cf.n_steps - cf.burn_in) * kmax_all > INT32_MAX)
    return fail(c, FSMP_EINVAL, "occupancy counts could exceed int32 (n_chains x recorded sweeps x kmax >= 2^31)");
  // ---- chains grouped by PE capacity
  const int *caps = kCaps;
  int64_t n_order = 0;
  int64_t bucket_start[kNumCaps + 1] = {0};
  const bool fp32 = cf.precision == FSMP_FP32_REFRESH;
  auto design_of = [&](int bi) {
    const int dz = effective_design(c, caps[bi], c->design[bi]);
    // a replay runs the device-memory groups: the wide ones where the context has chosen them
    // at capacity 64 and up, else the narrow ones
    if (force) return dz == FSMP_DESIGN_GROUP_DEVMEM_WIDE && caps[bi] >= 64 ? dz : FSMP_DESIGN_GROUP_DEVMEM;
    return dz;
  };
  // within a bucket, waveforms with per-waveform sweep counts in 16 bins of the batch's
  // largest count, the longest first, so that the chains of a workgroup end together and the
  // longest start first; within a bin in order of lambda (equal lambdas in batch order):
  // neighbouring lanes then carry chains of similar PE counts, which keeps the loops (bounded
  // by the largest K in a wavefront) short
  int64_t smax = 1;
  if (b->n_steps)
    for (int64_t i = 0; i < n; ++i) smax = std::max<int64_t>(smax, b->n_steps[i]);
  auto sbin = [&](int64_t i) { return b->n_steps ? (int64_t)b->n_steps[i] * 16 / (smax + 1) : 0; };
  for (int64_t i = 0; i < n; ++i) wsorted[i] = i;
  std::sort(wsorted, wsorted + n, [&](int64_t x, int64_t y) {
    if (sbin(x) != sbin(y)) return sbin(x) > sbin(y);
    return b->lambda[x] < b->lambda[y] || (b->lambda[x] == b->lambda[y] && x < y);
  });
  for (int bi = 0; bi < kNumCaps; ++bi) {
    bucket_start[bi] = n_order;
    for (int64_t ii = 0; ii < n; ++ii) {
      const int64_t i = wsorted[ii];
      int kc = chain_kcap_for(kmx[i]);
      if (fp32 && kc == 48) kc = 64;  // the precision form has no capacity-48 instance
      if (kc != caps[bi]) continue;
      for (int ch = 0; ch < cf.n_chains; ++ch) order[n_order++] = (int32_t)(i * cf.n_chains + ch);
    }
  }
  bucket_start[kNumCaps] = n_order;
  if (n_order != n * cf.n_chains)
    return fail(c, FSMP_ENOTSUP, "kmax above %d is not provided by this build", kCaps[kNumCaps - 1]);
  for (int bi = 0; bi < kNumCaps; ++bi)
    if (bucket_start[bi + 1] > bucket_start[bi] && !design_available(c, caps[bi], design_of(bi)))
      return fail(c, FSMP_ENOTSUP, "SER support %d too long for the design of PE capacity %d", c->tab.LV, caps[bi]);
  if (n == 0) {
    c->timings.clear();
    c->timing_events.clear();
    return FSMP_OK;
  }

  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  // ---- device workspace: the context's buffers (grown on demand), or in the allocation-free
  // variant pieces of this device's static scratch array
  if (noalloc && !c->scratch) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_EDEVICE, "the scratch array of fsmp_sample_noalloc has no address on device %d", c->device);
  }
  size_t sc_off = 0;
  bool sc_over = false;
  auto carve = [&](auto &buf, size_t count) {
    using T = typename std::remove_pointer<decltype(buf.p)>::type;
    if (noalloc) {
      const size_t at = (sc_off + 255) & ~(size_t)255;
      sc_off = at + std::max<size_t>(count, 1) * sizeof(T);
      if (sc_off > kScratchBytes) sc_over = true;
      return sc_over ? (T *)nullptr : (T *)(c->scratch + at);
    }
    if (e == hipSuccess) e = buf.ensure(count);
    return e == hipSuccess ? buf.p : (T *)nullptr;
  };
  int64_t *d_woff = carve(c->woff, n + 1);
  int64_t *d_mfoff = carve(c->mfoff, n + 1);
  double *d_lam = carve(c->lam, n);
  double *d_t0init = carve(c->t0init, n);
  int32_t *d_kmax = carve(c->kmax, n);
  int32_t *d_grange = carve(c->grange, 2 * n);
  uint64_t *d_wid = carve(c->wid, n);
  int32_t *d_wsteps = b->n_steps ? carve(c->wsteps, n) : nullptr;
  int64_t *d_zinit_off = b->z_init_offsets ? carve(c->zinit_off, n * cf.n_chains + 1) : nullptr;
  int32_t *d_zinit = n_init > 0 ? carve(c->zinit, n_init) : nullptr;
  uint32_t *d_wflags = carve(c->wflags, n);
  double *d_mf = carve(c->mf, (size_t)std::max<int64_t>(mfo[n], 1));
  int32_t *d_chains = carve(c->chains, n_order);
  size_t lane_doff[kNumCaps + 1] = {0}, lane_ioff[kNumCaps + 1] = {0};
  for (int bi = 0; bi < kNumCaps; ++bi) {
    const int64_t cnt = bucket_start[bi + 1] - bucket_start[bi];
    const int dz = design_of(bi);
    const size_t dd = dz == FSMP_DESIGN_LANE ? lane_ws_doubles(caps[bi], cnt)
                      : dz == FSMP_DESIGN_GROUP_DEVMEM ? group_dm_ws_doubles(caps[bi], cnt, fp32)
                      : dz == FSMP_DESIGN_GROUP_DEVMEM_WIDE ? group_dm_ws_doubles(caps[bi], cnt, fp32, true)
                                                       : 0;
    lane_doff[bi + 1] = lane_doff[bi] + dd;
    lane_ioff[bi + 1] = lane_ioff[bi] + (dz == FSMP_DESIGN_LANE ? lane_ws_ints(caps[bi], cnt) : 0);
  }
  double *d_lane = lane_doff[kNumCaps] > 0 ? carve(c->lane_d, lane_doff[kNumCaps]) : nullptr;
  int32_t *d_lanei = lane_ioff[kNumCaps] > 0 ? carve(c->lane_i, lane_ioff[kNumCaps]) : nullptr;
  size_t draw_off[kNumCaps + 1] = {0};
  double *d_draw = nullptr;
  if (cf.record_flags & FSMP_REC_CHARGE) {
    for (int bi = 0; bi < kNumCaps; ++bi) {
      const int64_t cnt = bucket_start[bi + 1] - bucket_start[bi];
      draw_off[bi + 1] = draw_off[bi] + (size_t)((cnt + 63) / 64 * 64) * caps[bi] * (caps[bi] + 1);
    }
    if (draw_off[kNumCaps] > 0) d_draw = carve(c->draw_scr, draw_off[kNumCaps]);
  }
  if (sc_over) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_EINVAL, "fsmp_sample_noalloc: the batch needs %zu bytes of scratch, the maximum is %zu", sc_off,
                kScratchBytes);
  }
  if (e == hipSuccess) {
    int64_t tmax = 0;
    for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, (int64_t)gr[2 * i + 1] - gr[2 * i] + 1);
    if (noalloc && !(c->md.ptab && c->md.ptab_n >= tmax + 1)) {
      (void)hipSetDevice(prev);
      return fail(c, FSMP_ENOTSUP,
                  "fsmp_sample_noalloc: a solution space of %lld grid points is longer than the context's light-curve "
                  "table (%lld); an fsmp_sample call with such a batch grows it",
                  (long long)tmax, (long long)c->md.ptab_n - 1);
    }
    if (!noalloc) e = ensure_ptab(c, tmax + 1);
  }
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_ENOMEM, "workspace allocation failed: %s", hipGetErrorString(e));
  }
  // ---- metadata upload: through the context's pinned stage (after its previous upload), or
  // in the allocation-free variant straight from host memory (pageable: the copy has read it
  // when hipMemcpyAsync returns)
  auto pad16 = [](size_t nb) { return (nb + 15) & ~(size_t)15; };
  char *sp = nullptr;
  if (!noalloc) {
    if (c->stage_pending) (void)hipEventSynchronize(c->stage_done);
    const size_t bytes = pad16(sizeof(int64_t) * (n + 1)) * 2 + pad16(sizeof(double) * n) * 2 +
                         pad16(sizeof(int32_t) * n) + pad16(sizeof(int32_t) * 2 * n) + pad16(sizeof(uint64_t) * n) +
                         pad16(sizeof(int32_t) * n_order) + pad16(sizeof(int32_t) * n) +
                         (b->z_init_offsets ? pad16(sizeof(int64_t) * (n * cf.n_chains + 1)) + pad16(sizeof(int32_t) * n_init)
                                            : 0);
    e = c->stage.ensure(bytes);
    if (e != hipSuccess) {
      (void)hipSetDevice(prev);
      return fail(c, FSMP_ENOMEM, "pinned staging allocation failed: %s", hipGetErrorString(e));
    }
    sp = (char *)c->stage.p;
  }
  auto put = [&](void *dst, const void *src, size_t nb) -> hipError_t {
    if (noalloc) return hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, st);
    std::memcpy(sp, src, nb);
    hipError_t r = hipMemcpyAsync(dst, sp, nb, hipMemcpyHostToDevice, st);
    sp += pad16(nb);
    return r;
  };
  if (e == hipSuccess) e = put(d_woff, b->offsets, sizeof(int64_t) * (n + 1));
  if (e == hipSuccess) e = put(d_mfoff, mfo, sizeof(int64_t) * (n + 1));
  if (e == hipSuccess) e = put(d_lam, b->lambda, sizeof(double) * n);
  if (e == hipSuccess) e = put(d_t0init, t0i, sizeof(double) * n);
  if (e == hipSuccess) e = put(d_kmax, kmx, sizeof(int32_t) * n);
  if (e == hipSuccess) e = put(d_grange, gr, sizeof(int32_t) * 2 * n);
  if (e == hipSuccess) e = put(d_wid, wid, sizeof(uint64_t) * n);
  if (e == hipSuccess) e = put(d_chains, order, sizeof(int32_t) * n_order);
  if (e == hipSuccess && b->n_steps) e = put(d_wsteps, b->n_steps, sizeof(int32_t) * n);
  if (e == hipSuccess && b->z_init_offsets && n > 0) {
    e = put(d_zinit_off, b->z_init_offsets, sizeof(int64_t) * (n * cf.n_chains + 1));
    if (e == hipSuccess && n_init > 0) e = put(d_zinit, b->z_init, sizeof(int32_t) * n_init);
  }
  if (!noalloc) {
    if (e == hipSuccess) e = hipEventRecord(c->stage_done, st);
    c->stage_pending = (e == hipSuccess);
  }
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_EDEVICE, "metadata upload failed: %s", hipGetErrorString(e));
  }

  c->timings.clear();
  c->timing_events.clear();
  size_t ev = 0;
  const hipStream_t upload_stream = st;
  if (c->capture) {
    // graph capture: the metadata upload above is complete before the kernels are recorded
    e = hipStreamSynchronize(upload_stream);
    if (e == hipSuccess) e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipSetDevice(prev);
      return fail(c, FSMP_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    st = c->capture;
  }
  auto timed = [&](const char *name, int kcap, hipStream_t ks, auto &&launch) -> hipError_t {
    fsmp_timing t{};
    if (noalloc) return launch(t);  // the allocation-free variant records no timings
    std::snprintf(t.name, sizeof t.name, "%s", name);
    t.kcap = kcap;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && !c->capture) {
      e0 = pool_event(c, ev++);
      e1 = pool_event(c, ev++);
      if (e0) (void)hipEventRecord(e0, ks);
    }
    hipError_t r = launch(t);
    if (e1) (void)hipEventRecord(e1, ks);
    c->timings.push_back(t);
    c->timing_events.push_back({e0, e1});
    return r;
  };

  // ---- prologue: matched filter over T, non-finite scan
  PrologueArgs pa{};
  pa.md = c->md;
  pa.vtab = c->d_vtab;
  pa.wave = b->wave;
  pa.woff = d_woff;
  pa.grange = d_grange;
  pa.mfoff = d_mfoff;
  pa.mf = d_mf;
  pa.wflags = d_wflags;
  pa.occ = o->occ;
  pa.n_wave = n;
  e = timed("prologue", 0, st, [&](fsmp_timing &t) {
    t.chains = 0;
    t.blocks = std::min<int64_t>(n, 65535 * 8);
    t.lanes = 0;
    return launch_prologue(pa, st);
  });
  // ---- chains
  ChainArgs ca{};
  ca.md = c->md;
  ca.vtab = c->d_vtab;
  ca.ovl = c->d_ovl;
  ca.woff = d_woff;
  ca.lam = d_lam;
  ca.kmax = d_kmax;
  ca.grange = d_grange;
  ca.t0init = d_t0init;
  ca.wid = d_wid;
  ca.mf = d_mf;
  ca.mfoff = d_mfoff;
  ca.n_chains = cf.n_chains;
  ca.n_steps = cf.n_steps;
  ca.burn_in = cf.burn_in;
  ca.thin = cf.thin;
  const int S = cf.n_steps - cf.burn_in;
  ca.wsteps = d_wsteps;
  ca.rec_steps = o->rec_steps;
  ca.n_rec = (cf.thin > 0 && S > 0) ? (S + cf.thin - 1) / cf.thin : 0;
  ca.key0 = (uint32_t)cf.seed;
  ca.key1 = (uint32_t)(cf.seed >> 32);
  ca.n_pe = o->n_pe;
  ca.t0 = o->t0;
  ca.z = o->z;
  ca.charge = o->charge;
  ca.acc = o->acc;
  ca.nhist = o->nhist;
  ca.counts = o->counts;
  ca.status = o->status;
  ca.log = (cf.record_flags & FSMP_REC_LOG) ? o->log : nullptr;
  ca.trace = (cf.record_flags & FSMP_REC_TRACE) ? o->trace : nullptr;
  ca.qdraw = (cf.record_flags & FSMP_REC_CHARGE) ? o->qdraw : nullptr;
  ca.zdraw = (cf.record_flags & FSMP_REC_CHARGE) ? o->zdraw : nullptr;
  ca.sigma_eps = cf.sigma_eps;
  ca.force = force;
  ca.rdnu = rdnu;
  ca.rla = rla;
  ca.kz = o->kz;
  ca.wflags = d_wflags;
  ca.work = o->work;
  ca.occ = o->occ;
  ca.comp = o->comp;
  ca.zinit = (b->z_init_offsets && n > 0) ? d_zinit : nullptr;
  ca.zinit_off = (b->z_init_offsets && n > 0) ? d_zinit_off : nullptr;
  ca.refresh_M = cf.refresh_M;
  ca.drift_bound = 1e-3;
  int n_buckets = 0;
  for (int bi = 0; bi < kNumCaps; ++bi) n_buckets += bucket_start[bi + 1] > bucket_start[bi];
  // the allocation-free variant runs the buckets one after the other on the caller's stream
  const bool fan = n_buckets > 1 && !noalloc && !c->serial;
  // Lanes of concurrent work: the caller's stream and up to GPU_MAX_HW_QUEUES - 1 side
  // streams (the process has that many hardware queues, HIP's default 4; the caller's stream
  // holds one, and streams beyond them would share a queue and run one after the other). The
  // buckets go to the lanes largest estimated cost first, each to the least loaded lane; a
  // lane runs its buckets in capacity order. A bucket's cost is the autotuner's trial time of
  // its design when the context has one for every bucket of the call, else its chains' sweeps
  // times a per-capacity weight (the measured time of one sweep of one chain relative to
  // capacity 16).
  int lane_of[kNumCaps] = {};
  int n_lanes = 1;
  if (fan) {
    int n_queues = 4;
    if (const char *q = std::getenv("GPU_MAX_HW_QUEUES")) {
      const int v = std::atoi(q);
      if (v > 0) n_queues = v;
    }
    n_lanes = std::min(std::min(n_queues, n_buckets), kNumCaps);
    static const double kWeight[kNumCaps] = {1.0, 3.8, 5.4, 8.8, 16.0, 25.0, 35.0, 45.0};
    double cost[kNumCaps] = {};
    bool tuned = true;
    for (int bi = 0; bi < kNumCaps; ++bi)
      if (bucket_start[bi + 1] > bucket_start[bi] &&
          !(c->tuned_ms[bi] > 0.0 && c->tuned_design[bi] == design_of(bi)))
        tuned = false;
    for (int bi = 0; bi < kNumCaps; ++bi) {
      if (tuned) {
        cost[bi] = bucket_start[bi + 1] > bucket_start[bi] ? c->tuned_ms[bi] : 0.0;
        continue;
      }
      double sweeps = 0.0;
      for (int64_t k = bucket_start[bi]; k < bucket_start[bi + 1]; ++k)
        sweeps += b->n_steps ? (double)b->n_steps[order[k] / cf.n_chains] : (double)cf.n_steps;
      cost[bi] = sweeps * kWeight[bi];
    }
    double load[kNumCaps] = {};
    bool done[kNumCaps] = {};
    for (int r = 0; r < n_buckets; ++r) {
      int best = -1;
      for (int bi = 0; bi < kNumCaps; ++bi)
        if (!done[bi] && bucket_start[bi + 1] > bucket_start[bi] && (best < 0 || cost[bi] > cost[best])) best = bi;
      int ln = 0;
      for (int k = 1; k < n_lanes; ++k)
        if (load[k] < load[ln]) ln = k;
      lane_of[best] = ln;
      load[ln] += cost[best];
      done[best] = true;
    }
  }
  const bool fork_join = fan && n_lanes > 1;
  if (fork_join && e == hipSuccess) {
    if (!c->fork) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(c->fork, st);
  }
  for (int bi = 0; bi < kNumCaps && e == hipSuccess; ++bi) {
    const int64_t cnt = bucket_start[bi + 1] - bucket_start[bi];
    if (cnt == 0) continue;
    hipStream_t ks = st;
    // lane 0 is the caller's stream, lane k > 0 side stream k - 1
    const bool side = fork_join && lane_of[bi] > 0;
    if (side) {
      const int sq = lane_of[bi] - 1;
      if (!c->side[sq]) e = hipStreamCreateWithFlags(&c->side[sq], hipStreamNonBlocking);
      if (e == hipSuccess && !c->join[bi]) e = hipEventCreateWithFlags(&c->join[bi], hipEventDisableTiming);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->side[sq], c->fork, 0);
      if (e != hipSuccess) break;
      ks = c->side[sq];
    }
    ca.chains = d_chains + bucket_start[bi];
    ca.n_list = cnt;
    char name[32];
    const int dz = design_of(bi);
    std::snprintf(name, sizeof name, "%s%s_k%d",
                  dz == FSMP_DESIGN_LANE ? "chain_lane" : dz == FSMP_DESIGN_GROUP ? "chain_group" : "chain_group_dm",
                  fp32 ? "_fp32" : "", caps[bi]);
    ca.dws = dz != FSMP_DESIGN_GROUP ? d_lane + lane_doff[bi] : nullptr;
    ca.iws = dz == FSMP_DESIGN_LANE ? d_lanei + lane_ioff[bi] : nullptr;
    ca.dscr = ca.qdraw ? d_draw + draw_off[bi] : nullptr;
    e = timed(name, caps[bi], ks, [&](fsmp_timing &t) {
      t.chains = cnt;
      return dz == FSMP_DESIGN_LANE    ? launch_chain_lane(caps[bi], ca, ks, &t.lanes, &t.blocks)
             : dz == FSMP_DESIGN_GROUP ? launch_chain(caps[bi], ca, ks, &t.lanes, &t.blocks)
                                       : launch_chain_dm(caps[bi], fp32, dz == FSMP_DESIGN_GROUP_DEVMEM_WIDE, ca, ks,
                                                         &t.lanes, &t.blocks);
    });
    if (side) {
      const hipError_t e2 = hipEventRecord(c->join[bi], ks);
      if (e == hipSuccess) e = e2;
    }
  }
  // the caller's stream waits for the side lanes after its own buckets are enqueued
  if (fork_join)
    for (int bi = 0; bi < kNumCaps && e == hipSuccess; ++bi)
      if (bucket_start[bi + 1] > bucket_start[bi] && lane_of[bi] > 0) e = hipStreamWaitEvent(st, c->join[bi], 0);
  if (c->capture) {
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->capture, &g);
    if (e == hipSuccess) e = e2;
    c->captured = g;
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return fail(c, FSMP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return FSMP_OK;
}

}  // namespace

extern "C" {

fsmp_status fsmp_sample(fsmp_ctx *c, const fsmp_batch *b, const fsmp_samples *o, void *hip_stream) {
  return sample_impl(c, b, o, hip_stream, nullptr, nullptr, nullptr);
}

fsmp_status fsmp_sample_noalloc(fsmp_ctx *c, const fsmp_batch *b, const fsmp_samples *o, void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  std::lock_guard<std::mutex> lk(g_na_mutex);
  return sample_impl(c, b, o, hip_stream, nullptr, nullptr, nullptr, true);
}

fsmp_status fsmp_replay(fsmp_ctx *c, const fsmp_batch *b, const fsmp_logrec *log, double *dnu, double *log_alpha,
                        const fsmp_samples *o, void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  if (!log || !dnu || !log_alpha) return fail(c, FSMP_EINVAL, "replay needs the log and both outputs");
  return sample_impl(c, b, o, hip_stream, log, dnu, log_alpha);
}

fsmp_status fsmp_set_design(fsmp_ctx *c, int32_t capacity, int32_t design) {
  if (!c) return FSMP_EINVAL;
  if (design != FSMP_DESIGN_GROUP && design != FSMP_DESIGN_LANE && design != FSMP_DESIGN_GROUP_DEVMEM &&
      design != FSMP_DESIGN_GROUP_DEVMEM_WIDE)
    return fail(c, FSMP_EINVAL, "unknown design %d", design);
  bool any = false;
  for (int q = 0; q < kNumCaps; ++q) {
    if (capacity != 0 && capacity != kCaps[q]) continue;
    any = true;
    if (!design_available(c, kCaps[q], design)) {
      if (capacity != 0) return fail(c, FSMP_ENOTSUP, "design %d does not exist for capacity %d", design, kCaps[q]);
      continue;
    }
    c->design[q] = design;
  }
  if (!any) return fail(c, FSMP_EINVAL, "capacity %d is not one of the kernel capacities", capacity);
  return FSMP_OK;
}

int32_t fsmp_get_design(const fsmp_ctx *c, int32_t capacity) {
  if (!c) return FSMP_EINVAL;
  for (int q = 0; q < kNumCaps; ++q)
    if (kCaps[q] == capacity) return c->design[q];
  return FSMP_EINVAL;
}

fsmp_status fsmp_autotune(fsmp_ctx *c, const fsmp_batch *b, int32_t trial_steps, void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  if (!b || b->n_wave < 1) return fail(c, FSMP_EINVAL, "autotune needs a non-empty batch");
  if (trial_steps < 1) return fail(c, FSMP_EINVAL, "trial_steps must be >= 1");
  const int64_t n = b->n_wave;
  int kz = 1;
  for (int64_t i = 0; i < n; ++i) kz = std::max(kz, b->kmax ? b->kmax[i] : c->cfg.k_max);
  const int64_t C = n * c->cfg.n_chains;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  // scratch outputs for the trials
  DevBuf<int32_t> i1, i2, i3, i4, i5, i6;
  DevBuf<double> d1, d2, d3;
  hipError_t e = i1.ensure(C);
  if (e == hipSuccess && b->n_steps) e = i6.ensure(C);
  if (e == hipSuccess) e = i2.ensure((size_t)C * kz);
  if (e == hipSuccess) e = i3.ensure((size_t)C * (kz + 1));
  if (e == hipSuccess) e = i4.ensure((size_t)C * 8);
  if (e == hipSuccess) e = i5.ensure(C);
  if (e == hipSuccess) e = d1.ensure(C);
  if (e == hipSuccess) e = d2.ensure((size_t)C * kz);
  if (e == hipSuccess) e = d3.ensure((size_t)C * 12);
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  }
  fsmp_samples o{};
  o.n_pe = i1.p;
  o.z = i2.p;
  o.nhist = i3.p;
  o.counts = i4.p;
  o.status = (uint32_t *)i5.p;
  o.t0 = d1.p;
  o.charge = d2.p;
  o.acc = d3.p;
  o.rec_steps = b->n_steps ? i6.p : nullptr;
  o.kz = kz;
  // with per-waveform sweep counts the trial keeps their proportions, scaled to a mean of
  // trial_steps, so that it sees what sets a launch's duration in the full run: its longest
  // chains against its total work
  fsmp_batch bt = *b;
  std::vector<int32_t> tsteps;
  int32_t tmax = trial_steps;
  if (b->n_steps) {
    double mean = 0.0;
    for (int64_t i = 0; i < n; ++i) mean += b->n_steps[i];
    mean /= (double)n;
    tsteps.resize(n);
    tmax = 1;
    for (int64_t i = 0; i < n; ++i) {
      tsteps[i] = (int32_t)std::max<double>(1.0, std::llround(b->n_steps[i] * (double)trial_steps / mean));
      tmax = std::max(tmax, tsteps[i]);
    }
    bt.n_steps = tsteps.data();
  }
  const fsmp_config saved = c->cfg;
  const bool saved_timing = c->timing;
  // the trials run the buckets one after the other, so that each launch's time is its own
  // (side by side, each would also carry what the others take from it)
  c->serial = true;
  int saved_design[kNumCaps];
  std::memcpy(saved_design, c->design, sizeof saved_design);
  c->cfg.n_steps = tmax;
  c->cfg.burn_in = 0;
  c->cfg.record_flags = 0;
  c->timing = true;
  constexpr int kDesigns = 4;
  double ms[kDesigns][kNumCaps];
  fsmp_status st = FSMP_OK;
  for (int d = 0; d < kDesigns && st == FSMP_OK; ++d) {
    for (int q = 0; q < kNumCaps; ++q) {
      ms[d][q] = -1.0;
      c->design[q] = design_available(c, kCaps[q], d) ? d : saved_design[q];
    }
    st = fsmp_sample(c, &bt, &o, hip_stream);
    if (st != FSMP_OK) break;
    std::vector<fsmp_timing> tv(c->timings.size() + 1);
    const int32_t nt = fsmp_last_timings(c, tv.data(), (int32_t)tv.size());
    for (int32_t k = 0; k < nt; ++k)
      for (int q = 0; q < kNumCaps; ++q)
        if (tv[k].kcap == kCaps[q] && c->design[q] == d) ms[d][q] = tv[k].ms;
  }
  c->cfg = saved;
  c->timing = saved_timing;
  c->serial = false;
  std::memcpy(c->design, saved_design, sizeof saved_design);
  // per capacity the fastest of the designs that ran it
  if (st == FSMP_OK)
    for (int q = 0; q < kNumCaps; ++q) {
      int best = -1;
      for (int d = 0; d < kDesigns; ++d)
        if (ms[d][q] >= 0.0 && (best < 0 || ms[d][q] < ms[best][q])) best = d;
      if (best >= 0) c->design[q] = best;
      c->tuned_design[q] = best;
      c->tuned_ms[q] = best >= 0 ? ms[best][q] : -1.0;
    }
  (void)hipStreamSynchronize((hipStream_t)hip_stream);
  i1.release();
  i2.release();
  i3.release();
  i4.release();
  i5.release();
  i6.release();
  d1.release();
  d2.release();
  d3.release();
  (void)hipSetDevice(prev);
  return st;
}

// The graph owns a private context: its kernels read that context's workspace
// (uploaded batch metadata, chain lists, lane-design state), which later calls on the
// caller's context may overwrite or reallocate without touching the graph.
fsmp_status fsmp_autotune_steps(fsmp_ctx *c, const fsmp_batch *b, int32_t pilot_steps, double target_rel_mcse,
                                int32_t min_steps, int32_t max_steps, int32_t *steps_out, void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  if (!b || b->n_wave < 1 || !steps_out) return fail(c, FSMP_EINVAL, "steps autotuner needs a batch and steps_out");
  if (pilot_steps < 4) return fail(c, FSMP_EINVAL, "pilot_steps must be >= 4");
  if (!(target_rel_mcse > 0.0)) return fail(c, FSMP_EINVAL, "target_rel_mcse must be > 0");
  if (min_steps < 1 || max_steps < min_steps) return fail(c, FSMP_EINVAL, "need 1 <= min_steps <= max_steps");
  const int64_t n = b->n_wave;
  int kz = 1;
  for (int64_t i = 0; i < n; ++i) kz = std::max(kz, b->kmax ? b->kmax[i] : c->cfg.k_max);
  const int64_t C = n * c->cfg.n_chains;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  DevBuf<int32_t> i1, i2, i3, i4, i5, i6;
  DevBuf<double> d1, d2, d3, pm, pv, pe, pa;
  DevBuf<uint32_t> ps;
  hipError_t e = i1.ensure(C);
  if (e == hipSuccess) e = i2.ensure((size_t)C * kz);
  if (e == hipSuccess) e = i3.ensure((size_t)C * (kz + 1));
  if (e == hipSuccess) e = i4.ensure((size_t)C * 8);
  if (e == hipSuccess) e = i5.ensure(C);
  if (e == hipSuccess) e = i6.ensure(C);
  if (e == hipSuccess) e = d1.ensure(C);
  if (e == hipSuccess) e = d2.ensure((size_t)C * kz);
  if (e == hipSuccess) e = d3.ensure((size_t)C * 12);
  if (e == hipSuccess) e = pm.ensure(3 * n);
  if (e == hipSuccess) e = pv.ensure(3 * n);
  if (e == hipSuccess) e = pe.ensure(3 * n);
  if (e == hipSuccess) e = pa.ensure(4 * n);
  if (e == hipSuccess) e = ps.ensure(n);
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_ENOMEM, "steps autotuner scratch: %s", hipGetErrorString(e));
  }
  fsmp_samples o{};
  o.n_pe = i1.p;
  o.z = i2.p;
  o.nhist = i3.p;
  o.counts = i4.p;
  o.status = (uint32_t *)i5.p;
  o.rec_steps = i6.p;
  o.t0 = d1.p;
  o.charge = d2.p;
  o.acc = d3.p;
  o.kz = kz;
  fsmp_posterior_out po{};
  po.mean = pm.p;
  po.var = pv.p;
  po.mcse = pe.p;
  po.accept = pa.p;
  po.status = ps.p;
  // the pilot: pilot_steps sweeps with the configured burn-in fraction, no records
  const fsmp_config saved = c->cfg;
  const bool saved_timing = c->timing;
  const int burn_pilot = (int)((int64_t)pilot_steps * saved.burn_in / saved.n_steps);
  c->cfg.n_steps = pilot_steps;
  c->cfg.burn_in = burn_pilot;
  c->cfg.record_flags = 0;
  c->timing = false;
  fsmp_batch bp = *b;
  bp.n_steps = nullptr;
  fsmp_status st = fsmp_sample(c, &bp, &o, hip_stream);
  if (st == FSMP_OK) st = fsmp_posterior(c, n, &o, &po, hip_stream);
  c->cfg = saved;
  c->timing = saved_timing;
  std::vector<double> mean(3 * n), mcse(3 * n);
  if (st == FSMP_OK) {
    e = hipMemcpyAsync(mean.data(), pm.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, (hipStream_t)hip_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(mcse.data(), pe.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, (hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) st = fail(c, FSMP_EDEVICE, "steps autotuner read-back: %s", hipGetErrorString(e));
  }
  if (st == FSMP_OK) {
    // MCSE ~ 1 / sqrt(recorded sweeps): the recorded sweeps that reach the target, then the
    // sweeps that leave that many after the configured burn-in fraction
    const double kept_pilot = (double)(pilot_steps - burn_pilot);
    const double keep_frac = (double)(saved.n_steps - saved.burn_in) / saved.n_steps;
    const int32_t hi = std::min(max_steps, saved.n_steps);
    for (int64_t i = 0; i < n; ++i) {
      const double target = target_rel_mcse * std::max(1.0, mean[3 * i]);
      const double m = mcse[3 * i];
      double want = (m > 0.0 && kept_pilot > 0.0) ? kept_pilot * (m / target) * (m / target) / keep_frac : 0.0;
      if (!std::isfinite(want)) want = (double)hi;
      int64_t w = (int64_t)std::ceil(want);
      w = std::max<int64_t>(w, min_steps);
      w = std::min<int64_t>(w, hi);
      steps_out[i] = (int32_t)std::max<int64_t>(w, 1);
    }
  }
  (void)hipSetDevice(prev);
  return st;
}

struct fsmp_graph {
  fsmp_ctx *ctx = nullptr;
  fsmp_ctx *own = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
};

fsmp_status fsmp_graph_create(fsmp_ctx *c, const fsmp_batch *b, const fsmp_samples *o, void *hip_stream,
                              fsmp_graph **out) {
  if (!c) return FSMP_EINVAL;
  if (!out) return fail(c, FSMP_EINVAL, "graph output pointer is NULL");
  *out = nullptr;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  auto *g = new fsmp_graph();
  g->ctx = c;
  fsmp_status st = fsmp_create(&g->own, &c->ser, &c->phi, &c->cfg, c->device);
  if (st != FSMP_OK) {
    delete g;
    (void)hipSetDevice(prev);
    return fail(c, st, "graph context: %s", fsmp_last_error(nullptr));
  }
  std::memcpy(g->own->design, c->design, sizeof c->design);
  hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    fsmp_graph_destroy(g);
    (void)hipSetDevice(prev);
    return fail(c, FSMP_EDEVICE, "graph stream: %s", hipGetErrorString(e));
  }
  fsmp_ctx *k = g->own;
  k->capture = g->stream;
  k->captured = nullptr;
  st = fsmp_sample(k, b, o, hip_stream);
  k->capture = nullptr;
  g->graph = k->captured;
  k->captured = nullptr;
  if (st != FSMP_OK) st = fail(c, st, "%s", k->err.c_str());
  if (st == FSMP_OK && g->graph) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = fail(c, FSMP_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  } else if (st == FSMP_OK) {
    st = fail(c, FSMP_EDEVICE, "graph capture produced no graph");
  }
  if (st != FSMP_OK) {
    fsmp_graph_destroy(g);
    (void)hipSetDevice(prev);
    return st;
  }
  (void)hipSetDevice(prev);
  *out = g;
  return FSMP_OK;
}

fsmp_status fsmp_graph_launch(fsmp_graph *g, void *hip_stream) {
  if (!g || !g->exec) return FSMP_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(g->ctx->device);
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return fail(g->ctx, FSMP_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  return FSMP_OK;
}

void fsmp_graph_destroy(fsmp_graph *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  if (g->own) fsmp_destroy(g->own);
  delete g;
}

int32_t fsmp_ser_support(const fsmp_ctx *c) { return c ? c->tab.LV : -1; }

fsmp_status fsmp_lucy(fsmp_ctx *c, const fsmp_batch *b, int32_t n_iter, double threshold, int32_t margin,
                      fsmp_lucy_out *out, void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  if (!b || !out) return fail(c, FSMP_EINVAL, "null batch or output");
  const int64_t n = b->n_wave;
  if (n < 0) return fail(c, FSMP_EINVAL, "n_wave < 0");
  if (n == 0) return FSMP_OK;
  if (!b->wave || !b->offsets) return fail(c, FSMP_EINVAL, "wave and offsets are required");
  if (!out->z || !out->n_pe || !out->g_range || !out->t0 || !out->lambda || !out->cut)
    return fail(c, FSMP_EINVAL, "an output buffer is NULL");
  if (n_iter < 0 || !(threshold >= 0.0) || !std::isfinite(threshold) || margin < 0)
    return fail(c, FSMP_EINVAL, "need n_iter >= 0, a finite threshold >= 0 and margin >= 0");
  if (b->offsets[0] != 0) return fail(c, FSMP_EINVAL, "offsets[0] must be 0");
  const int LV = c->tab.LV, sub = c->cfg.grid_sub;
  const int LVp = (LV + 23) / 24 * 24;  // a multiple of both window widths of the kernel
  std::vector<int32_t> kmx(n);
  int64_t max_len = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = b->offsets[i + 1] - b->offsets[i];
    if (L < 1 || L > 65536) return fail(c, FSMP_EINVAL, "waveform %lld: window of %lld samples (need 1..65536)", (long long)i, (long long)L);
    kmx[i] = b->kmax ? b->kmax[i] : c->cfg.k_max;
    if (kmx[i] < 1 || kmx[i] > 192 || kmx[i] > out->kz)
      return fail(c, FSMP_EINVAL, "waveform %lld: kmax %d outside 1..192 or above kz %d", (long long)i, kmx[i], out->kz);
    max_len = std::max(max_len, L);
  }
  if (lucy_lds_bytes(max_len, LVp) + 1024 > 160 * 1024)
    return fail(c, FSMP_ENOTSUP, "a window of %lld samples does not fit the deconvolution's LDS", (long long)max_len);
  // the SER at whole samples, normalised to unit sum
  std::vector<double> kern(2 * (size_t)LVp, 0.0);  // K, then K reversed
  double area = 0.0;
  for (int s0 = 0; s0 < LV; ++s0) area += c->tab.vtab[(size_t)s0 * sub];
  if (!(area > 0.0)) return fail(c, FSMP_EINVAL, "the SER has no area at whole samples");
  for (int s0 = 0; s0 < LV; ++s0) kern[s0] = c->tab.vtab[(size_t)s0 * sub] / area;
  for (int s0 = 0; s0 < LV; ++s0) kern[LVp + s0] = kern[LV - 1 - s0];
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  const hipStream_t st = (hipStream_t)hip_stream;
  if (c->stage_pending) (void)hipEventSynchronize(c->stage_done);
  auto pad16 = [](size_t nb) { return (nb + 15) & ~(size_t)15; };
  const size_t nbo = sizeof(int64_t) * (n + 1), nbk = sizeof(int32_t) * n, nbv = sizeof(double) * 2 * LVp;
  hipError_t e = c->lwoff.ensure(n + 1);
  if (e == hipSuccess) e = c->lkmax.ensure(n);
  if (e == hipSuccess) e = c->lkern.ensure(2 * (size_t)LVp);
  if (e == hipSuccess) e = c->stage.ensure(pad16(nbo) + pad16(nbk) + pad16(nbv));
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(c, FSMP_ENOMEM, "deconvolution workspace allocation failed: %s", hipGetErrorString(e));
  }
  char *sp = (char *)c->stage.p;
  std::memcpy(sp, b->offsets, nbo);
  std::memcpy(sp + pad16(nbo), kmx.data(), nbk);
  std::memcpy(sp + pad16(nbo) + pad16(nbk), kern.data(), nbv);
  e = hipMemcpyAsync(c->lwoff.p, sp, nbo, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->lkmax.p, sp + pad16(nbo), nbk, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->lkern.p, sp + pad16(nbo) + pad16(nbk), nbv, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(c->stage_done, st);
  c->stage_pending = (e == hipSuccess);
  LucyArgs a{};
  a.wave = b->wave;
  a.woff = c->lwoff.p;
  a.kmax = c->lkmax.p;
  a.kern = c->lkern.p;
  a.kern_rev = c->lkern.p + LVp;
  a.LV = LV;
  a.LVp = LVp;
  a.sub = sub;
  a.n_iter = n_iter;
  a.kz = out->kz;
  a.n_wave = n;
  a.inv_area = 1.0 / area;
  a.threshold = threshold;
  a.margin = margin;
  a.t0_min = c->phi.t0_min;
  a.t0_max = c->phi.t0_max;
  a.z = out->z;
  a.n_pe = out->n_pe;
  a.g_range = out->g_range;
  a.t0 = out->t0;
  a.lam = out->lambda;
  a.cut = out->cut;
  a.qhat = out->qhat;
  if (e == hipSuccess) e = launch_lucy(a, max_len, st);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return fail(c, FSMP_EDEVICE, "deconvolution failed: %s", hipGetErrorString(e));
  return FSMP_OK;
}

fsmp_status fsmp_posterior(fsmp_ctx *c, int64_t n_wave, const fsmp_samples *in, fsmp_posterior_out *out,
                           void *hip_stream) {
  if (!c) return FSMP_EINVAL;
  if (!in || !out) return fail(c, FSMP_EINVAL, "null samples or posterior output");
  if (n_wave < 0) return fail(c, FSMP_EINVAL, "n_wave < 0");
  if (n_wave == 0) return FSMP_OK;
  if (!in->acc || !in->nhist || !in->counts || !in->status) return fail(c, FSMP_EINVAL, "sample accumulators are NULL");
  if (!out->mean || !out->var || !out->mcse || !out->accept || !out->status)
    return fail(c, FSMP_EINVAL, "a posterior output buffer is NULL");
  PosteriorArgs a{};
  a.acc = in->acc;
  a.nhist = in->nhist;
  a.counts = in->counts;
  a.cstatus = in->status;
  a.n_wave = n_wave;
  a.n_chains = c->cfg.n_chains;
  a.kz = in->kz;
  a.n_steps = c->cfg.n_steps;
  a.burn_in = c->cfg.burn_in;
  a.rec_steps = in->rec_steps;
  a.mean = out->mean;
  a.var = out->var;
  a.mcse = out->mcse;
  a.p_n = out->p_n;
  a.accept = out->accept;
  a.status = out->status;
  if (out->occupancy) {
    if (!in->occ || !out->offsets) return fail(c, FSMP_EINVAL, "occupancy needs fsmp_samples.occ and the batch offsets");
    if (out->offsets[0] != 0) return fail(c, FSMP_EINVAL, "offsets[0] must be 0");
    for (int64_t i = 0; i < n_wave; ++i)
      if (out->offsets[i + 1] < out->offsets[i]) return fail(c, FSMP_EINVAL, "offsets must be non-decreasing");
  }
  if (out->lambda_hat) {
    if (!out->lambda) return fail(c, FSMP_EINVAL, "lambda_hat needs the batch's lambda0");
    for (int64_t i = 0; i < n_wave; ++i)
      if (!(out->lambda[i] >= 0.0) || !std::isfinite(out->lambda[i]))
        return fail(c, FSMP_EINVAL, "waveform %lld: lambda0 must be finite and >= 0", (long long)i);
  }
  a.rhat = out->rhat;
  a.mcse_chains = out->mcse_chains;
  a.lambda_hat = out->lambda_hat;
  a.mu_q = c->cfg.mu_q;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  hipError_t e = hipSuccess;
  if (out->occupancy || out->lambda_hat) {
    // the row offsets and lambda0 go up through the pinned stage, after the previous upload
    const hipStream_t st = (hipStream_t)hip_stream;
    const size_t nbo = out->occupancy ? sizeof(int64_t) * (n_wave + 1) : 0;
    const size_t nbl = out->lambda_hat ? sizeof(double) * n_wave : 0;
    if (c->stage_pending) (void)hipEventSynchronize(c->stage_done);
    if (nbo) e = c->poff.ensure(n_wave + 1);
    if (e == hipSuccess && nbl) e = c->plam.ensure(n_wave);
    if (e == hipSuccess) e = c->stage.ensure(nbo + nbl);
    if (e != hipSuccess) {
      (void)hipSetDevice(prev);
      return fail(c, FSMP_ENOMEM, "posterior workspace allocation failed: %s", hipGetErrorString(e));
    }
    char *sp = (char *)c->stage.p;
    if (nbo) {
      std::memcpy(sp, out->offsets, nbo);
      e = hipMemcpyAsync(c->poff.p, sp, nbo, hipMemcpyHostToDevice, st);
      a.occ = in->occ;
      a.occupancy = out->occupancy;
      a.woff = c->poff.p;
      a.sub = c->cfg.grid_sub;
    }
    if (e == hipSuccess && nbl) {
      std::memcpy(sp + nbo, out->lambda, nbl);
      e = hipMemcpyAsync(c->plam.p, sp + nbo, nbl, hipMemcpyHostToDevice, st);
      a.lam0 = c->plam.p;
    }
    if (e == hipSuccess) e = hipEventRecord(c->stage_done, st);
    c->stage_pending = (e == hipSuccess);
  }
  if (e == hipSuccess) e = launch_posterior(a, (hipStream_t)hip_stream);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return fail(c, FSMP_EDEVICE, "posterior launch failed: %s", hipGetErrorString(e));
  return FSMP_OK;
}

}  // extern "C"
