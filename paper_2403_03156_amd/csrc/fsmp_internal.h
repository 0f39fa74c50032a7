// Internal types shared by the host runtime (fsmp_api.hip) and the kernels
// (fsmp_kernels.hip) of libfsmp.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fsmp.h"

namespace fsmp {

// Model constants in the form the kernels use them (all FP64).
struct ModelDev {
  // likelihood in PE space: s = sigma_eps^2, rho = s / sigma_q^2, m = mu_q
  double s, inv_s, rho, log_rho, m, rhom, rhom2;
  // grid and SER table: dt = 1 / sub samples, M = sub * LV table entries; sub_shift =
  // log2(sub) when sub is a power of two (divisions of grid indices become shifts), else -1
  int32_t sub, LV, M, sub_shift;
  double dt;
  // light curve
  int32_t kind, pad1;
  double inv_tau2, inv_tau12, inv_tau1, log_tau2, C, logC;
  double den2, den12;  // -expm1(-dt / tau) for tau2 and tau12
  // t0 prior and proposals
  double t0_min, t0_max, t0_sd, shift_sd;
  double J, logJ;
  // [k][2]: (1 - e^{-k dt / tau2}) / den2, (1 - e^{-k dt / tau12}) / den12 for k = 0 .. ptab_n - 1
  // (device; the geometric series' denominators divided out on the host)
  const double *ptab;
  int64_t ptab_n;
  // MCP-PMT mixture (n_mix > 0): cumulative weights (accumulated in index order) and, per
  // component, rho_e = s / sigma_e^2, log rho_e, rho_e mu_e, rho_e mu_e^2
  int32_t n_mix, pad2;
  double mix_cdf[8], mix_rho[8], mix_lrho[8], mix_rhom[8], mix_rhom2[8];
};

struct ChainArgs {
  ModelDev md;
  const double *vtab;  // [M]  V(m / sub)
  const double *ovl;   // [sub][M] stationary overlaps, lower grid index's phase, offset >= 0
  // batch (device copies)
  const int64_t *woff;
  const double *lam;
  const int32_t *kmax;
  const int32_t *grange;  // [2n]
  const double *t0init;
  const uint64_t *wid;
  const double *mf;       // matched filter sum_n w[n] V(n - g/sub) for g in T, per waveform
  const int64_t *mfoff;   // [n+1]
  const int32_t *chains;  // chain indices (wave * n_chains + chain) of this launch
  int64_t n_list;
  int32_t n_chains, n_steps, burn_in, thin;
  int64_t n_rec;
  uint32_t key0, key1;
  // outputs
  int32_t *n_pe;
  double *t0;
  int32_t *z;
  double *charge;
  double *acc;
  int32_t *nhist;
  int32_t *counts;
  uint32_t *status;
  fsmp_logrec *log;
  double *trace;
  int32_t kz;
  const uint32_t *wflags;  // per waveform, from the prologue (FSMP_ST_NONFINITE)
  double *work;            // optional [chain][5]
  // lane-per-chain kernels: chain state in device memory, interleaved in tiles of
  // 64 chains (element e of the chain in lane l of tile t at (t * E + e) * 64 + l)
  double *dws;
  int32_t *iws;
  // G^-1 rebuilt in FP64 every refresh_M sweeps (0: never; both forms), and the precision
  // form's drift flag bound
  int32_t refresh_M;
  double drift_bound;
  // charge draws at recorded steps (optional): outputs [chain][n_rec][kz] and FP64
  // scratch of KCAP (KCAP + 1) words per chain (per-chain rows for the lane-group kernels,
  // interleaved in tiles of 64 for the lane kernels)
  double *qdraw;
  int32_t *zdraw;
  double *dscr;
  double sigma_eps;
  // replay (lane groups with H in device memory only): recorded proposals [chain][n_steps]
  // to follow, and the delta-nu / log-acceptance computed along them
  const fsmp_logrec *force;
  double *rdnu, *rla;
  // per-waveform sweep counts (device, or NULL: n_steps for all) and the per-chain count
  // of recorded sweeps (output, or NULL)
  const int32_t *wsteps;
  int32_t *rec_steps;
  // grid occupancy rows (zeroed by the prologue), or null: row of waveform w at
  // md.sub * woff[w], one count per grid point
  int32_t *occ;
  // optional initial PE lists (device): chain c starts from zinit[zinit_off[c] ..
  // zinit_off[c + 1]) instead of the empty list
  const int32_t *zinit;
  const int64_t *zinit_off;
  int32_t *comp;  // mixture form: final components [chain][kz], or null
};

struct PrologueArgs {
  ModelDev md;
  const double *vtab;
  const float *wave;
  const int64_t *woff;
  const int32_t *grange;
  const int64_t *mfoff;
  double *mf;
  uint32_t *wflags;  // per waveform: bit1 non-finite sample
  int32_t *occ;      // grid occupancy rows to zero, or null
  int64_t n_wave;
};

struct PosteriorArgs {
  const double *acc;
  const int32_t *nhist;
  const int32_t *counts;
  const uint32_t *cstatus;
  int64_t n_wave;
  int32_t n_chains, kz, n_steps, burn_in;
  const int32_t *rec_steps;  // per chain recorded sweeps, or NULL (n_steps - burn_in)
  double *mean, *var, *mcse, *p_n, *accept;
  uint32_t *status;
  // optional grid occupancy: counts in, expected PEs per grid point out (rows of sub * L_w
  // points at sub * woff[w], woff on the device)
  const int32_t *occ;
  double *occupancy;
  const int64_t *woff;
  int32_t sub;
  // optional chain diagnostics [n_wave][3] and lambda estimates [n_wave][2] (lambda0 per
  // waveform on the device, mu_q of the charge model)
  double *rhat, *mcse_chains, *lambda_hat;
  const double *lam0;
  double mu_q;
};

// Lucy-Richardson initialisation (one workgroup per waveform, everything in LDS)
struct LucyArgs {
  const float *wave;
  const int64_t *woff;     // [n+1]
  const int32_t *kmax;     // [n]
  const double *kern;      // [LVp] V(s) / sum V, zero-padded to LVp (a multiple of 24)
  const double *kern_rev;  // [LVp] kern[LV - 1 - s], zero beyond LV
  int32_t LV, LVp, sub, n_iter, kz;
  int64_t n_wave;
  double inv_area;         // 1 / sum_s V(s): deconvolved flux -> PE charge
  double threshold;
  int32_t margin;          // ns
  double t0_min, t0_max;
  // outputs
  int32_t *z;              // [n][kz]
  int32_t *n_pe;           // [n]
  int32_t *g_range;        // [n][2]
  double *t0;              // [n]
  double *lam;             // [n]
  int32_t *cut;            // [n][2]
  double *qhat;            // optional: row w at woff[w] + w (LV - 1), L_w + LV - 1 entries
};
size_t lucy_lds_bytes(int64_t Lw, int LVp);
hipError_t launch_lucy(const LucyArgs &a, int64_t max_len, hipStream_t st);

// Launchers (fsmp_kernels.hip).  Each returns hipSuccess or the launch error.
hipError_t launch_prologue(const PrologueArgs &a, hipStream_t st);
hipError_t launch_posterior(const PosteriorArgs &a, hipStream_t st);
// lane-group instances for kcap in {16, 32, 48, 64}; fills lanes per chain and blocks
hipError_t launch_chain(int kcap, const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks);
// lane-per-chain variant (FP64, capacities 16 and 32); dws / iws must hold lane_ws_doubles /
// lane_ws_ints(kcap, n_list)
hipError_t launch_chain_lane(int kcap, const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks);
size_t lane_ws_doubles(int kcap, int64_t n_list);
size_t lane_ws_ints(int kcap, int64_t n_list);
// PE capacities of the chain kernels; a waveform runs in the smallest one >= its kmax
constexpr int kNumCaps = 8;
constexpr int kCaps[kNumCaps] = {16, 32, 48, 64, 96, 128, 160, 192};
bool chain_kcap_supported(int kcap, int M, int sub);  // lane-group (LDS) instance exists and fits
// lane groups with H in device memory (FP64, or FP32 in the precision form; `wide`: the
// wider groups, FP64 sampling with the single charge law only): dws must hold
// group_dm_ws_doubles(kcap, n_list, fp32, wide)
hipError_t launch_chain_dm(int kcap, bool fp32, bool wide, const ChainArgs &a, hipStream_t st, int32_t *lanes,
                           int64_t *blocks);
size_t group_dm_ws_doubles(int kcap, int64_t n_list, bool fp32, bool wide = false);
bool chain_dm_supported(int kcap, int M, int sub, bool fp32, bool mcp = false, bool wide = false);
int chain_kcap_for(int kmax);

}  // namespace fsmp
