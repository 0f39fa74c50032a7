// fsmp_kernels.hip -- gfx950 kernels of libfsmp.so.
//
//  * prologue_kernel: per waveform, the matched filter c(g) = sum_n w[n] V(n - g/sub)
//    over the solution space T (FP64 accumulation) and a scan for non-finite samples.
//  * chain_kernel<KCAP, LPC, WPB>: the Gibbs / RJMCMC chains (Sec. 2.4).  A group of
//    LPC lanes owns one chain; a 64-lane wavefront runs 64 / LPC chains side by side.
//    Per chain the LDS holds the inverse PE-space Gram matrix H = G^{-1},
//    G = A^T A + rho I (full symmetric, KCAP x KCAP), the matched-filter terms b, the
//    charge means x = H b and the PE grid indices.  With H at hand
//      birth  : eta = H gamma (one mat-vec), delta^2 = d - gamma^T eta,
//               u+ = (beta - gamma^T x) / delta,
//               delta-nu = -1/2 [-log rho + log delta^2 + (rho m^2 - u+^2) / s];
//      death  : omega = H_jj, delta-nu = 1/2 [-log rho - log omega + (rho m^2 - x_j^2/omega) / s];
//      update : one mat-vec with gamma' (zero at j) and O(1) corrections;
//    accepted moves are rank-one (birth, death) or rank-two (update) edits of H.
//    These are the determinant lemma and Woodbury identity applied in PE space to the
//    normal law of App. A (eq. mgauss); they give the same delta-nu as the paper's
//    N_w x N_w rank-2 form (eqs. 11-18) at O(K^2) instead of O(N_w^2) per step.
//  * posterior_kernel: per waveform, pooled mean / variance / batch-means MCSE.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed,
// counter = (step, block, uid lo, uid hi).  Words of one step: r0,r1 Box-Muller pair
// (t0 step, update shift), r2 t0 accept, r3 move, r4 (r5) index or 53-bit birth
// uniform, r6 jump accept, r7 the mixture component of a born or updated PE (MCP-PMT law).
// Where a chain owns a whole wavefront (and in the FP64 form's 32-lane groups), its lanes
// make these values LPC sweeps at a time, lane l of its group those of sweep LPC m + l, and
// each sweep reads its own by lane reads.

#include <math.h>

#include <algorithm>
#include <type_traits>

#include "fsmp_internal.h"

namespace fsmp {
namespace {

constexpr int kWave = 64;
// FP32 form: the largest error bound, relative to max(1, |delta-nu|), with which a
// proposal is decided from the corrected FP32 evaluation (above it: the FP64 rebuild)
constexpr double kF32Tol = 1e-5;

// Intra-wavefront ordering of LDS traffic between lanes: the LDS executes one
// wavefront's instructions in order; the fences keep the compiler from moving
// memory operations across this point.
#define WAVE_SYNC()                                        \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                     uint32_t *out) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product is one v_mad_u64_u32 (high and low halves together)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ inline double u01(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

__device__ inline double u53(uint32_t lo, uint32_t hi) {
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return (double)(v >> 11) * 0x1p-53 + 0x1p-54;
}

// Standard normal k of the charge draw at `step`: Philox block 2 + k/2, Box-Muller of
// words 0 and 1, the cosine branch for even k and the sine branch for odd k.
__device__ inline double charge_normal(int step, int k, uint32_t uid0, uint32_t uid1, uint32_t key0, uint32_t key1) {
  uint32_t r[4];
  philox4x32_10((uint32_t)step, 2u + (uint32_t)(k >> 1), uid0, uid1, key0, key1, r);
  const double R = sqrt(-2.0 * log(u01(r[0])));
  const double th = 2.0 * M_PI * u01(r[1]);
  return (k & 1) ? R * sin(th) : R * cos(th);
}

// log phi(x); -inf where phi vanishes (x < 0, and x = 0 for BIEXP)
__device__ inline double log_phi(const ModelDev &md, double x) {
  if (md.kind == FSMP_PHI_EXP) return x < 0.0 ? -INFINITY : -x * md.inv_tau2 - md.log_tau2;
  if (!(x > 0.0)) return -INFINITY;
  return md.logC - x * md.inv_tau2 + log(-expm1(-x * md.inv_tau1));
}

// v from the lane the DPP control CTRL selects, for a double (its two halves moved alike)
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// v of lane L of the wavefront, in scalar registers
__device__ inline double lane_value(double v, int L) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), L);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), L);
  return __hiloint2double(hi, lo);
}

// v of lane L of the caller's group of W lanes (group index grp; W >= 16, so at most four
// groups): one lane read per group, the caller's own picked by a select
template <int W>
__device__ inline uint32_t group_lane_u32(uint32_t v, int L, int grp) {
  uint32_t out = (uint32_t)__builtin_amdgcn_readlane((int)v, L);
#pragma unroll
  for (int g = 1; g < kWave / W; ++g) {
    const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)v, g * W + L);
    out = grp == g ? x : out;
  }
  return out;
}
template <int W>
__device__ inline double group_lane(double v, int L, int grp) {
  const uint32_t lo = group_lane_u32<W>((uint32_t)__double2loint(v), L, grp);
  const uint32_t hi = group_lane_u32<W>((uint32_t)__double2hiint(v), L, grp);
  return __hiloint2double((int)hi, (int)lo);
}

// The value of lane K of the caller's group of W lanes (groups aligned to W, every lane of
// the group active): a DPP broadcast inside a quad (W = 4: quad_perm [K, K, K, K]) or a row
// (W = 16: row_newbcast:K), a lane read into scalar registers for a whole wavefront, else a
// lane permute from lane base + K
template <int W, int K>
__device__ inline double group_bcast(double v, int base) {
  if constexpr (W == 4) return dpp_move<K * 0x55>(v);
  else if constexpr (W == 16) return dpp_move<0x150 + K>(v);
  else if constexpr (W == kWave) return lane_value(v, K);
  else return __shfl(v, base + K, kWave);
}
template <int W, int K>
__device__ inline uint32_t group_bcast(uint32_t v, int base) {
  if constexpr (W == 4) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, K * 0x55, 0xF, 0xF, false);
  else if constexpr (W == 16) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + K, 0xF, 0xF, false);
  else if constexpr (W == kWave) return (uint32_t)__builtin_amdgcn_readlane((int)v, K);
  else return (uint32_t)__shfl((int)v, base + K, kWave);
}

// The partial sums of phi over the grid points at or after t0 are geometric series:
// with xs = (first point) dt - t0, the sum over the first k points is
//   EXP:   e^{-xs/tau2} (1 - e^{-k dt/tau2}) / (1 - e^{-dt/tau2}) / tau2,
//   BIEXP: C [e^{-xs/tau2} (1 - e^{-k dt/tau2}) / (1 - e^{-dt/tau2})
//             - e^{-xs/tau12} (1 - e^{-k dt/tau12}) / (1 - e^{-dt/tau12})].
// The t0-dependent factors are computed once per use (XsExp); the count-dependent ones,
// (1 - e^{-k dt/tau}) / (1 - e^{-dt/tau}), come from the table md.ptab ([k][2], k up to the
// longest T, divided on the host), which turns each evaluation of a search into two loads
// and two multiplies.
struct XsExp {
  double e2, e12;
};

__device__ inline XsExp xs_exp(const ModelDev &md, double xs) {
  XsExp x;
  x.e2 = exp(-xs * md.inv_tau2);
  x.e12 = md.kind == FSMP_PHI_EXP ? 0.0 : exp(-xs * md.inv_tau12);
  return x;
}

__device__ inline double phi_partial(const ModelDev &md, const XsExp &x, int64_t k) {
  const double a = x.e2 * md.ptab[2 * k];
  if (md.kind == FSMP_PHI_EXP) return a * md.inv_tau2;
  const double b = x.e12 * md.ptab[2 * k + 1];
  return md.C * (a - b);
}

struct GridPos {
  int64_t gs;  // first grid point of T with g dt >= t0
  int64_t n;   // points of T from gs on (<= 0: none)
  double xs;   // gs dt - t0
};

__device__ inline GridPos grid_pos(const ModelDev &md, double t0, int glo, int ghi) {
  GridPos p;
  int64_t gs = (int64_t)ceil(t0 / md.dt);
  if (gs < glo) gs = glo;
  p.gs = gs;
  p.n = (int64_t)ghi - gs + 1;
  p.xs = (double)gs * md.dt - t0;
  return p;
}

__device__ inline double phi_total(const ModelDev &md, double t0, int glo, int ghi) {
  const GridPos p = grid_pos(md, t0, glo, ghi);
  return p.n > 0 ? phi_partial(md, xs_exp(md, p.xs), p.n) : 0.0;
}

// phi_total for a chain's lane group (t0, glo, ghi the same in all its lanes, every lane
// active): the two exponentials are one evaluation (the group's first lane e2, its second
// e12)
template <int W>
__device__ inline double phi_total_group(const ModelDev &md, double t0, int glo, int ghi, int lane, int base) {
  const GridPos p = grid_pos(md, t0, glo, ghi);
  const double v = exp(-p.xs * (lane == 0 ? md.inv_tau2 : md.inv_tau12));
  XsExp x;
  x.e2 = group_bcast<W, 0>(v, base);
  const double v12 = group_bcast<W, 1>(v, base);
  x.e12 = md.kind == FSMP_PHI_EXP ? 0.0 : v12;
  return p.n > 0 ? phi_partial(md, x, p.n) : 0.0;
}

// Sum over a group of W lanes (W a power of two, groups aligned to W): a butterfly over lane
// offsets W/2, ..., 2, 1, each lane adding the value of lane (its index xor the offset), so
// every lane ends with the same sum.  Offsets of 16 and more go through lane permutes; the
// rest are DPP moves inside a row of 16: xor 8 is a rotation of the row by 8, xor 4 after it
// a rotation by 4 (the values then depend only on the lane index mod 8, where a rotation by
// 4 and xor 4 agree), xor 2 and xor 1 quad permutations.  The pairs, and so the sums, are
// the same as with lane permutes for every offset.  A whole wavefront (W = 64) sums its four
// rows of 16 so and adds the row sums, read from lanes 0, 16, 32 and 48 into scalar
// registers, in that order (no lane permutes, and the result is a scalar).
template <int W>
__device__ inline double group_sum(double v) {
  if constexpr (W == kWave) {
    // a whole wavefront: the rows of 16 lanes by DPP, then their four sums from lanes 0, 16,
    // 32 and 48 into scalar registers, added in that order
    v += dpp_move<0x128>(v);  // row_ror:8
    v += dpp_move<0x124>(v);  // row_ror:4
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]: xor 2
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]: xor 1
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
  }
#pragma unroll
  for (int o = W / 2; o >= 16; o >>= 1) v += __shfl_xor(v, o, W);
  if constexpr (W >= 16) {
    v += dpp_move<0x128>(v);  // row_ror:8
    v += dpp_move<0x124>(v);  // row_ror:4
  } else if constexpr (W == 8) {
    v += __shfl_xor(v, 4, W);
  }
  if constexpr (W >= 4) v += dpp_move<0x4E>(v);  // quad_perm [2, 3, 0, 1]: xor 2
  if constexpr (W >= 2) v += dpp_move<0xB1>(v);  // quad_perm [1, 0, 3, 2]: xor 1
  return v;
}

template <int W>
__device__ inline int group_or(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, W);
  return v;
}

template <int W>
__device__ inline int group_min(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    const int u = __shfl_xor(v, o, W);
    v = u < v ? u : v;
  }
  return v;
}

// The logs of two values that are the same in every lane of a chain's group, in one
// evaluation: the group's first lane takes x0, its second x1, and both results go to the
// whole group (base = the group's first lane; every lane of the group must be active)
template <int W>
__device__ inline void group_log2(double x0, double x1, int lane, int base, double &l0, double &l1) {
  const double v = log(lane == 0 ? x0 : x1);
  l0 = group_bcast<W, 0>(v, base);
  l1 = group_bcast<W, 1>(v, base);
}

// BIEXP part of log phi that depends on t0: log(1 - e^{-(t - t0) / tau_rise})
__device__ inline double rise_term(const ModelDev &md, int g, double t0) {
  return log(-expm1(-((double)g * md.dt - t0) * md.inv_tau1));
}

// its factor 1 - e^{-(t - t0) / tau_rise}, in (0, 1) for t > t0; t - t0 is at least an ulp
// of t0, so a product of eight factors stays far above the FP64 underflow threshold
__device__ inline double rise_factor(const ModelDev &md, int g, double t0) {
  return -expm1(-((double)g * md.dt - t0) * md.inv_tau1);
}

// v / sub and v % sub for v >= 0 (grid indices): shifts when sub is a power of two
__device__ inline int sub_div(const ModelDev &md, int v) { return md.sub_shift >= 0 ? v >> md.sub_shift : v / md.sub; }
__device__ inline int sub_mod(const ModelDev &md, int v) {
  return md.sub_shift >= 0 ? v & (md.sub - 1) : v % md.sub;
}

// overlap sum_{n < Lw} V(n - g1/sub) V(n - g2/sub): the stationary table unless both
// columns run past the window end, then the direct sum over the samples left
__device__ inline double overlap(const ModelDev &md, const double *vt, const double *ov, int g1, int g2, int Lw) {
  const int lo = g1 < g2 ? g1 : g2, hi = g1 < g2 ? g2 : g1;
  const int d = hi - lo;
  if (d >= md.M) return 0.0;
  const int nhi = sub_div(md, lo + md.M - 1);  // last sample of the earlier column
  if (nhi < Lw) return ov[sub_mod(md, lo) * md.M + d];
  double s = 0.0;
  const int n0 = sub_div(md, hi + md.sub - 1);
  for (int n = n0; n < Lw; ++n) s += vt[md.sub * n - lo] * vt[md.sub * n - hi];
  return s;
}

// birth position: smallest g in T with sum_{g' <= g} phi(g' dt - t0) > target
template <int LPC>
__device__ inline int birth_draw(const ModelDev &md, double t0, int glo, int ghi, double target, int lane, int grp) {
  const GridPos p = grid_pos(md, t0, glo, ghi);
  XsExp xe;
  {
    // the two exponentials in one evaluation (the group's first lane e2, its second e12)
    const double v = exp(-p.xs * (lane == 0 ? md.inv_tau2 : md.inv_tau12));
    xe.e2 = group_bcast<LPC, 0>(v, grp * LPC);
    const double v12 = group_bcast<LPC, 1>(v, grp * LPC);
    xe.e12 = md.kind == FSMP_PHI_EXP ? 0.0 : v12;
  }
  int64_t k;
  if (md.kind == FSMP_PHI_EXP) {
    // closed-form inverse of the truncated geometric law
    const double c = target * exp(p.xs * md.inv_tau2) * md.den2 / md.inv_tau2;
    if (c >= 1.0) {
      k = p.n - 1;
    } else {
      const double L = -log1p(-c) / (md.dt * md.inv_tau2);
      k = (int64_t)floor(L);
      if (k < 0) k = 0;
      if (k > p.n - 1) k = p.n - 1;
      // settle rounding at the boundary against the partial sums
      if (k > 0 && phi_partial(md, xe, k) > target) k -= 1;
      else if (k < p.n - 1 && !(phi_partial(md, xe, k + 1) > target)) k += 1;
    }
  } else {
    // LPC-ary search on the closed-form partial sums
    int64_t lo = 0, hi = p.n - 1;
    const uint64_t gmask = (LPC == 64) ? ~0ull : ((1ull << LPC) - 1ull);
    while (hi > lo) {
      const int64_t span = hi - lo + 1;
      const int64_t step = (span + LPC - 1) / LPC;
      int64_t kl = lo + (int64_t)(lane + 1) * step - 1;
      if (kl > hi) kl = hi;
      const bool pred = phi_partial(md, xe, kl + 1) > target;
      const uint64_t bal = (__ballot(pred) >> (grp * LPC)) & gmask;
      if (bal == 0) {
        lo = hi;
        break;
      }
      const int l = __ffsll((unsigned long long)bal) - 1;
      int64_t khi = lo + (int64_t)(l + 1) * step - 1;
      if (khi > hi) khi = hi;
      const int64_t klo = (l == 0) ? lo : lo + (int64_t)l * step;
      lo = klo;
      hi = khi;
    }
    k = lo;
  }
  return (int)(p.gs + k);
}

// ------------------------------------------------------------------ grid occupancy
// The occupancy row of waveform w (grid_sub * L_w points from grid_sub * offsets[w]) counts,
// over its chains' recorded sweeps, the PEs at every grid point.  It is accumulated by
// residence instead of per sweep: a PE that arrives in sweep s is present at the end of
// the sweeps s .. n_steps - 1, so it adds the recorded ones among them, n_steps - max(s,
// burn); one that leaves in sweep s removes the same amount.  The sum over a PE's arrival
// and departure is its number of recorded sweeps at that point, PEs still present at the
// end keep their arrival's count, and a chain starts empty.  Edits that cancel (both before
// burn-in) cost two atomics; nothing waits for the adds.
__device__ inline void occ_edit(const ChainArgs &a, int64_t c, int move, int gj, int gnew, int step, int burn,
                                int n_steps) {
  const int rem = n_steps - (step > burn ? step : burn);
  if (!a.occ || rem <= 0) return;
  // the row is looked up here rather than kept live across the sweep loop
  int32_t *row = a.occ + a.md.sub * a.woff[c / a.n_chains];
  if (move != 1) atomicAdd(row + gj, -rem);
  if (move != 2) atomicAdd(row + gnew, rem);
}

// ------------------------------------------------------------------ prologue
__global__ void __launch_bounds__(256) prologue_kernel(PrologueArgs a) {
  extern __shared__ double vt[];
  const ModelDev &md = a.md;
  for (int i = threadIdx.x; i < md.M; i += blockDim.x) vt[i] = a.vtab[i];
  __syncthreads();
  for (int64_t w = blockIdx.x; w < a.n_wave; w += gridDim.x) {
    const float *x = a.wave + a.woff[w];
    const int Lw = (int)(a.woff[w + 1] - a.woff[w]);
    int bad = 0;
    for (int n = threadIdx.x; n < Lw; n += blockDim.x)
      if (!isfinite(x[n])) bad = 1;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) a.wflags[w] = bad ? FSMP_ST_NONFINITE : 0u;
    if (a.occ)
      for (int64_t g = threadIdx.x; g < (int64_t)md.sub * Lw; g += blockDim.x) a.occ[md.sub * a.woff[w] + g] = 0;
    const int glo = a.grange[2 * w], ghi = a.grange[2 * w + 1];
    double *out = a.mf + a.mfoff[w];
    // four consecutive grid points per thread share each sample load; every point sums its
    // own samples n0(g) .. n1(g) in increasing n (both bounds nondecreasing in g)
    for (int g0 = glo + 4 * (int)threadIdx.x; g0 <= ghi; g0 += 4 * (int)blockDim.x) {
      int n0[4], n1[4];
      double s[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = g0 + u;
        n0[u] = g <= ghi ? sub_div(md, g + md.sub - 1) : INT32_MAX;
        n1[u] = g <= ghi ? sub_div(md, g + md.M - 1) : -1;
        if (n1[u] > Lw - 1) n1[u] = Lw - 1;
        s[u] = 0.0;
      }
      const int gl = ghi - g0 < 3 ? ghi - g0 : 3;
      // samples that all four points take (four points in T) need no range checks
      const int blo = gl == 3 ? n0[3] : INT32_MAX, bhi = n1[0];
      int n = n0[0];
      for (; n <= n1[gl] && n < blo; ++n) {
        const double xv = (double)x[n];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (n >= n0[u] && n <= n1[u]) s[u] += xv * vt[md.sub * n - (g0 + u)];
      }
      for (; n <= bhi; ++n) {
        const double xv = (double)x[n];
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += xv * vt[md.sub * n - (g0 + u)];
      }
      for (; n <= n1[gl]; ++n) {
        const double xv = (double)x[n];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (n >= n0[u] && n <= n1[u]) s[u] += xv * vt[md.sub * n - (g0 + u)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (g0 + u <= ghi) out[g0 + u - glo] = s[u];
    }
  }
}

// ------------------------------------------------------------------ chains
// LDS block of one chain: H (unless it lives in device memory), x, two scratch vectors (six
// and b in the FP32 form; b and the residual b - G x in the corrected FP64 form), the
// accumulators (kAcc doubles: 12 sums, 3 open batch sums, 5 work counters, then 8 int
// proposal / accept counts and the current run of N: value, first step), then the int grid
// indices.  The accumulators live in LDS, updated by the group's first lane, to keep
// registers free; the N histogram is kept in the output row by run lengths.
//
// kCorr, the corrected FP64 form (H in device memory, capacities from 48 up): FP64 arithmetic through an explicit inverse leaves x = G^-1 b with an error of about
// kappa(G) eps, which u+ = beta - gamma^T x and x_j carry into delta-nu magnified by
// 1 / (sigma_eps^2 delta^2) -- about 1e-8 of delta-nu on pile-up windows at K ~ 100, with or
// without rebuilds of G^-1.  That form keeps the exact G in device memory and the residual
// s = b - G x (recomputed after every accepted move), and evaluates
// gamma^T G^-1 b = gamma^T x + eta^T s and x_j = x_j + h^T s (eta = H gamma, h = row j of H),
// exact to first order in the error of H; the other quantities (delta^2, omega) need no
// correction at this precision.
template <int KCAP, bool HG, bool F32 = false, bool MCP = false>
struct ChainLayout {
  static constexpr int LD = KCAP;
  static constexpr int kAcc = 25;
  static constexpr bool kCorr = HG && !F32 && KCAP >= 48;
  static constexpr bool kKeepG = F32 || kCorr;  // the exact G in device memory, b per PE
  // the FP32 form keeps b (matched filter + rho mu_q per PE) for its residuals and refresh,
  // and the vectors of its corrected proposals; the mixture form the PEs' components after
  // their grid indices
  static constexpr int kVec = F32 ? 8 : (kCorr ? 5 : 3);
  static constexpr int kDoubles =
      (HG ? 0 : KCAP * KCAP) + kVec * KCAP + kAcc + (KCAP + 1) / 2 + (MCP ? (KCAP + 1) / 2 : 0);
};

// Column i of H owned by one lane: element (k, i) at H[(k * LD + i) * HS] (HS = 1 in LDS;
// the number of chains of a wavefront in device memory, where the wavefront's chains are
// interleaved element by element).  Loads go in chunks of 16 rows with one chain per
// wavefront and of 8 with several (whose kernels are short of registers: the smaller chunk
// keeps their spills down), issued unconditionally (rows below the capacity, a multiple of
// 16) with the rows past N dropped by a select, so a chunk costs one memory round trip;
// terms are summed in row order.
template <int LD, int HS, typename MT>
__device__ inline double grp_col_dot(const MT *H, const double *g, int i, int N) {
  constexpr int RC = HS > 1 ? 8 : 16;
  double e = 0.0;
  for (int k0 = 0; k0 < N; k0 += RC) {
    double h[RC], v[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      h[u] = (double)H[((k0 + u) * LD + i) * HS];
      v[u] = g[k0 + u];
    }
#pragma unroll
    for (int u = 0; u < RC; ++u) e = (k0 + u < N) ? e + h[u] * v[u] : e;
  }
  return e;
}

// H(k, i) += ai A_k cA [+ bi B_k cB] for k < N (loads of a chunk unconditional, stores guarded;
// an FP32 H is read into FP64 and written back rounded)
template <int LD, int HS, bool TWO, typename MT>
__device__ inline void grp_col_update(MT *H, int i, int N, double ai, const double *A, double cA, double bi,
                                      const double *B, double cB) {
  for (int k0 = 0; k0 < N; k0 += 8) {
    double h[8], av[8], bw[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      h[u] = (double)H[((k0 + u) * LD + i) * HS];
      av[u] = A[k0 + u];
      if (TWO) bw[u] = B[k0 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double v = TWO ? h[u] + (ai * av[u] * cA + bi * bw[u] * cB) : h[u] + ai * av[u] * cA;
      if (k0 + u < N) H[((k0 + u) * LD + i) * HS] = (MT)v;
    }
  }
}

// Residuals against the exact Gram matrix G = A^T A + rho I of the PE list (FP64, kept in
// device memory in the layout of H), for the rows i owned by this lane of the group:
//   r1 = g1 - G v1 (if v1),  r2 = e_u2 - G v2 (if v2; e_u2 the unit vector at u2),
//   r3 = t3 - G v3.
// Loads in chunks of 8 rows, terms in row order.
template <int LPC, int LD, int HS>
__device__ inline void gram_resid3(const double *Gm, int N, int lane, const double *g1, const double *v1, int u2,
                                   const double *v2, const double *t3, const double *v3, double *r1, double *r2,
                                   double *r3) {
  for (int i = lane; i < N; i += LPC) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k0 = 0; k0 < N; k0 += 8) {
      double g[8], x1[8], x2[8], x3[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        g[u] = Gm[((k0 + u) * LD + i) * HS];
        x1[u] = v1 ? v1[k0 + u] : 0.0;
        x2[u] = v2 ? v2[k0 + u] : 0.0;
        x3[u] = v3[k0 + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = k0 + u < N;
        a = in ? a + g[u] * x1[u] : a;
        b = in ? b + g[u] * x2[u] : b;
        c = in ? c + g[u] * x3[u] : c;
      }
    }
    if (v1) r1[i] = g1[i] - a;
    if (v2) r2[i] = (i == u2 ? 1.0 : 0.0) - b;
    r3[i] = t3[i] - c;
  }
}

// s = b - G x against the exact G, for the rows i owned by this lane of the group
template <int LPC, int LD, int HS>
__device__ inline void gram_resid_b(const double *Gm, const double *bv, const double *xv, double *rs, int N,
                                    int lane) {
  for (int i = lane; i < N; i += LPC) rs[i] = bv[i] - grp_col_dot<LD, HS>(Gm, xv, i, N);
}

// column i of G (overlap tables, plus the PE's own ridge rho_g on the diagonal) for the PE at
// grid point g against the list zg[0..N), written as row and column i of Gm by the lanes of
// the group (g's own entry by the first lane); zg[i] is not read
template <int LPC, int LD, int HS>
__device__ inline void gram_set(const ModelDev &md, const double *vt, const double *ov, int Lw, double *Gm,
                                const int *zg, int N, int i, int g, double rho_g, int lane) {
  for (int k = lane; k < N; k += LPC) {
    if (k == i) continue;
    const double v = overlap(md, vt, ov, g, zg[k], Lw);
    Gm[(i * LD + k) * HS] = v;
    Gm[(k * LD + i) * HS] = v;
  }
  if (lane == 0) Gm[(i * LD + i) * HS] = overlap(md, vt, ov, g, g, Lw) + rho_g;
}

template <int W>
__device__ inline double group_max(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
  return v;
}

// G^-1 of the PE list zg[0..N) by bordering, in FP64 into M (layout of the lane-group
// kernels; M may hold the old G^-1: only its leading block built so far is read), each step
// the birth update of the inverse of the leading block, its columns owned by the group's
// lanes: false if a Schur complement is not positive.  ek: the PEs' mixture components (their
// own ridge rho_e on the diagonal), or null for the single charge law.  s1, s2: scratch.
template <int LPC, int LD, int HS>
__device__ bool grp_build(const ModelDev &md, const double *vt, const double *ov, int Lw, double *M, double *s1,
                          double *s2, const int *zg, int N, int lane, const int *ek = nullptr) {
  for (int k = 0; k < N; ++k) {
    const int gk = zg[k];
    for (int i = lane; i < k; i += LPC) s1[i] = overlap(md, vt, ov, gk, zg[i], Lw);
    const double d = overlap(md, vt, ov, gk, gk, Lw) + (ek ? md.mix_rho[ek[k]] : md.rho);
    WAVE_SYNC();
    double q = 0.0;
    for (int i = lane; i < k; i += LPC) {
      const double e = grp_col_dot<LD, HS>(M, s1, i, k);
      s2[i] = e;
      q += s1[i] * e;
    }
    q = group_sum<LPC>(q);
    const double delta2 = d - q;
    if (!(delta2 > 0.0)) return false;
    const double inv = 1.0 / delta2;
    WAVE_SYNC();
    for (int i = lane; i < k; i += LPC) {
      const double ei = s2[i];
      grp_col_update<LD, HS, false>(M, i, k, ei, s2, inv, 0.0, s2, 0.0);
      M[(k * LD + i) * HS] = -ei * inv;
      M[(i * LD + k) * HS] = -ei * inv;
    }
    if (lane == 0) M[(k * LD + k) * HS] = inv;
    WAVE_SYNC();
  }
  return true;
}

// Precision form: rebuild G^-1 of the current PE list in FP64 into W, recompute x = G^-1 b in
// FP64 and round W into the FP32 H.  False if a Schur complement is not positive.  `drift` =
// the largest change of a charge mean, relative to max(1, |x|).  s1, s2 are scratch.
template <int LPC, int LD, int HS, typename HT>
__device__ bool grp_refresh(const ModelDev &md, const double *vt, const double *ov, int Lw, double *W, HT *H,
                            double *xv, const double *bv, double *s1, double *s2, const int *zg, int N, int lane,
                            double &drift) {
  if (!grp_build<LPC, LD, HS>(md, vt, ov, Lw, W, s1, s2, zg, N, lane)) return false;
  double dr = 0.0;
  for (int i = lane; i < N; i += LPC) {
    const double xi = grp_col_dot<LD, HS>(W, bv, i, N);
    dr = fmax(dr, fabs(xi - xv[i]) / fmax(1.0, fabs(xi)));
    xv[i] = xi;
  }
  drift = group_max<LPC>(dr);
  for (int i = lane; i < N; i += LPC)
    for (int k = 0; k < N; ++k) H[(k * LD + i) * HS] = (HT)W[(k * LD + i) * HS];
  WAVE_SYNC();
  return true;
}

// HG: H in device memory (a.dws, the chains of a wavefront interleaved element by element),
// which leaves the LDS to the tables and the vectors and so fits many more chains per CU;
// otherwise H in LDS.  FORCE (replay): every step follows the recorded proposal of a.force
// (t0 after the half-step, move, index, grid point, accept bit) instead of the chain's
// own draws, and writes the delta-nu and log-acceptance it computes to a.rdnu / a.rla.
// MCP: the Gaussian-mixture charge law, every PE with its component.
template <int KCAP, int LPC, int WPB, bool HG, bool FORCE, bool F32, bool MCP>
__global__ void __launch_bounds__(kWave *WPB) __attribute__((amdgpu_waves_per_eu(2))) chain_kernel(ChainArgs a) {
  static_assert(!F32 || (HG && !FORCE), "the FP32 form keeps H in device memory and does not replay");
  static_assert(!MCP || (HG && !FORCE && !F32), "the mixture form runs FP64 with H in device memory");
  static_assert(KCAP % 16 == 0, "the column loads go in chunks of 16 rows below the capacity");
  using HT = typename std::conditional<F32, float, double>::type;
  constexpr int CPW = kWave / LPC;
  using CL = ChainLayout<KCAP, HG, F32, MCP>;
  constexpr int LD = CL::LD;
  constexpr int HS = HG ? CPW : 1;
  extern __shared__ double smem[];
  const ModelDev &md = a.md;
  double *vt = smem;
  double *ov = smem + md.M;
  for (int i = threadIdx.x; i < md.M; i += blockDim.x) vt[i] = a.vtab[i];
  for (int i = threadIdx.x; i < md.sub * md.M; i += blockDim.x) ov[i] = a.ovl[i];
  double *lgn = ov + md.sub * md.M;  // log k, k = 0..KCAP + 1
  for (int i = threadIdx.x; i < KCAP + 2; i += blockDim.x) lgn[i] = log((double)i);
  __syncthreads();

  // the wavefront's index is the same in all its lanes: taken from the first, it and what
  // follows from it (the tile, and with one chain per wavefront the chain and its waveform's
  // parameters) are held in scalar registers, which keeps those kernels free of spills
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)), l64 = threadIdx.x % kWave;
  const int grp = l64 / LPC, lane = l64 % LPC;
  const int gbase = grp * LPC;  // the group's first lane in the wavefront
  const int64_t tile = (int64_t)blockIdx.x * WPB + wv;
  const int64_t slot = tile * CPW + grp;
  if (slot >= a.n_list) return;

  double *cb = smem + md.M * (1 + md.sub) + (KCAP + 2) + (int64_t)(wv * CPW + grp) * CL::kDoubles;
  // device memory of a tile (the wavefront's chains interleaved element by element): H in its
  // storage type; in the FP32 form then the FP64 refresh matrix W and the exact G (FP64), in
  // the corrected FP64 form the exact G
  constexpr bool CORR = CL::kCorr, KEEPG = CL::kKeepG;
  constexpr int64_t kHD = (int64_t)KCAP * LD * CPW * (int64_t)sizeof(HT) / 8;
  constexpr int64_t kTile = kHD + (F32 ? 2 : CORR ? 1 : 0) * (int64_t)KCAP * LD * CPW;
  HT *H = HG ? (HT *)(a.dws + tile * kTile) + grp : (HT *)cb;
  double *W = F32 ? a.dws + tile * kTile + kHD + grp : nullptr;
  double *Gm = F32    ? a.dws + tile * kTile + kHD + (int64_t)KCAP * LD * CPW + grp
               : CORR ? a.dws + tile * kTile + kHD + grp
                      : nullptr;
  double *xv = HG ? cb : cb + KCAP * LD;
  double *s1 = xv + KCAP;
  double *s2 = s1 + KCAP;
  // FP32 form: four more scratch vectors and b of each PE; corrected FP64 form: b and the
  // residual s = b - G x
  double *s3 = F32 ? s2 + KCAP : nullptr;
  double *s4 = F32 ? s3 + KCAP : nullptr;
  double *s5 = F32 ? s4 + KCAP : nullptr;
  double *s6 = F32 ? s5 + KCAP : nullptr;
  double *bv = F32 ? s6 + KCAP : CORR ? s2 + KCAP : nullptr;
  double *rs = CORR ? bv + KCAP : nullptr;
  double *acc = xv + CL::kVec * KCAP;  // [0..11] sums, [12..14] open batch sums, [15..19] work counters
  int *cnt = (int *)(acc + 20);
  int *run = cnt + 8;  // N of the current run among the recorded steps (-1: none yet), its first step
  int *zg = (int *)(acc + CL::kAcc);
  int *ek = zg + 2 * ((KCAP + 1) / 2);  // mixture form: the PEs' components

  const int64_t c = a.chains[slot];
  const int64_t w = c / a.n_chains;
  const int ch = (int)(c % a.n_chains);
  const int Lw = (int)(a.woff[w + 1] - a.woff[w]);
  const double lam = a.lam[w];
  const int kmax = a.kmax[w];
  const int glo = a.grange[2 * w], ghi = a.grange[2 * w + 1];
  const double *mf = a.mf + a.mfoff[w];
  const uint64_t uid = a.wid[w] * (uint64_t)a.n_chains + (uint64_t)ch;
  const uint32_t uid0 = (uint32_t)uid, uid1 = (uint32_t)(uid >> 32);
  uint32_t st = a.wflags[w];
  if (glo > ghi) st |= FSMP_ST_EMPTY_T;
  // this waveform's sweeps and burn-in (the configured burn-in fraction), batch means
  const int steps_w = a.wsteps ? a.wsteps[w] : a.n_steps;
  const int burn = a.wsteps ? (int)((int64_t)steps_w * a.burn_in / a.n_steps) : a.burn_in;
  const int n_steps = (st & FSMP_ST_NONFINITE) ? 0 : steps_w;
  const int S_rec = n_steps > burn ? n_steps - burn : 0;
  const int nb = S_rec > 0 ? (int)floor(sqrt((double)S_rec)) : 0;
  const int lb = nb > 0 ? S_rec / nb : 0;

  // N histogram: the output row, zeroed here, receives the length of every run of equal
  // N among the recorded steps (atomic adds that nothing waits for)
  for (int k = lane; k <= a.kz; k += LPC) a.nhist[c * (a.kz + 1) + k] = 0;
  if (lane == 0) {
    run[0] = -1;
    run[1] = 0;
  }
  WAVE_SYNC();

  double t0 = a.t0init[w];
  int N = 0;
  double Phi = (glo <= ghi) ? phi_total_group<LPC>(md, t0, glo, ghi, lane, gbase) : 0.0;
  // Lambda_T changes only with t0 (its log is taken with the jump's own log); S_cur = sum
  // over PEs of the BIEXP rise term at the current t0 and gmin = the smallest PE grid index
  // (phi must stay positive at every PE) make the t0 step one term per PE
  double Lam = lam * md.dt * Phi;
  const bool biexp = md.kind == FSMP_PHI_BIEXP;
  double S_cur = 0.0;
  int gmin = INT32_MAX;
  if (lane == 0) {
    for (int i = 0; i < 20; ++i) acc[i] = 0.0;
    for (int i = 0; i < 8; ++i) cnt[i] = 0;
  }
  WAVE_SYNC();

  // a caller-supplied initial PE list: G^-1 (FP64, by bordering) and x = G^-1 b of the
  // list before the first sweep; no random numbers are drawn for it
  if (a.zinit && n_steps > 0) {
    const int n0 = (int)(a.zinit_off[c + 1] - a.zinit_off[c]);
    if (n0 > 0) {
      const int32_t *z0 = a.zinit + a.zinit_off[c];
      for (int k = lane; k < n0; k += LPC) zg[k] = z0[k];
      WAVE_SYNC();
      double *M = F32 ? W : (double *)H;
      if (grp_build<LPC, LD, HS>(md, vt, ov, Lw, M, s1, s2, zg, n0, lane)) {
        for (int k = lane; k < n0; k += LPC) s1[k] = mf[zg[k] - glo] + md.rhom;  // b
        WAVE_SYNC();
        for (int i = lane; i < n0; i += LPC) {
          xv[i] = grp_col_dot<LD, HS>(M, s1, i, n0);
          if constexpr (KEEPG) {
            bv[i] = s1[i];
            for (int k = 0; k < n0; ++k) {
              if constexpr (F32) H[(k * LD + i) * HS] = (HT)W[(k * LD + i) * HS];
              Gm[(k * LD + i) * HS] = overlap(md, vt, ov, zg[k], zg[i], Lw) + (k == i ? md.rho : 0.0);
            }
          }
        }
        if constexpr (CORR) {
          WAVE_SYNC();
          gram_resid_b<LPC, LD, HS>(Gm, bv, xv, rs, n0, lane);
        }
        N = n0;
        double sn = 0.0;
        int m = INT32_MAX;
        for (int i = lane; i < N; i += LPC) {
          if (biexp) sn += rise_term(md, zg[i], t0);
          m = zg[i] < m ? zg[i] : m;
          occ_edit(a, c, 1, -1, zg[i], 0, burn, n_steps);
        }
        S_cur = group_sum<LPC>(sn);
        gmin = group_min<LPC>(m);
      } else {
        st |= FSMP_ST_FACTOR;
      }
      WAVE_SYNC();
    }
  }
  // with one chain per wavefront, or in the FP64 form's 32-lane groups, lane l of a chain's
  // group keeps the random values of its sweep LPC m + l
  constexpr bool kStash = LPC == kWave || (LPC == 32 && !F32 && !MCP);
  uint32_t st_r3 = 0, st_r4 = 0, st_r5 = 0, st_r7 = 0;
  double st_l2 = 0.0, st_l6 = 0.0, st_xt = 0.0, st_xs = 0.0;
  for (int step = 0; step < n_steps; ++step) {
    if (a.refresh_M > 0 && step > 0 && step % a.refresh_M == 0 && N > 0) {
      if constexpr (F32) {
        // precision form: FP64 rebuild of G^{-1} every refresh_M sweeps
        double drift;
        if (!grp_refresh<LPC, LD, HS>(md, vt, ov, Lw, W, H, xv, bv, s1, s2, zg, N, lane, drift)) st |= FSMP_ST_FACTOR;
        else if (drift > a.drift_bound) st |= FSMP_ST_DRIFT;
      } else if constexpr (!CORR) {
        // FP64 form: G^-1 rebuilt in place by bordering and x = G^-1 b recomputed, against the
        // rounding the rank-one and rank-two edits accumulate (the corrected form needs none:
        // the residual against the exact G takes up what the edits leave in x, and over 4,000
        // sweeps at K ~ 100 its delta-nu is as close to the exact one without rebuilds as with)
        if (grp_build<LPC, LD, HS>(md, vt, ov, Lw, (double *)H, s1, s2, zg, N, lane, MCP ? ek : nullptr)) {
          for (int i = lane; i < N; i += LPC) s1[i] = mf[zg[i] - glo] + (MCP ? md.mix_rhom[ek[i]] : md.rhom);
          WAVE_SYNC();
          for (int i = lane; i < N; i += LPC) xv[i] = grp_col_dot<LD, HS>((double *)H, s1, i, N);
          WAVE_SYNC();
        } else {
          st |= FSMP_ST_FACTOR;
        }
      }
    }
    // The step's random words and the logs of its three uniforms (Box-Muller radius, t0
    // acceptance, jump acceptance) do not depend on the chain's state: the group's first
    // lane makes Philox block 0 and its second lane block 1, its first three lanes one log
    // each, and the values go to the whole group by lane permutes (the same values as
    // computing all of it in every lane, with a third of the VALU work)
    static_assert(LPC >= 4, "a chain's group needs at least three lanes");
    uint32_t r[8];
    double lg2, lg6;      // log u01(r2), log u01(r6)
    double xi_t0, xi_sh;  // the Box-Muller pair of (r0, r1)
    if constexpr (kStash) {
      // every LPC sweeps each lane of a chain's group makes the random values of one of the
      // group's next LPC sweeps (both Philox blocks, the three logs, the Box-Muller pair), the
      // same functions of the same words as below, so the same values; a sweep reads its own
      // by lane reads (one per group of the wavefront, its own picked), off the sweep's
      // dependent path
      const int sl = step & (LPC - 1);
      if (sl == 0) {
        uint32_t q0[4], q1[4];
        philox4x32_10((uint32_t)(step + lane), 0u, uid0, uid1, a.key0, a.key1, q0);
        philox4x32_10((uint32_t)(step + lane), 1u, uid0, uid1, a.key0, a.key1, q1);
        const double R = sqrt(-2.0 * log(u01(q0[0])));
        const double th = 2.0 * M_PI * u01(q0[1]);
        st_xt = R * cos(th);
        st_xs = R * sin(th);
        st_l2 = log(u01(q0[2]));
        st_l6 = log(u01(q1[2]));
        st_r3 = q0[3];
        st_r4 = q1[0];
        st_r5 = q1[1];
        st_r7 = q1[3];
      }
      r[0] = r[1] = r[2] = r[6] = 0u;  // consumed by the values above
      r[3] = group_lane_u32<LPC>(st_r3, sl, grp);
      r[4] = group_lane_u32<LPC>(st_r4, sl, grp);
      r[5] = group_lane_u32<LPC>(st_r5, sl, grp);
      r[7] = group_lane_u32<LPC>(st_r7, sl, grp);
      lg2 = group_lane<LPC>(st_l2, sl, grp);
      lg6 = group_lane<LPC>(st_l6, sl, grp);
      xi_t0 = group_lane<LPC>(st_xt, sl, grp);
      xi_sh = group_lane<LPC>(st_xs, sl, grp);
    } else {
      double lg0;  // log u01(r0)
      {
        const int base = gbase;
        uint32_t q[4];
        philox4x32_10((uint32_t)step, (uint32_t)(lane & 1), uid0, uid1, a.key0, a.key1, q);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          r[u] = group_bcast<LPC, 0>(q[u], base);
          r[4 + u] = group_bcast<LPC, 1>(q[u], base);
        }
        const double lv = log(u01(lane == 0 ? r[0] : lane == 1 ? r[2] : r[6]));
        lg0 = group_bcast<LPC, 0>(lv, base);
        lg2 = group_bcast<LPC, 1>(lv, base);
        lg6 = group_bcast<LPC, 2>(lv, base);
      }
      const double R = sqrt(-2.0 * lg0);
      const double th = 2.0 * M_PI * u01(r[1]);
      xi_t0 = R * cos(th);
      xi_sh = R * sin(th);
    }

    // ---- Gibbs half-step 1: t0 by Metropolis-Hastings
    const double t0p = t0 + md.t0_sd * xi_t0;
    bool t0acc = false;
    if (lane == 0) cnt[0]++;
    fsmp_logrec rec{};
    if (FORCE) {
      rec = a.force[c * (int64_t)a.n_steps + step];
      t0acc = (rec.flags & 4) != 0;
      if (rec.t0 != t0) {
        t0 = rec.t0;
        Phi = (glo <= ghi) ? phi_total_group<LPC>(md, t0, glo, ghi, lane, gbase) : 0.0;
        Lam = lam * md.dt * Phi;
        if (biexp) {
          double sn = 0.0;
          for (int i = lane; i < N; i += LPC) sn += rise_term(md, zg[i], t0);
          S_cur = group_sum<LPC>(sn);
        }
      }
    } else if (t0p >= md.t0_min && t0p <= md.t0_max) {
      const double xmin = (N > 0) ? (double)gmin * md.dt - t0p : 1.0;
      if (biexp ? (xmin > 0.0) : (xmin >= 0.0)) {
        double S_new = 0.0;
        if (biexp) {
          // the rise factors of a lane's PEs multiplied in runs of up to eight, one log per run
          double pr = 1.0;
          int m = 0;
          for (int i = lane; i < N; i += LPC) {
            pr *= rise_factor(md, zg[i], t0p);
            if (++m == 8) {
              S_new += log(pr);
              pr = 1.0;
              m = 0;
            }
          }
          S_new += log(pr);
          S_new = group_sum<LPC>(S_new);
        }
        const double part = (double)N * (t0p - t0) * md.inv_tau2 + (S_new - S_cur);
        const double Phip = (glo <= ghi) ? phi_total_group<LPC>(md, t0p, glo, ghi, lane, gbase) : 0.0;
        const double la0 = part - (lam * md.dt * Phip - lam * md.dt * Phi);
        if (lg2 < la0) {
          t0 = t0p;
          Phi = Phip;
          Lam = lam * md.dt * Phi;
          S_cur = S_new;
          t0acc = true;
          if (lane == 0) cnt[1]++;
        }
      }
    }

    // ---- Gibbs half-step 2: one RJMCMC jump
    const double um = u01(r[3]);
    const int move = FORCE ? rec.move : ((N == 0 || um < md.J) ? 1 : (um < 2.0 * md.J ? 2 : 3));
    // replay: only the recorded valid proposals are evaluated, and only well-formed ones
    const bool consider =
        !FORCE || ((rec.flags & 1) && (move == 1 ? (rec.g >= glo && rec.g <= ghi)
                                                 : (move == 2 || move == 3) && rec.j >= 0 && rec.j < N));
    // A wavefront carries several chains whose moves differ; the expensive parts are
    // written once so that it executes them once: the proposal evaluation shared by
    // births and time shifts, and one rank-two edit for every accepted move.
    int j = -1, gnew = -1, sh = 0;
    // need_mv: a birth part (births, shifts); need_dp: in the FP32 form, a death part
    // (deaths, shifts) evaluated with the residual correction
    bool valid = false, need_mv = false, need_dp = false;
    double dnu = 0.0, la = -INFINITY, lpn = 0.0, lpo = 0.0;
    // xjp: x_j as stored (the corrected FP64 form evaluates with xj = x_j + h^T s and edits x
    // with the stored value, which keeps x = H b along the edits)
    double delta2 = 1.0, up = 0.0, om = 1.0, xj = 0.0, xjp = 0.0, ej = 0.0, beta = 0.0;
    // mixture form: the component of a born or updated PE from word r7 (inverse CDF of the
    // weights); rho, its log, rho mu, rho mu^2 of the new and of the removed / moved PE
    int enew = 0;
    double rn = md.rho, lrn = md.log_rho, rmn = md.rhom, rm2n = md.rhom2;
    double lro = md.log_rho, rm2o = md.rhom2;
    if constexpr (MCP) {
      const double ue = u01(r[7]);
      enew = md.n_mix - 1;
      for (int q = md.n_mix - 2; q >= 0; --q)
        if (ue < md.mix_cdf[q]) enew = q;
      rn = md.mix_rho[enew];
      lrn = md.mix_lrho[enew];
      rmn = md.mix_rhom[enew];
      rm2n = md.mix_rhom2[enew];
    }
    if (move == 1) {
      if (lane == 0) cnt[2]++;
      if (N >= kmax) {
        st |= FSMP_ST_KMAX;
      } else if (Phi > 0.0 && consider) {
        gnew = FORCE ? rec.g : birth_draw<LPC>(md, t0, glo, ghi, u53(r[4], r[5]) * Phi, lane, grp);
        need_mv = Lam > 0.0;
      }
    } else {
      j = FORCE ? rec.j : (int)(((uint64_t)r[4] * (uint64_t)N) >> 32);
      if (!consider) {
        j = -1;  // replay: not a recorded valid proposal
      } else if (move == 2) {
        if (lane == 0) cnt[4]++;
        if constexpr (F32) {
          need_dp = true;
        } else {
          om = H[(j * LD + j) * HS];
          xj = xjp = xv[j];
          if constexpr (CORR) {
            double xc = 0.0;
            for (int i = lane; i < N; i += LPC) xc += H[(j * LD + i) * HS] * rs[i];
            xj += group_sum<LPC>(xc);
          }
          if constexpr (MCP) {
            lro = md.mix_lrho[ek[j]];
            rm2o = md.mix_rhom2[ek[j]];
          }
          if (om > 0.0) {
            double lom, lLam;
            group_log2<LPC>(om, Lam, lane, gbase, lom, lLam);
            dnu = 0.5 * (-lro - lom + (rm2o - xj * xj / om) * md.inv_s);
            la = dnu - lLam + lgn[N] - (N == 1 ? md.logJ : 0.0);
            valid = true;
          } else {
            st |= FSMP_ST_FACTOR;
          }
        }
      } else {
        if (lane == 0) cnt[6]++;
        sh = FORCE ? rec.g - zg[j] : (int)rint(xi_sh * md.shift_sd / md.dt);
        gnew = zg[j] + sh;
        if (gnew >= glo && gnew <= ghi) {
          // log phi at the new and at the old position, one evaluation for both
          const double lv = log_phi(md, (double)(lane == 0 ? gnew : zg[j]) * md.dt - t0);
          lpn = group_bcast<LPC, 0>(lv, gbase);
          const double lpo_v = group_bcast<LPC, 1>(lv, gbase);
          if (lpn > -INFINITY) {
            lpo = lpo_v;
            if constexpr (MCP) {
              lro = md.mix_lrho[ek[j]];
              rm2o = md.mix_rhom2[ek[j]];
            }
            if (sh == 0 && (!MCP || enew == ek[j])) {
              valid = true;
              dnu = 0.0;
              la = lpn - lpo;
            } else {
              need_mv = true;
              need_dp = F32;
            }
          }
        }
      }
    }
    // birth or time shift: gamma = overlaps of the new position with the PEs (zero at the
    // shifted one), eta = M gamma, q = gamma^T eta, p = gamma^T x, for M = H or (precision
    // form, near the threshold) its FP64 rebuild W
    auto eval_mv = [&](auto *M) {
      valid = false;
      const int jz = move == 3 ? j : -1;
      for (int i = lane; i < N; i += LPC) s1[i] = (i == jz) ? 0.0 : overlap(md, vt, ov, gnew, zg[i], Lw);
      const double d = overlap(md, vt, ov, gnew, gnew, Lw) + rn;
      beta = mf[gnew - glo] + rmn;
      WAVE_SYNC();
      double q = 0.0, p = 0.0, pc = 0.0, xc = 0.0;
      for (int i = lane; i < N; i += LPC) {
        const double e = grp_col_dot<LD, HS>(M, s1, i, N);
        s2[i] = e;
        q += s1[i] * e;
        p += s1[i] * xv[i];
        if constexpr (CORR) {
          pc += e * rs[i];
          if (move == 3) xc += (double)M[(j * LD + i) * HS] * rs[i];
        }
      }
      q = group_sum<LPC>(q);
      p = group_sum<LPC>(p);
      if constexpr (CORR) {
        p += group_sum<LPC>(pc);
        if (move == 3) xc = group_sum<LPC>(xc);
      }
      if (move == 1) {
        delta2 = d - q;
        if (delta2 > 0.0) {
          up = beta - p;
          double ld2, lLam;
          group_log2<LPC>(delta2, Lam, lane, gbase, ld2, lLam);
          dnu = -0.5 * (-lrn + ld2 + (rm2n - up * up / delta2) * md.inv_s);
          la = dnu + lLam - lgn[N + 1] + (N == 0 ? md.logJ : 0.0);
          valid = true;
        } else {
          st |= FSMP_ST_FACTOR;
        }
      } else {
        WAVE_SYNC();
        om = (double)M[(j * LD + j) * HS];
        xj = xjp = xv[j];
        if constexpr (CORR) xj += xc;
        ej = s2[j];
        delta2 = d - (q - ej * ej / om);
        up = beta - (p - ej * xj / om);
        if (delta2 > 0.0 && om > 0.0) {
          double lom, ld2;
          group_log2<LPC>(om, delta2, lane, gbase, lom, ld2);
          dnu = 0.5 * (-lom - ld2 + (up * up / delta2 - xj * xj / om) * md.inv_s);
          // mixture form: the removed and the added PE carry their own rho and rho mu^2
          if constexpr (MCP) dnu += 0.5 * (lrn - lro + (rm2o - rm2n) * md.inv_s);
          la = dnu + lpn - lpo;
          valid = true;
        } else {
          st |= FSMP_ST_FACTOR;
        }
      }
    };
    // The FP32 form evaluates a proposal from its FP32 H with a two-term correction against
    // the exact G (FP64 in device memory, kept with the list).  For a vector f and its
    // approximate solve a = H f, the residual r = f - G a and the correction H r, the bilinear
    // form f'^T G^-1 f is f'^T a + a^T r' + r^T H r' to second order in the error of H (the
    // first term of the correction cancels the first-order error exactly; the last term is
    // the size of what is corrected at second order, taken as the bound of what is left, as
    // the error contracts by |I - H G| per term).  The vectors are gamma (the new position's
    // overlaps, 0 at j for a shift: births and shifts), e_j (deaths and shifts) and b:
    //   Qgg = gamma^T G^-1 gamma, Qjg = e_j^T G^-1 gamma, omega = (G^-1)_jj,
    //   Pg = gamma^T G^-1 b, xj = e_j^T G^-1 b,
    // from one pass over H (eta = H gamma, h = row j), one over G (r_eta, r_h, s = b - G x)
    // and one over H again (H r_eta, H r_h).  A shift's birth part is on the PEs without j, by
    // the identities (G without j)^-1 = (G^-1 - u u^T / omega) there, u = G^-1 e_j:
    //   delta^2 = d - (Qgg - Qjg^2 / omega),  u+ = beta - (Pg - Qjg xj / omega),
    // with each bound carried through them.  bnd is the bound of delta-nu to first order, times
    // four.  Vectors left for the edit: u = h + H r_h in s1, eta + H r_eta (for a shift minus
    // u Qjg / omega, 0 at j) in s3.
    double bnd = 0.0;
    bool inexact = false;
    auto f32_dnu = [&](double Bom, double Bxj, double Bq, double Bp) {
      const double s = md.s;
      if (move == 1) {
        double ld2, lLam;
        group_log2<LPC>(delta2, Lam, lane, gbase, ld2, lLam);
        dnu = -0.5 * (-md.log_rho + ld2 + (md.rhom2 - up * up / delta2) * md.inv_s);
        la = dnu + lLam - lgn[N + 1] + (N == 0 ? md.logJ : 0.0);
      } else if (move == 2) {
        double lom, lLam;
        group_log2<LPC>(om, Lam, lane, gbase, lom, lLam);
        dnu = 0.5 * (-md.log_rho - lom + (md.rhom2 - xj * xj / om) * md.inv_s);
        la = dnu - lLam + lgn[N] - (N == 1 ? md.logJ : 0.0);
      } else {
        double lom, ld2;
        group_log2<LPC>(om, delta2, lane, gbase, lom, ld2);
        dnu = 0.5 * (-lom - ld2 + (up * up / delta2 - xj * xj / om) * md.inv_s);
        la = dnu + lpn - lpo;
      }
      double b = 0.0;
      if (move != 2) b += 0.5 * fabs(1.0 / delta2 + up * up / (delta2 * delta2 * s)) * Bq + fabs(up) / (delta2 * s) * Bp;
      if (move != 1) b += 0.5 * fabs(1.0 / om - xj * xj / (om * om * s)) * Bom + fabs(xj) / (om * s) * Bxj;
      bnd = 4.0 * b;
      valid = true;
    };
    auto f32_eval = [&]() {
      valid = false;
      const bool wg = need_mv, wj = need_dp;  // gamma (births, shifts), e_j (deaths, shifts)
      const int jz = move == 3 ? j : -1;
      double d = 0.0;
      if (wg) {
        for (int i = lane; i < N; i += LPC) s2[i] = (i == jz) ? 0.0 : overlap(md, vt, ov, gnew, zg[i], Lw);
        d = overlap(md, vt, ov, gnew, gnew, Lw) + md.rho;
        beta = mf[gnew - glo] + md.rhom;
      }
      WAVE_SYNC();
      // pass 1 over H: eta = H gamma, h = row j; gamma^T eta, gamma^T x
      double qa = 0.0, pa = 0.0;
      for (int i = lane; i < N; i += LPC) {
        if (wg) {
          const double e = grp_col_dot<LD, HS>(H, s2, i, N);
          s3[i] = e;
          qa += s2[i] * e;
          pa += s2[i] * xv[i];
        }
        if (wj) s1[i] = (double)H[(j * LD + i) * HS];
      }
      if (wg) {
        qa = group_sum<LPC>(qa);
        pa = group_sum<LPC>(pa);
      }
      WAVE_SYNC();
      // the residuals against G: r_eta = gamma - G eta (s5), r_h = e_j - G h (s4), s = b - G x (s6)
      gram_resid3<LPC, LD, HS>(Gm, N, lane, s2, wg ? s3 : nullptr, j, wj ? s1 : nullptr, bv, xv, s5, s4, s6);
      WAVE_SYNC();
      double eta_j = 0.0, h_j = 0.0, x_j = 0.0;
      if (wj) {
        eta_j = wg ? s3[j] : 0.0;
        h_j = s1[j];
        x_j = xv[j];
      }
      // first correction terms
      double qb = 0.0, pb = 0.0, jb = 0.0, ob = 0.0, xb = 0.0;
      for (int i = lane; i < N; i += LPC) {
        if (wg) {
          qb += s3[i] * s5[i];
          pb += s3[i] * s6[i];
        }
        if (wj) {
          if (wg) jb += s1[i] * s5[i];
          ob += s1[i] * s4[i];
          xb += s1[i] * s6[i];
        }
      }
      if (wg) {
        qb = group_sum<LPC>(qb);
        pb = group_sum<LPC>(pb);
      }
      if (wj) {
        if (wg) jb = group_sum<LPC>(jb);
        ob = group_sum<LPC>(ob);
        xb = group_sum<LPC>(xb);
      }
      // pass 2 over H: H r_eta, H r_h; the second terms, then eta and h corrected in place
      double qc = 0.0, pc = 0.0, jc = 0.0, oc = 0.0, xc = 0.0;
      for (int i = lane; i < N; i += LPC) {
        double te = 0.0, th = 0.0;
        if (wg) {
          te = grp_col_dot<LD, HS>(H, s5, i, N);
          qc += s5[i] * te;
          pc += te * s6[i];
        }
        if (wj) {
          th = grp_col_dot<LD, HS>(H, s4, i, N);
          if (wg) jc += s4[i] * te;
          oc += s4[i] * th;
          xc += th * s6[i];
        }
        if (wg) s3[i] += te;
        if (wj) s1[i] += th;
      }
      double Qgg = 0.0, Pg = 0.0, Qjg = 0.0, Bgg = 0.0, Bp = 0.0, Bjg = 0.0, Bom = 0.0, Bxj = 0.0;
      if (wg) {
        qc = group_sum<LPC>(qc);
        pc = group_sum<LPC>(pc);
        Qgg = qa + qb + qc;
        Pg = pa + pb + pc;
        Bgg = fabs(qc);
        Bp = fabs(pc);
      }
      if (wj) {
        if (wg) jc = group_sum<LPC>(jc);
        oc = group_sum<LPC>(oc);
        xc = group_sum<LPC>(xc);
        om = h_j + ob + oc;
        xj = x_j + xb + xc;
        Qjg = eta_j + jb + jc;
        Bom = fabs(oc);
        Bxj = fabs(xc);
        Bjg = fabs(jc);
        if (!(om > 0.0) || !(Bom < 0.1 * om)) {
          inexact = true;
          return;
        }
      }
      WAVE_SYNC();
      double Bq = Bgg;
      if (move == 1) {
        delta2 = d - Qgg;
        up = beta - Pg;
      } else if (move == 3) {
        const double cj = Qjg / om, cx = xj / om;
        delta2 = d - (Qgg - Qjg * cj);
        up = beta - (Pg - Qjg * cx);
        Bq = Bgg + 2.0 * fabs(cj) * Bjg + cj * cj * Bom;
        Bp = Bp + fabs(cx) * Bjg + fabs(cj) * Bxj + fabs(cj * cx) * Bom;
        // v = eta - u Qjg / omega on the PEs without j
        for (int i = lane; i < N; i += LPC) s3[i] = (i == j) ? 0.0 : s3[i] - s1[i] * cj;
        WAVE_SYNC();
      }
      if (move != 2 && (!(delta2 > 0.0) || !(Bq < 0.1 * delta2))) {
        inexact = true;
        return;
      }
      f32_dnu(Bom, Bxj, Bq, Bp);
    };
    // the same proposal from the FP64 rebuild W (exact to FP64 rounding), vectors as above
    auto f64_eval_W = [&]() {
      valid = false;
      if (need_dp) {
        for (int i = lane; i < N; i += LPC) s1[i] = W[(j * LD + i) * HS];
        WAVE_SYNC();
        om = s1[j];
        xj = xv[j];
      }
      if (need_mv) {
        const int jz = move == 3 ? j : -1;
        for (int i = lane; i < N; i += LPC) s2[i] = (i == jz) ? 0.0 : overlap(md, vt, ov, gnew, zg[i], Lw);
        const double d = overlap(md, vt, ov, gnew, gnew, Lw) + md.rho;
        beta = mf[gnew - glo] + md.rhom;
        WAVE_SYNC();
        double q = 0.0, p = 0.0;
        for (int i = lane; i < N; i += LPC) {
          const double e = grp_col_dot<LD, HS>(W, s2, i, N);
          s3[i] = e;
          q += s2[i] * e;
          p += s2[i] * xv[i];
        }
        q = group_sum<LPC>(q);
        p = group_sum<LPC>(p);
        if (move == 3) {
          WAVE_SYNC();
          const double e = s3[j];
          q -= e * e / om;
          p -= e * xj / om;
          WAVE_SYNC();
          for (int i = lane; i < N; i += LPC) s3[i] = (i == j) ? 0.0 : s3[i] - s1[i] * e / om;
          WAVE_SYNC();
        }
        delta2 = d - q;
        up = beta - p;
      }
      if ((move != 1 && !(om > 0.0)) || (move != 2 && !(delta2 > 0.0))) {
        st |= FSMP_ST_FACTOR;
        return;
      }
      f32_dnu(0.0, 0.0, 0.0, 0.0);
      bnd = 0.0;
    };

    const double logu = lg6;
    if constexpr (F32) {
      if (need_mv || need_dp) {
        f32_eval();
        // an estimate above the tolerance, or a decision the error could turn: decide with
        // the FP64 rebuild
        if (inexact || (valid && (bnd > kF32Tol * fmax(1.0, fabs(dnu)) || fabs(logu - la) <= bnd))) {
          double drift;
          if (N == 0 || grp_refresh<LPC, LD, HS>(md, vt, ov, Lw, W, H, xv, bv, s1, s2, zg, N, lane, drift)) {
            f64_eval_W();
          } else {
            valid = false;
            st |= FSMP_ST_FACTOR;
          }
          if (lane == 0) acc[19] += 1.0;
        } else if (!valid) {
          st |= FSMP_ST_FACTOR;
        }
        if (lane == 0) acc[17] += (double)N * N * (need_dp ? 1.0 : 0.0) + (double)N * N * (need_mv ? 2.0 : 0.0) +
                                  (need_dp ? (double)N : 0.0);
      }
    } else if (need_mv) {
      // (the corrected form also reads row j of H for a shift's x_j)
      if (lane == 0) acc[17] += (double)N * N + (CORR && move == 3 ? (double)N : 0.0);
      eval_mv(H);
    } else if (move == 2 && valid && lane == 0) {
      acc[17] += CORR ? (double)N : 1.0;
    }
    // the word count of the proposal in a packed Cholesky factor: birth K(K+1)/2 +
    // 2K + 3, death (K - j)(K - j + 1)/2 + 1, update both (the birth on K - 1 PEs)
    if (lane == 0 && (valid || need_mv || need_dp)) {
      const double K = N, r = N - j;
      const double wb = move == 1 ? K * (K + 1) / 2 + 2 * K + 3 : (K - 1) * K / 2 + 2 * (K - 1) + 3;
      const double wd = r * (r + 1) / 2 + 1;
      acc[15] += move == 1 ? wb : move == 2 ? wd : (need_mv ? wd + wb : 0.0);
    }

    bool accepted = false;
    if (valid && (FORCE ? (rec.flags & 2) != 0 : logu < la)) {
      accepted = true;
      if (lane == 0) cnt[2 * move + 1]++;
      WAVE_SYNC();
      // an accepted zero shift changes nothing (unless it changes the PE's component)
      const bool shift = move == 3 && (sh != 0 || (MCP && enew != ek[j]));
      if (lane == 0) {
        // the word count of the edit in a packed Cholesky factor: birth K + 3, death
        // (K - 1 - j)(K - j) + K(K + 1)/2, update both; and the G^-1 elements this kernel reads
        // and writes in its rank-one or rank-two edit
        const double K = N, r = N - j;
        const double eb = move == 1 ? K + 3 : (K - 1) + 3, ed = (r - 1) * r + K * (K + 1) / 2;
        acc[16] += move == 1 ? eb : move == 2 ? ed : (shift ? ed + eb : 0.0);
        if (move != 3 || shift) acc[18] += 2.0 * K * K;
      }
      if (move != 3 || shift) {
        const double inv_d2 = move == 2 ? 0.0 : 1.0 / delta2;
        const double inv_om = move == 1 ? 0.0 : 1.0 / om;
        const double xn = up * inv_d2;
        const int gj = move == 1 ? -1 : zg[j];
        // the FP32 form has its corrected vectors at hand: u (column j of G^-1) in s1, eta or v
        // in s3
        if constexpr (!F32) {
          if (move != 1) {
            for (int i = lane; i < N; i += LPC) s1[i] = H[(j * LD + i) * HS];  // h = row j of H
            WAVE_SYNC();
          }
          if (shift) {
            for (int i = lane; i < N; i += LPC) s2[i] = (i == j) ? 0.0 : s2[i] - s1[i] * ej * inv_om;
            WAVE_SYNC();
          }
        }
        double *EV = F32 ? s3 : s2;  // eta (birth) or v (shift)
        // H(k, i) += cu u_i u_k + cv v_i v_k for i, k < N:
        //   birth: u = eta, cu = 1/delta^2; death: u = h, cu = -1/omega;
        //   shift: u = h, cu = -1/omega, and v = eta (zero at j), cv = 1/delta^2
        const double *U = move == 1 ? EV : s1;
        const double *V = shift ? EV : U;
        const double cu = move == 1 ? inv_d2 : -inv_om, cv = shift ? inv_d2 : 0.0;
        const double xe = CORR ? xjp : xj;
        for (int i = lane; i < N; i += LPC) {
          const double ui = U[i], vi = V[i];
          if (move == 1) xv[i] -= ui * xn;
          else if (move == 2) xv[i] -= ui * xe * inv_om;
          else xv[i] = (i == j) ? xn : xv[i] - ui * xe * inv_om - vi * xn;
          grp_col_update<LD, HS, true>(H, i, N, ui, U, cu, vi, V, cv);
          if (move == 1) {
            H[(N * LD + i) * HS] = -ui * inv_d2;
            H[(i * LD + N) * HS] = -ui * inv_d2;
          }
        }
        WAVE_SYNC();
        // the exact G follows the list: the new PE's row and column, or the last PE's moved
        // into a freed slot (s2 is free once the edit is done)
        if constexpr (KEEPG) {
          if (move == 1) {
            gram_set<LPC, LD, HS>(md, vt, ov, Lw, Gm, zg, N, N, gnew, rn, lane);
          } else if (move == 3) {
            gram_set<LPC, LD, HS>(md, vt, ov, Lw, Gm, zg, N, j, gnew, rn, lane);
          } else if (j != N - 1) {
            const int last = N - 1;
            for (int i = lane; i < N; i += LPC) s2[i] = Gm[(last * LD + i) * HS];
            WAVE_SYNC();
            const double gd = s2[last];
            for (int i = lane; i < N; i += LPC) {
              if (i == j) {
                Gm[(j * LD + j) * HS] = gd;
              } else {
                Gm[(j * LD + i) * HS] = s2[i];
                Gm[(i * LD + j) * HS] = s2[i];
              }
            }
          }
        }
        if (move == 1) {
          if (lane == 0) {
            H[(N * LD + N) * HS] = inv_d2;
            zg[N] = gnew;
            if constexpr (MCP) ek[N] = enew;
            xv[N] = xn;
            if (KEEPG) bv[N] = beta;
          }
          N++;
          if (biexp) S_cur += rise_term(md, gnew, t0);
          gmin = gnew < gmin ? gnew : gmin;
        } else if (move == 2) {
          const int last = N - 1;
          if (j != last) {
            for (int i = lane; i < N; i += LPC) s1[i] = H[(last * LD + i) * HS];
            WAVE_SYNC();
            const double vd = s1[last];
            for (int i = lane; i < N; i += LPC) {
              if (i == j) {
                H[(j * LD + j) * HS] = vd;
              } else {
                H[(j * LD + i) * HS] = s1[i];
                H[(i * LD + j) * HS] = s1[i];
              }
            }
            if (lane == 0) {
              zg[j] = zg[last];
              if constexpr (MCP) ek[j] = ek[last];
              xv[j] = xv[last];
              if (KEEPG) bv[j] = bv[last];
            }
          }
          N--;
          if (biexp) S_cur -= rise_term(md, gj, t0);
        } else {
          for (int i = lane; i < N; i += LPC) {
            if (i == j) {
              H[(j * LD + j) * HS] = inv_d2;
            } else {
              const double v = -EV[i] * inv_d2;
              H[(j * LD + i) * HS] = v;
              H[(i * LD + j) * HS] = v;
            }
          }
          if (lane == 0) {
            zg[j] = gnew;
            if constexpr (MCP) ek[j] = enew;
            if (KEEPG) bv[j] = beta;
          }
          if (biexp) S_cur += rise_term(md, gnew, t0) - rise_term(md, gj, t0);
        }
        WAVE_SYNC();
        // the corrected FP64 form: the residual of the new x against the new G
        if constexpr (CORR) {
          gram_resid_b<LPC, LD, HS>(Gm, bv, xv, rs, N, lane);
          if (lane == 0) acc[18] += (double)N * N;
          WAVE_SYNC();
        }
        if (move != 1) {
          if (move == 3 && gnew < gmin) {
            gmin = gnew;
          } else if (gj == gmin) {
            int m = INT32_MAX;
            for (int i = lane; i < N; i += LPC) m = zg[i] < m ? zg[i] : m;
            gmin = group_min<LPC>(m);
          }
        }
        if (lane == 0) occ_edit(a, c, move, gj, gnew, step, burn, n_steps);
      }
    }

    if (a.log && lane == 0) {
      fsmp_logrec *lr = a.log + c * (int64_t)a.n_steps + step;
      lr->move = move;
      lr->flags = (valid ? 1 : 0) | (accepted ? 2 : 0) | (t0acc ? 4 : 0);
      lr->j = j;
      lr->g = gnew;
      lr->t0 = t0;
      lr->dnu = valid ? dnu : 0.0;
      lr->log_alpha = valid ? la : -INFINITY;
    }
    if (FORCE && lane == 0) {
      a.rdnu[c * (int64_t)a.n_steps + step] = valid ? dnu : 0.0;
      a.rla[c * (int64_t)a.n_steps + step] = valid ? la : -INFINITY;
    }

    // ---- record after burn-in
    if (step >= burn) {
      double Q = 0.0;
      for (int i = lane; i < N; i += LPC) Q += xv[i];
      Q = group_sum<LPC>(Q);
      const double v0 = (double)N, v1 = Q, v2 = t0;
      const int64_t i = step - burn;
      if (lane == 0) {
        acc[0] += v0;
        acc[1] += v0 * v0;
        acc[2] += v1;
        acc[3] += v1 * v1;
        acc[4] += v2;
        acc[5] += v2 * v2;
        if (nb > 0 && i < (int64_t)nb * lb) {
          acc[12] += v0;
          acc[13] += v1;
          acc[14] += v2;
          if ((i + 1) % lb == 0) {
            acc[6] += acc[12];
            acc[7] += acc[12] * acc[12];
            acc[8] += acc[13];
            acc[9] += acc[13] * acc[13];
            acc[10] += acc[14];
            acc[11] += acc[14] * acc[14];
            acc[12] = acc[13] = acc[14] = 0.0;
          }
        }
        if (N != run[0]) {
          if (run[0] >= 0) atomicAdd(a.nhist + c * (a.kz + 1) + run[0], step - run[1]);
          run[0] = N;
          run[1] = step;
        }
      }
      if (a.trace && a.thin > 0 && (i % a.thin) == 0 && lane == 0) {
        double *tr = a.trace + (c * a.n_rec + i / a.thin) * 3;
        tr[0] = v0;
        tr[1] = v2;
        tr[2] = v1;
      }
      if (a.qdraw && a.thin > 0 && (i % a.thin) == 0) {
        // charge draw q = x + sigma_eps R xi, H = R R^T with R upper triangular: the
        // factorisation runs from the last PE backwards on a copy of H's lower triangle
        // in the chain's device-memory scratch; y = R xi accumulates column by column.  The
        // FP32 form draws from its FP64 rebuild W (and the x it recomputes).
        const int64_t rec = c * a.n_rec + i / a.thin;
        double *Ad = a.dscr + slot * (int64_t)(KCAP * KCAP + KCAP);
        double *Av = Ad + KCAP * KCAP;  // the column being eliminated
        WAVE_SYNC();
        bool ok = true;
        if constexpr (F32) {
          double drift;
          if (N > 0 && !grp_refresh<LPC, LD, HS>(md, vt, ov, Lw, W, H, xv, bv, s1, s2, zg, N, lane, drift)) ok = false;
        }
        for (int r = lane; r < N; r += LPC) {
          for (int k = 0; k <= r; ++k) {
            if constexpr (F32) Ad[r * KCAP + k] = W[(k * LD + r) * HS];
            else Ad[r * KCAP + k] = H[(k * LD + r) * HS];
          }
          s1[r] = charge_normal(step, r, uid0, uid1, a.key0, a.key1);
          s2[r] = 0.0;
        }
        WAVE_SYNC();
        for (int jj = N - 1; jj >= 0 && ok; --jj) {
          const double ajj = Ad[jj * KCAP + jj];
          if (!(ajj > 0.0)) {
            ok = false;
            break;
          }
          const double d = sqrt(ajj), xij = s1[jj];
          for (int r = lane; r < jj; r += LPC) {
            const double v = Ad[jj * KCAP + r] / d;
            Av[r] = v;
            s2[r] += v * xij;
          }
          if (lane == 0) s2[jj] += d * xij;
          WAVE_SYNC();
          for (int r = lane; r < jj; r += LPC) {
            const double vr = Av[r];
            for (int k = 0; k <= r; ++k) Ad[r * KCAP + k] -= vr * Av[k];
          }
          WAVE_SYNC();
        }
        if (!ok) st |= FSMP_ST_FACTOR;
        for (int r = lane; r < a.kz; r += LPC) {
          a.zdraw[rec * a.kz + r] = r < N ? zg[r] : -1;
          a.qdraw[rec * a.kz + r] = r < N ? (ok ? xv[r] + a.sigma_eps * s2[r] : NAN) : 0.0;
        }
        WAVE_SYNC();
      }
    }
  }

  WAVE_SYNC();
  const int kz = a.kz;
  for (int k = lane; k < kz; k += LPC) {
    a.z[c * kz + k] = k < N ? zg[k] : -1;
    a.charge[c * kz + k] = k < N ? xv[k] : 0.0;
    if (MCP && a.comp) a.comp[c * kz + k] = k < N ? ek[k] : -1;
  }
  if (lane == 0 && run[0] >= 0) atomicAdd(a.nhist + c * (a.kz + 1) + run[0], n_steps - run[1]);
  if (lane == 0) {
    a.n_pe[c] = N;
    a.t0[c] = t0;
    if (a.rec_steps) a.rec_steps[c] = S_rec;
    for (int i = 0; i < 12; ++i) a.acc[c * 12 + i] = acc[i];
    for (int i = 0; i < 8; ++i) a.counts[c * 8 + i] = cnt[i];
    a.status[c] = st;
    if (a.work) {
      for (int i = 0; i < 5; ++i) a.work[c * 5 + i] = acc[15 + i];
    }
  }
}


// ------------------------------------------------------------------ chains, one lane each
// birth position for one lane: EXP by the closed-form inverse, BIEXP by bisection on the
// closed-form partial sums (same rule as birth_draw: smallest g with F(g) > target)
__device__ inline int birth_draw_lane(const ModelDev &md, double t0, int glo, int ghi, double target) {
  const GridPos p = grid_pos(md, t0, glo, ghi);
  const XsExp xe = xs_exp(md, p.xs);
  int64_t k;
  if (md.kind == FSMP_PHI_EXP) {
    const double c = target * exp(p.xs * md.inv_tau2) * md.den2 / md.inv_tau2;
    if (c >= 1.0) {
      k = p.n - 1;
    } else {
      const double L = -log1p(-c) / (md.dt * md.inv_tau2);
      k = (int64_t)floor(L);
      if (k < 0) k = 0;
      if (k > p.n - 1) k = p.n - 1;
      if (k > 0 && phi_partial(md, xe, k) > target) k -= 1;
      else if (k < p.n - 1 && !(phi_partial(md, xe, k + 1) > target)) k += 1;
    }
  } else {
    // bisection: the same number of steps in every lane (a Newton inverse with per-lane
    // iteration counts measured slower on the GPU)
    int64_t lo = 0, hi = p.n - 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (phi_partial(md, xe, mid + 1) > target) hi = mid;
      else lo = mid + 1;
    }
    k = lo;
  }
  return (int)(p.gs + k);
}


// Interleaved per-lane state helpers: element e of this lane's chain is p[e * 64].
// Every loop below issues a chunk of independent loads before any store, so one
// memory round trip covers kChunk elements.  Matrices are read into FP64 whatever
// their storage type (FP64, or FP32 in the precision form) and written back rounded.
constexpr int kChunk = 8;

// eta = M gamma over the first n rows; q = gamma^T eta and, when X is given,
// p = gamma^T x, both summed in row order.  Rows go in blocks of 4 and columns in
// chunks of 4: the 20 loads of a chunk are issued unconditionally (indices stay below
// KCAP, a multiple of 4) and the columns past n are dropped by a select, so a chunk
// costs one memory round trip; each row still sums its terms in column order.
template <int KCAP, typename MT>
__device__ inline void lane_matvec(const MT *Mp, const double *G, double *E, const double *X, int n, double &q,
                                   double &p) {
  static_assert(KCAP % 8 == 0, "capacity must be a multiple of 8");
  q = 0.0;
  p = 0.0;
  for (int i0 = 0; i0 < n; i0 += 4) {
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 4) {
      double g[4], h[4][4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        g[kk] = G[(k0 + kk) * 64];
#pragma unroll
        for (int u = 0; u < 4; ++u) h[kk][u] = (double)Mp[((k0 + kk) * KCAP + i0 + u) * 64];
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = (k0 + kk < n) ? e[u] + h[kk][u] * g[kk] : e[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u < n) {
        E[(i0 + u) * 64] = e[u];
        const double gi = G[(i0 + u) * 64];
        q += gi * e[u];
        if (X) p += gi * X[(i0 + u) * 64];
      }
  }
}

// M(k, i) += (A_i A_k) cA [+ (B_i B_k) cB] for i, k < n.  Loads of a chunk of 8 columns
// are unconditional (below KCAP), stores are guarded.
template <int KCAP, bool TWO, typename MT>
__device__ inline void lane_rank_update(MT *Mp, const double *A, double cA, const double *B, double cB, int n) {
  for (int k = 0; k < n; ++k) {
    const double ak = A[k * 64];
    const double bk = TWO ? B[k * 64] : 0.0;
    for (int i0 = 0; i0 < n; i0 += kChunk) {
      double h[kChunk], av[kChunk], bv[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        h[u] = (double)Mp[(k * KCAP + i0 + u) * 64];
        av[u] = A[(i0 + u) * 64];
        if (TWO) bv[u] = B[(i0 + u) * 64];
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        double v = h[u] + av[u] * ak * cA;
        if (TWO) v += bv[u] * bk * cB;
        if (i0 + u < n) Mp[(k * KCAP + i0 + u) * 64] = (MT)v;
      }
    }
  }
}

// n elements src[e * 64] -> dst[e * 64] (chunked, loads unconditional below the
// capacity of both rows), converting the type
template <typename DT, typename ST>
__device__ inline void lane_copy(DT *dst, const ST *src, int n) {
  for (int i0 = 0; i0 < n; i0 += kChunk) {
    double v[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) v[u] = (double)src[(i0 + u) * 64];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (i0 + u < n) dst[(i0 + u) * 64] = (DT)v[u];
  }
}

// Charge draw of one lane's chain (q = x + sigma_eps R xi, H = R R^T, R upper
// triangular): the same backward factorisation as the lane-group kernels on a copy of
// H's lower triangle in the interleaved scratch Ap, y = R xi accumulated in S2.  Not
// inlined: it runs only at recorded steps and stays out of the sweep's registers.
template <int KCAP, typename HT>
__device__ __attribute__((noinline)) bool lane_charge_draw(double *Ap, const HT *Hp, const double *Xp, double *S1,
                                                           double *S2, double *S3, const int32_t *Zp, int N, int step,
                                                           uint32_t uid0, uint32_t uid1, uint32_t key0, uint32_t key1,
                                                           double sig, double *q, int32_t *zq, int kz) {
  for (int r = 0; r < N; ++r) {
    for (int k = 0; k <= r; ++k) Ap[(r * KCAP + k) * 64] = (double)Hp[(k * KCAP + r) * 64];
    S1[r * 64] = charge_normal(step, r, uid0, uid1, key0, key1);
    S2[r * 64] = 0.0;
  }
  bool ok = true;
  for (int jj = N - 1; jj >= 0; --jj) {
    const double ajj = Ap[(jj * KCAP + jj) * 64];
    if (!(ajj > 0.0)) {
      ok = false;
      break;
    }
    const double d = sqrt(ajj), xij = S1[jj * 64];
    for (int r = 0; r < jj; ++r) {
      const double v = Ap[(jj * KCAP + r) * 64] / d;
      S3[r * 64] = v;
      S2[r * 64] += v * xij;
    }
    S2[jj * 64] += d * xij;
    for (int r = 0; r < jj; ++r) {
      const double vr = S3[r * 64];
      for (int k = 0; k <= r; ++k) Ap[(r * KCAP + k) * 64] -= vr * S3[k * 64];
    }
  }
  for (int r = 0; r < kz; ++r) {
    zq[r] = r < N ? Zp[r * 64] : -1;
    q[r] = r < N ? (ok ? Xp[r * 64] + sig * S2[r * 64] : NAN) : 0.0;
  }
  return ok;
}

// Workspace of one tile of 64 chains, in doubles: the inverse Gram matrix, five vectors
// (b, x and three scratch); grid indices and the N histogram are in the int workspace.
template <int KCAP>
struct LaneLayout {
  static constexpr int HD = KCAP * KCAP;  // doubles per chain for H
  static constexpr int ED = HD + 5 * KCAP;
  static constexpr int EI = 2 * KCAP + 1;
};

// The inverse Gram matrix of the PE list Zp[0..N) in FP64 by bordering (each step is the
// birth update of the PE-space factor: the exact inverse of the leading block), into Wp.
// Returns false if a Schur complement is not positive.
template <int KCAP>
__device__ bool lane_build(const ModelDev &md, const double *vt, const double *ov, int Lw, double *Wp, double *S1,
                           double *S2, const int32_t *Zp, int N) {
  for (int k = 0; k < N; ++k) {
    const int gk = Zp[k * 64];
    for (int i = 0; i < k; ++i) S1[i * 64] = overlap(md, vt, ov, gk, Zp[i * 64], Lw);
    const double d = overlap(md, vt, ov, gk, gk, Lw) + md.rho;
    double q, p;
    lane_matvec<KCAP, double>(Wp, S1, S2, nullptr, k, q, p);
    const double delta2 = d - q;
    if (!(delta2 > 0.0)) return false;
    const double inv = 1.0 / delta2;
    lane_rank_update<KCAP, false, double>(Wp, S2, inv, nullptr, 0.0, k);
    for (int i = 0; i < k; ++i) {
      const double v = -S2[i * 64] * inv;
      Wp[(k * KCAP + i) * 64] = v;
      Wp[(i * KCAP + k) * 64] = v;
    }
    Wp[(k * KCAP + k) * 64] = inv;
  }
  return true;
}

// Delta-nu and log-acceptance of a birth or update proposal from the inverse Gram
// matrix M (gamma in S1 with a zero at the moved PE, eta = M gamma written to S2).
struct MvResult {
  bool valid;
  double dnu, la, delta2, up, om, xj, ej;
};

template <int KCAP, typename MT>
__device__ inline MvResult lane_propose(const ModelDev &md, const MT *Mp, const double *S1, double *S2,
                                        const double *Xp, int N, int move, int j, double d, double beta, double logLam,
                                        double logN1, double la_ratio) {
  MvResult r;
  r.valid = false;
  r.dnu = 0.0;
  r.la = -INFINITY;
  r.om = 1.0;
  r.xj = 0.0;
  r.ej = 0.0;
  double q, p;
  lane_matvec<KCAP, MT>(Mp, S1, S2, Xp, N, q, p);
  if (move == 1) {
    r.delta2 = d - q;
    r.up = beta - p;
    if (r.delta2 > 0.0) {
      r.dnu = -0.5 * (-md.log_rho + log(r.delta2) + (md.rhom2 - r.up * r.up / r.delta2) * md.inv_s);
      r.la = r.dnu + logLam - logN1 + (N == 0 ? md.logJ : 0.0);
      r.valid = true;
    }
  } else {
    r.om = (double)Mp[(j * KCAP + j) * 64];
    r.xj = Xp[j * 64];
    r.ej = S2[j * 64];
    r.delta2 = d - (q - r.ej * r.ej / r.om);
    r.up = beta - (p - r.ej * r.xj / r.om);
    if (r.delta2 > 0.0 && r.om > 0.0) {
      r.dnu = 0.5 * (-log(r.om) - log(r.delta2) + (r.up * r.up / r.delta2 - r.xj * r.xj / r.om) * md.inv_s);
      r.la = r.dnu + la_ratio;
      r.valid = true;
    }
  }
  return r;
}

// One chain per lane.  The chain's H = G^{-1} (full, KCAP x KCAP, FP64), x, b, scratch and
// PE list live in device memory, interleaved across the 64 chains of a tile so that every
// access of a wavefront is one contiguous segment.  Two wavefronts per SIMD at the least
// (the register budget halves): with one, nothing hides the device-memory round trips of
// the state (measured 21% slower at capacity 16).
template <int KCAP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) chain_lane_kernel(ChainArgs a) {
  using LL = LaneLayout<KCAP>;
  extern __shared__ double smem[];
  const ModelDev &md = a.md;
  double *vt = smem;
  double *ov = smem + md.M;
  for (int i = threadIdx.x; i < md.M; i += blockDim.x) vt[i] = a.vtab[i];
  for (int i = threadIdx.x; i < md.sub * md.M; i += blockDim.x) ov[i] = a.ovl[i];
  double *lgn = ov + md.sub * md.M;  // log k, k = 0..KCAP + 1
  for (int i = threadIdx.x; i < KCAP + 2; i += blockDim.x) lgn[i] = log((double)i);
  __syncthreads();
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= a.n_list) return;

  const int64_t tile = slot >> 6;
  const int ln = (int)(slot & 63);
  double *base = a.dws + tile * (int64_t)LL::ED * 64;
  double *Hp = base + ln;
  double *Xp = base + (int64_t)LL::HD * 64 + ln;
  double *Bp = Xp + KCAP * 64;
  double *S1 = Bp + KCAP * 64;
  double *S2 = S1 + KCAP * 64;
  double *S3 = S2 + KCAP * 64;
  int32_t *Zp = a.iws + tile * (int64_t)LL::EI * 64 + ln;
  int32_t *Hs = Zp + KCAP * 64;
#define HM(k, i) Hp[((k) * KCAP + (i)) * 64]
#define XV(i) Xp[(i) * 64]
#define BV(i) Bp[(i) * 64]
#define G1(i) S1[(i) * 64]
#define G2(i) S2[(i) * 64]
#define G3(i) S3[(i) * 64]
#define ZG(i) Zp[(i) * 64]
#define HIST(i) Hs[(i) * 64]

  const int64_t c = a.chains[slot];
  const int64_t w = c / a.n_chains;
  const int ch = (int)(c % a.n_chains);
  const int Lw = (int)(a.woff[w + 1] - a.woff[w]);
  const double lam = a.lam[w];
  const int kmax = a.kmax[w];
  const int glo = a.grange[2 * w], ghi = a.grange[2 * w + 1];
  const double *mf = a.mf + a.mfoff[w];
  const uint64_t uid = a.wid[w] * (uint64_t)a.n_chains + (uint64_t)ch;
  const uint32_t uid0 = (uint32_t)uid, uid1 = (uint32_t)(uid >> 32);
  uint32_t st = a.wflags[w];
  if (glo > ghi) st |= FSMP_ST_EMPTY_T;
  // this waveform's sweeps and burn-in (the configured burn-in fraction), batch means
  const int steps_w = a.wsteps ? a.wsteps[w] : a.n_steps;
  const int burn = a.wsteps ? (int)((int64_t)steps_w * a.burn_in / a.n_steps) : a.burn_in;
  const int n_steps = (st & FSMP_ST_NONFINITE) ? 0 : steps_w;
  const int S_rec = n_steps > burn ? n_steps - burn : 0;
  const int nb = S_rec > 0 ? (int)floor(sqrt((double)S_rec)) : 0;
  const int lb = nb > 0 ? S_rec / nb : 0;
  for (int k = 0; k <= KCAP; ++k) HIST(k) = 0;

  double t0 = a.t0init[w];
  int N = 0;
  int gmin = INT32_MAX;  // smallest PE grid index (phi must stay positive at every PE)
  double S_cur = 0.0;    // BIEXP: sum_k log(1 - e^{-(t_k - t0)/tau_rise})
  double Phi = (glo <= ghi) ? phi_total(md, t0, glo, ghi) : 0.0;
  double logLam = log(lam * md.dt * Phi);  // changes only with t0
  double acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = 0.0;
  double bs0 = 0.0, bs1 = 0.0, bs2 = 0.0;
  int cnt[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) cnt[i] = 0;
  double wk0 = 0.0, wk1 = 0.0, wk2 = 0.0, wk3 = 0.0;
  const bool biexp = md.kind == FSMP_PHI_BIEXP;

  // a caller-supplied initial PE list: G^-1 (FP64, by bordering) and x = G^-1 b of the
  // list before the first sweep; no random numbers are drawn for it
  if (a.zinit && n_steps > 0) {
    const int n0 = (int)(a.zinit_off[c + 1] - a.zinit_off[c]);
    if (n0 > 0) {
      const int32_t *z0 = a.zinit + a.zinit_off[c];
      for (int k = 0; k < n0; ++k) ZG(k) = z0[k];
      if (lane_build<KCAP>(md, vt, ov, Lw, Hp, S1, S2, Zp, n0)) {
        for (int k = 0; k < n0; ++k) BV(k) = mf[ZG(k) - glo] + md.rhom;
        for (int i = 0; i < n0; ++i) {
          double xi = 0.0;
          for (int k = 0; k < n0; ++k) xi += Hp[(i * KCAP + k) * 64] * BV(k);
          XV(i) = xi;
        }
        N = n0;
        for (int i = 0; i < N; ++i) {
          if (biexp) S_cur += log(-expm1(-((double)ZG(i) * md.dt - t0) * md.inv_tau1));
          gmin = ZG(i) < gmin ? ZG(i) : gmin;
          occ_edit(a, c, 1, -1, ZG(i), 0, burn, n_steps);
        }
      } else {
        st |= FSMP_ST_FACTOR;
      }
    }
  }
  for (int step = 0; step < n_steps; ++step) {
    if (a.refresh_M > 0 && step > 0 && step % a.refresh_M == 0 && N > 0) {
      // G^-1 rebuilt by bordering and x = G^-1 b recomputed, against the rounding the edits
      // accumulate
      if (lane_build<KCAP>(md, vt, ov, Lw, Hp, S1, S2, Zp, N)) {
        for (int i = 0; i < N; ++i) {
          double xi = 0.0;
          for (int k = 0; k < N; ++k) xi += Hp[(i * KCAP + k) * 64] * BV(k);
          XV(i) = xi;
        }
      } else {
        st |= FSMP_ST_FACTOR;
      }
    }
    uint32_t r[8];
    philox4x32_10((uint32_t)step, 0u, uid0, uid1, a.key0, a.key1, r);
    philox4x32_10((uint32_t)step, 1u, uid0, uid1, a.key0, a.key1, r + 4);
    const double R = sqrt(-2.0 * log(u01(r[0])));
    const double th = 2.0 * M_PI * u01(r[1]);
    const double xi_t0 = R * cos(th), xi_sh = R * sin(th);

    // ---- Gibbs half-step 1: t0 by Metropolis-Hastings
    const double t0p = t0 + md.t0_sd * xi_t0;
    bool t0acc = false;
    cnt[0]++;
    if (t0p >= md.t0_min && t0p <= md.t0_max) {
      const double xmin = (N > 0) ? (double)gmin * md.dt - t0p : 1.0;
      const bool ok = biexp ? (xmin > 0.0) : (xmin >= 0.0);
      if (ok) {
        double S_new = 0.0;
        if (biexp)
        {
          // the rise factors multiplied in runs of up to eight, one log per run
          double pr = 1.0;
          int m = 0;
          for (int i = 0; i < N; ++i) {
            pr *= rise_factor(md, ZG(i), t0p);
            if (++m == 8) {
              S_new += log(pr);
              pr = 1.0;
              m = 0;
            }
          }
          S_new += log(pr);
        }
        const double part = (double)N * (t0p - t0) * md.inv_tau2 + (S_new - S_cur);
        const double Phip = (glo <= ghi) ? phi_total(md, t0p, glo, ghi) : 0.0;
        const double la0 = part - (lam * md.dt * Phip - lam * md.dt * Phi);
        if (log(u01(r[2])) < la0) {
          t0 = t0p;
          Phi = Phip;
          logLam = log(lam * md.dt * Phi);
          S_cur = S_new;
          t0acc = true;
          cnt[1]++;
        }
      }
    }

    // ---- Gibbs half-step 2: one RJMCMC jump
    const double Lam = lam * md.dt * Phi;
    const double um = u01(r[3]);
    const int move = (N == 0 || um < md.J) ? 1 : (um < 2.0 * md.J ? 2 : 3);
    int j = -1, gnew = -1, sh = 0;
    bool valid = false;
    double dnu = 0.0, la = -INFINITY;
    double delta2 = 1.0, up = 0.0, om = 1.0, xj = 0.0, ej = 0.0, beta = 0.0, dself = 0.0, la_ratio = 0.0;
    bool need_mv = false;
    if (move == 1) {
      cnt[2]++;
      if (N >= kmax) {
        st |= FSMP_ST_KMAX;
      } else if (Phi > 0.0) {
        gnew = birth_draw_lane(md, t0, glo, ghi, u53(r[4], r[5]) * Phi);
        need_mv = Lam > 0.0;
      }
    } else {
      j = (int)(((uint64_t)r[4] * (uint64_t)N) >> 32);
      if (move == 2) {
        cnt[4]++;
        om = HM(j, j);
        xj = XV(j);
        if (om > 0.0) {
          dnu = 0.5 * (-md.log_rho - log(om) + (md.rhom2 - xj * xj / om) * md.inv_s);
          la = dnu - logLam + lgn[N] - (N == 1 ? md.logJ : 0.0);
          valid = true;
          const double r = N - j;
          wk0 += r * (r + 1) / 2 + 1;
          wk2 += 1.0;
        } else {
          st |= FSMP_ST_FACTOR;
        }
      } else {
        cnt[6]++;
        sh = (int)rint(xi_sh * md.shift_sd / md.dt);
        gnew = ZG(j) + sh;
        if (gnew >= glo && gnew <= ghi) {
          const double lpn = log_phi(md, (double)gnew * md.dt - t0);
          if (lpn > -INFINITY) {
            const double lpo = log_phi(md, (double)ZG(j) * md.dt - t0);
            if (sh == 0) {
              valid = true;
              dnu = 0.0;
              la = lpn - lpo;
            } else {
              need_mv = true;
              la_ratio = lpn - lpo;
            }
          }
        }
      }
    }
    if (need_mv) {
      for (int i = 0; i < N; ++i) G1(i) = (i == j) ? 0.0 : overlap(md, vt, ov, gnew, ZG(i), Lw);
      dself = overlap(md, vt, ov, gnew, gnew, Lw) + md.rho;
      beta = mf[gnew - glo] + md.rhom;
      // the word count of the proposal in a packed Cholesky factor, and the G^-1 elements read
      {
        const double K = N, r = N - j;
        wk0 += move == 1 ? K * (K + 1) / 2 + 2 * K + 3 : r * (r + 1) / 2 + 1 + (K - 1) * K / 2 + 2 * (K - 1) + 3;
        wk2 += K * K;
      }
      const MvResult mr =
          lane_propose<KCAP, double>(md, Hp, S1, S2, Xp, N, move, j, dself, beta, logLam, lgn[N + 1], la_ratio);
      valid = mr.valid;
      dnu = mr.dnu;
      la = mr.la;
      delta2 = mr.delta2;
      up = mr.up;
      om = mr.om;
      xj = mr.xj;
      ej = mr.ej;
      if (!valid) st |= FSMP_ST_FACTOR;
    }

    const double logu = log(u01(r[6]));
    bool accepted = false;
    if (valid && logu < la) {
      accepted = true;
      cnt[2 * move + 1]++;
      // One edit path for every accepted move (the wavefront's 64 chains run whichever
      // moves they drew; one path is executed once): with h = row j of H and eta from the
      // proposal, M(k, i) += cu u_i u_k + cv v_i v_k over i, k < N with
      //   birth: u = eta, cu = 1/delta^2; death: u = h, cu = -1/omega;
      //   shift: u = h, cu = -1/omega and v = eta (zero at j), cv = 1/delta^2.
      const bool shift = move == 3 && sh != 0;  // an accepted zero shift changes nothing
      {
        const double K = N, r = N - j;
        const double eb = move == 1 ? K + 3 : (K - 1) + 3, ed = (r - 1) * r + K * (K + 1) / 2;
        wk1 += move == 1 ? eb : move == 2 ? ed : (shift ? ed + eb : 0.0);
      }
      if (move != 3 || shift) {
        wk3 += 2.0 * (double)N * N;
        const double inv_d2 = move == 2 ? 0.0 : 1.0 / delta2;
        const double inv_om = move == 1 ? 0.0 : 1.0 / om;
        const double xn = up * inv_d2;
        const int gj = move == 1 ? -1 : ZG(j);
        occ_edit(a, c, move, gj, gnew, step, burn, n_steps);
        if (move != 1) lane_copy(S3, Hp + (int64_t)j * KCAP * 64, N);  // h = row j of H
        if (shift)
          for (int i = 0; i < N; ++i) G2(i) = (i == j) ? 0.0 : G2(i) - G3(i) * ej * inv_om;
        const double *U = move == 1 ? S2 : S3;
        const double *V = shift ? S2 : U;
        const double cu = move == 1 ? inv_d2 : -inv_om, cv = shift ? inv_d2 : 0.0;
        for (int i = 0; i < N; ++i) {
          const double ui = U[i * 64], vi = V[i * 64];
          XV(i) = move == 1 ? XV(i) - ui * xn
                  : move == 2 ? XV(i) - ui * xj * inv_om
                              : ((i == j) ? xn : XV(i) - ui * xj * inv_om - vi * xn);
        }
        lane_rank_update<KCAP, true, double>(Hp, U, cu, V, cv, N);
        if (move == 1) {
          for (int i = 0; i < N; ++i) {
            const double v = -G2(i) * inv_d2;
            HM(N, i) = v;
            HM(i, N) = v;
          }
          HM(N, N) = inv_d2;
          ZG(N) = gnew;
          BV(N) = beta;
          XV(N) = xn;
          if (biexp) S_cur += log(-expm1(-((double)gnew * md.dt - t0) * md.inv_tau1));
          gmin = gnew < gmin ? gnew : gmin;
          N++;
        } else if (move == 2) {
          const int last = N - 1;
          if (j != last) {
            lane_copy(S3, Hp + (int64_t)last * KCAP * 64, N);  // row `last` moves into slot j
            const double vd = G3(last);
            lane_copy(Hp + (int64_t)j * KCAP * 64, S3, N);
            for (int i = 0; i < N; ++i) HM(i, j) = G3(i);
            HM(j, j) = vd;
            ZG(j) = ZG(last);
            BV(j) = BV(last);
            XV(j) = XV(last);
          }
          N--;
          if (biexp) S_cur -= log(-expm1(-((double)gj * md.dt - t0) * md.inv_tau1));
        } else {
          for (int i = 0; i < N; ++i) {
            if (i == j) {
              HM(j, j) = inv_d2;
            } else {
              const double v = -G2(i) * inv_d2;
              HM(j, i) = v;
              HM(i, j) = v;
            }
          }
          ZG(j) = gnew;
          BV(j) = beta;
          if (biexp)
            S_cur += log(-expm1(-((double)gnew * md.dt - t0) * md.inv_tau1)) -
                     log(-expm1(-((double)gj * md.dt - t0) * md.inv_tau1));
        }
        if (move != 1) {
          if (move == 3 && gnew < gmin) {
            gmin = gnew;
          } else if (gj == gmin) {
            gmin = INT32_MAX;
            for (int i = 0; i < N; ++i) gmin = ZG(i) < gmin ? ZG(i) : gmin;
          }
        }
      }
    }

    if (a.log) {
      fsmp_logrec *lr = a.log + c * (int64_t)a.n_steps + step;
      lr->move = move;
      lr->flags = (valid ? 1 : 0) | (accepted ? 2 : 0) | (t0acc ? 4 : 0);
      lr->j = j;
      lr->g = gnew;
      lr->t0 = t0;
      lr->dnu = valid ? dnu : 0.0;
      lr->log_alpha = valid ? la : -INFINITY;
    }

    // ---- record after burn-in
    if (step >= burn) {
      double Q = 0.0;
      for (int i = 0; i < N; ++i) Q += XV(i);
      const double v0 = (double)N, v1 = Q, v2 = t0;
      acc[0] += v0;
      acc[1] += v0 * v0;
      acc[2] += v1;
      acc[3] += v1 * v1;
      acc[4] += v2;
      acc[5] += v2 * v2;
      const int64_t i = step - burn;
      if (nb > 0 && i < (int64_t)nb * lb) {
        bs0 += v0;
        bs1 += v1;
        bs2 += v2;
        if ((i + 1) % lb == 0) {
          acc[6] += bs0;
          acc[7] += bs0 * bs0;
          acc[8] += bs1;
          acc[9] += bs1 * bs1;
          acc[10] += bs2;
          acc[11] += bs2 * bs2;
          bs0 = bs1 = bs2 = 0.0;
        }
      }
      HIST(N) += 1;
      if (a.trace && a.thin > 0 && (i % a.thin) == 0) {
        double *tr = a.trace + (c * a.n_rec + i / a.thin) * 3;
        tr[0] = v0;
        tr[1] = v2;
        tr[2] = v1;
      }
      if (a.qdraw && a.thin > 0 && (i % a.thin) == 0) {
        const int64_t rec = c * a.n_rec + i / a.thin;
        if (!lane_charge_draw<KCAP, double>(a.dscr + tile * (int64_t)KCAP * KCAP * 64 + ln, Hp, Xp, S1, S2, S3, Zp, N,
                                        step, uid0, uid1, a.key0, a.key1, a.sigma_eps, a.qdraw + rec * a.kz,
                                        a.zdraw + rec * a.kz, a.kz))
          st |= FSMP_ST_FACTOR;
      }
    }
  }

  const int kz = a.kz;
  for (int k = 0; k < kz; ++k) {
    a.z[c * kz + k] = k < N ? ZG(k) : -1;
    a.charge[c * kz + k] = k < N ? XV(k) : 0.0;
  }
  for (int k = 0; k <= kz; ++k) a.nhist[c * (kz + 1) + k] = k <= KCAP ? HIST(k) : 0;
  a.n_pe[c] = N;
  a.t0[c] = t0;
  if (a.rec_steps) a.rec_steps[c] = S_rec;
  for (int i = 0; i < 12; ++i) a.acc[c * 12 + i] = acc[i];
  for (int i = 0; i < 8; ++i) a.counts[c * 8 + i] = cnt[i];
  a.status[c] = st;
  if (a.work) {
    a.work[c * 5 + 0] = wk0;
    a.work[c * 5 + 1] = wk1;
    a.work[c * 5 + 2] = wk2;
    a.work[c * 5 + 3] = wk3;
    a.work[c * 5 + 4] = 0.0;
  }
#undef HM
#undef XV
#undef BV
#undef G1
#undef G2
#undef G3
#undef ZG
#undef HIST
}

// ------------------------------------------------------------------ posterior
// Expected number of PEs at every grid point: the occupancy counts of a waveform's chains
// over its recorded (chain, sweep) pairs; one workgroup per waveform, coalesced over its row.
__global__ void __launch_bounds__(256) occupancy_kernel(PosteriorArgs a) {
  for (int64_t w = blockIdx.x; w < a.n_wave; w += gridDim.x) {
    const int S = a.rec_steps ? a.rec_steps[w * a.n_chains] : a.n_steps - a.burn_in;
    const double inv = S > 0 ? 1.0 / ((double)S * a.n_chains) : 0.0;
    const int64_t b = (int64_t)a.sub * a.woff[w], e = (int64_t)a.sub * a.woff[w + 1];
    for (int64_t g = b + threadIdx.x; g < e; g += blockDim.x) a.occupancy[g] = (double)a.occ[g] * inv;
  }
}

__global__ void __launch_bounds__(256) posterior_kernel(PosteriorArgs a) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.n_wave) return;
  // the chains of one waveform ran the same number of sweeps
  const int S = a.rec_steps ? a.rec_steps[w * a.n_chains] : a.n_steps - a.burn_in;
  const int nb = S > 0 ? (int)floor(sqrt((double)S)) : 0;
  const int lb = nb > 0 ? S / nb : 0;
  const int C = a.n_chains;
  uint32_t st = 0;
  for (int v = 0; v < 3; ++v) {
    double s1 = 0.0, s2 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int ch = 0; ch < C; ++ch) {
      const double *ac = a.acc + (w * C + ch) * 12;
      s1 += ac[2 * v];
      s2 += ac[2 * v + 1];
      b1 += ac[6 + 2 * v];
      b2 += ac[7 + 2 * v];
    }
    const double n = (double)S * C;
    const double mean = S > 0 ? s1 / n : 0.0;
    const double var = S > 0 ? fmax(s2 / n - mean * mean, 0.0) : 0.0;
    const double B = (double)nb * C;
    double mcse = 0.0;
    if (nb > 0 && B > 1.0) {
      const double bm = b1 / (B * lb);
      const double bv = fmax((b2 / ((double)lb * lb) - B * bm * bm) / (B - 1.0), 0.0);
      mcse = sqrt(bv / B);
    }
    a.mean[w * 3 + v] = mean;
    a.var[w * 3 + v] = var;
    a.mcse[w * 3 + v] = mcse;
  }
  double prop[4] = {0, 0, 0, 0}, accp[4] = {0, 0, 0, 0};
  for (int ch = 0; ch < C; ++ch) {
    const int32_t *cn = a.counts + (w * C + ch) * 8;
    for (int m = 0; m < 4; ++m) {
      prop[m] += cn[2 * m];
      accp[m] += cn[2 * m + 1];
    }
    st |= a.cstatus[w * C + ch];
  }
  for (int m = 0; m < 4; ++m) a.accept[w * 4 + m] = prop[m] > 0 ? accp[m] / prop[m] : 0.0;
  if (a.p_n) {
    const int kz = a.kz;
    double tot = 0.0;
    for (int ch = 0; ch < C; ++ch)
      for (int k = 0; k <= kz; ++k) tot += a.nhist[(w * C + ch) * (kz + 1) + k];
    for (int k = 0; k <= kz; ++k) {
      double s = 0.0;
      for (int ch = 0; ch < C; ++ch) s += a.nhist[(w * C + ch) * (kz + 1) + k];
      a.p_n[w * (kz + 1) + k] = tot > 0 ? s / tot : 0.0;
    }
  }
  a.status[w] = st;
}

// ---- posterior extras: chain diagnostics and the lambda estimates, one thread per waveform

// d(lambda) = m(lambda) - lambda, m the mean of k under the weights h_k (lambda / lambda0)^k
// (computed from the largest log-weight down); with `f` also the log-likelihood estimate
// f(lambda) = -(lambda - lambda0) + log sum_k h_k (lambda / lambda0)^k.  lambda = 0 keeps k = 0.
__device__ inline double lam_tilt(const int32_t *nh, int C, int kz1, int k_lo, int k_hi, double lam, double lam0,
                                  double *f) {
  const double lr = lam > 0.0 ? log(lam / lam0) : 0.0;
  const int top = lam > 0.0 ? k_hi : 0;
  double mx = -INFINITY;
  for (int k = k_lo; k <= top; ++k) {
    double h = 0.0;
    for (int ch = 0; ch < C; ++ch) h += nh[ch * kz1 + k];
    if (h > 0.0) mx = fmax(mx, log(h) + k * lr);
  }
  double se = 0.0, sk = 0.0;
  for (int k = k_lo; k <= top; ++k) {
    double h = 0.0;
    for (int ch = 0; ch < C; ++ch) h += nh[ch * kz1 + k];
    if (h > 0.0) {
      const double e = exp(log(h) + k * lr - mx);
      se += e;
      sk += k * e;
    }
  }
  if (f) *f = -(lam - lam0) + mx + log(se);
  return sk / se - lam;
}

__global__ void __launch_bounds__(256) posterior_extra_kernel(PosteriorArgs a) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.n_wave) return;
  const int C = a.n_chains;
  const int S = a.rec_steps ? a.rec_steps[w * C] : a.n_steps - a.burn_in;
  // Gelman-Rubin R and the Monte Carlo error from the spread of the chain means
  for (int v = 0; v < 3; ++v) {
    double msum = 0.0;
    for (int ch = 0; ch < C; ++ch) msum += a.acc[(w * C + ch) * 12 + 2 * v] / S;
    const double mbar = msum / C;
    double dev2 = 0.0, wsum = 0.0;
    for (int ch = 0; ch < C; ++ch) {
      const double *ac = a.acc + (w * C + ch) * 12;
      const double m = ac[2 * v] / S;
      dev2 += (m - mbar) * (m - mbar);
      wsum += fmax((ac[2 * v + 1] - S * m * m) / (S - 1), 0.0);
    }
    double r = NAN, mc = NAN;
    if (C >= 2 && S >= 1) mc = sqrt(dev2 / ((double)C * (C - 1)));
    if (C >= 2 && S >= 2) {
      const double W = wsum / C;
      const double B = S * dev2 / (C - 1);
      const double V = (double)(S - 1) / S * W + B / S;
      r = W > 0.0 ? sqrt(V / W) : (V > 0.0 ? INFINITY : 1.0);
    }
    if (a.rhat) a.rhat[w * 3 + v] = r;
    if (a.mcse_chains) a.mcse_chains[w * 3 + v] = mc;
  }
  if (!a.lambda_hat) return;
  // lambda-hat: the + to - crossings of d on 64 grid points of [k_lo, k_hi], each refined by
  // bisection, and lambda = 0 when k_lo = 0 and d <= 0 at the second point; the largest f wins
  const int kz1 = a.kz + 1;
  const int32_t *nh = a.nhist + w * C * kz1;
  int k_lo = -1, k_hi = -1;
  for (int k = 0; k < kz1; ++k) {
    int32_t h = 0;
    for (int ch = 0; ch < C; ++ch) h += nh[ch * kz1 + k];
    if (h > 0) {
      if (k_lo < 0) k_lo = k;
      k_hi = k;
    }
  }
  double est = NAN;
  const double lam0 = a.lam0[w];
  if (k_lo >= 0 && k_lo == k_hi) {
    est = k_lo;
  } else if (k_lo >= 0) {
    constexpr int kGrid = 64;
    const double span = (double)(k_hi - k_lo);
    double best_f = -INFINITY;
    double dprev = 0.0;
    for (int i = 0; i < kGrid; ++i) {
      const double x = k_lo + span * i / (kGrid - 1);
      const double dx = lam_tilt(nh, C, kz1, k_lo, k_hi, x, lam0, nullptr);
      double cand = NAN;
      if (i == 1 && k_lo == 0 && dx <= 0.0) {
        double f0;
        (void)lam_tilt(nh, C, kz1, k_lo, k_hi, 0.0, lam0, &f0);
        if (f0 > best_f) {
          best_f = f0;
          est = 0.0;
        }
      }
      if (i > 0 && dprev > 0.0 && dx <= 0.0) {
        if (dx == 0.0) {
          cand = x;
        } else {
          double lo = k_lo + span * (i - 1) / (kGrid - 1), hi = x;
          for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            if (lam_tilt(nh, C, kz1, k_lo, k_hi, mid, lam0, nullptr) > 0.0) lo = mid;
            else hi = mid;
          }
          cand = 0.5 * (lo + hi);
        }
        double fc;
        (void)lam_tilt(nh, C, kz1, k_lo, k_hi, cand, lam0, &fc);
        if (fc > best_f) {
          best_f = fc;
          est = cand;
        }
      }
      dprev = dx;
    }
  }
  a.lambda_hat[w * 2] = est;
  a.lambda_hat[w * 2 + 1] = a.mean[w * 3 + 1] / a.mu_q;  // lambda-hat_Q = E[Q] / mu_q
}

template <int KCAP, int LPC, int WPB, bool HG, bool FORCE = false, bool F32 = false, bool MCP = false>
hipError_t launch_chain_t(const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks) {
  constexpr int CPB = WPB * (kWave / LPC);
  const int64_t nb = (a.n_list + CPB - 1) / CPB;
  const size_t lds = sizeof(double) * ((size_t)a.md.M * (1 + a.md.sub) + (KCAP + 2) +
                                       (size_t)CPB * ChainLayout<KCAP, HG, F32, MCP>::kDoubles);
  *lanes = LPC;
  *blocks = nb;
  if (nb == 0) return hipSuccess;
  if (HG && a.dws == nullptr) return hipErrorInvalidValue;
  if (lds > 160 * 1024) return hipErrorInvalidValue;  // the host checks the configurations against this
  if (lds > 64 * 1024) {
    // lift the default dynamic-LDS limit; gfx950 has 160 KB per workgroup
    (void)hipFuncSetAttribute((const void *)chain_kernel<KCAP, LPC, WPB, HG, FORCE, F32, MCP>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
  }
  if (FORCE && (a.force == nullptr || a.rdnu == nullptr || a.rla == nullptr)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((chain_kernel<KCAP, LPC, WPB, HG, FORCE, F32, MCP>), dim3((unsigned)nb), dim3(kWave * WPB), lds,
                     st, a);
  return hipGetLastError();
}


template <int KCAP>
hipError_t launch_chain_lane_t(const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks) {
  const int64_t nb = (a.n_list + 255) / 256;
  const size_t lds = sizeof(double) * ((size_t)a.md.M * (1 + a.md.sub) + KCAP + 2);
  *lanes = 1;
  *blocks = nb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((chain_lane_kernel<KCAP>), dim3((unsigned)nb), dim3(256), lds, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Lucy-Richardson
// Initial PE sequence by deconvolution (Sec. 2.3): one workgroup per waveform, all arrays
// in LDS, FP64.  Both sums of an iteration are correlations of an LDS array with the
// kernel, out[i] = sum_s X[i + s] k[s]:
//   w^r(t)  = sum_s u[t + s] K[LV - 1 - s]          (u indexed by tau + LV - 1)
//   c(tau)  = sum_s rp[tau + LV - 1 + s] K[s]        (rp: the ratio d / w^r, zero-padded)
// each thread computes R consecutive outputs from a sliding window of X in registers:
// one LDS read of X per R FMAs.  The kernel k is the same for every lane: it is read from
// a read-only device array by scalar loads (eight values per load, through the scalar
// cache), which costs no LDS bandwidth and no vector issue slot.  The lanes of a wavefront
// read X R elements apart, so X is stored skewed by one pad element per R (element e at
// e + e / R): the lanes' reads then fall in different banks.  The first sum uses R = 8;
// the second, which has L_V - 1 more outputs, R = 6, which fills whole wavefronts at the
// usual window lengths (1,024 samples: 128 and 187 chunks, three wavefronts).
constexpr int kLucyR1 = 8, kLucyR2 = 6;

template <int R>
__device__ inline int lsk(int e) {
  return e + e / R;
}

// the read-only kernel array, seen through the constant address space so that its
// wavefront-uniform reads compile to scalar loads
typedef const __attribute__((address_space(4))) double *ConstD;

template <int R>
__device__ inline void lucy_corr(const double *X, ConstD k, int LVp, int i0, double *acc) {
  // i0 and LVp are multiples of R, so every R-element block of X starts at (R + 1) * block
  double xw[R];
  const double *xb = X + (R + 1) * (i0 / R);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    xw[j] = xb[j];
    acc[j] = 0.0;
  }
  const double *nb = xb + (R + 1);  // the next block; one block further per R taps
  for (int s = 0; s < LVp; s += R, nb += R + 1) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const double ks = k[s + u];
#pragma unroll
      for (int j = 0; j < R; ++j) acc[j] = fma(xw[j], ks, acc[j]);
#pragma unroll
      for (int j = 0; j < R - 1; ++j) xw[j] = xw[j + 1];
      xw[R - 1] = nb[u];
    }
  }
}

__global__ void __launch_bounds__(256) lucy_kernel(LucyArgs a) {
  extern __shared__ double lds[];
  const int LV = a.LV, LVp = a.LVp;
  const ConstD K = (ConstD)a.kern;       // [LVp] K[s], zero beyond LV
  const ConstD Kr = (ConstD)a.kern_rev;  // [LVp] K[LV - 1 - s], zero beyond LV
  __shared__ double redl[8];
  __shared__ int redc[8];
  constexpr int R1 = kLucyR1, R2 = kLucyR2;
  for (int64_t w = blockIdx.x; w < a.n_wave; w += gridDim.x) {
    const int Lw = (int)(a.woff[w + 1] - a.woff[w]);
    const int ntau = Lw + LV - 1;
    const int nd = (Lw + R1 - 1) / R1 * R1;       // d zero-padded to whole first-sum chunks
    const int n2 = (ntau + R2 - 1) / R2 * R2;     // outputs of the second sum, whole chunks
    const int nu = n2 + LVp + R1;                 // elements of u (zero beyond ntau)
    const int nrp = n2 + LVp + R2;                // elements of rp: LV - 1 zeros | ratio | zeros
    double *d = lds;                              // [nd], plain layout
    double *u = d + nd;                           // skewed by R1
    double *rp = u + lsk<R1>(nu) + 1;             // skewed by R2
    const float *x = a.wave + a.woff[w];
    __syncthreads();
    double sd = 0.0;
    for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      const double v = t < Lw ? fmax((double)x[t], 0.0) : 0.0;
      d[t] = v;
      sd += v;
    }
    for (int o = 32; o > 0; o >>= 1) sd += __shfl_xor(sd, o);
    if ((threadIdx.x & 63) == 0) redl[threadIdx.x >> 6] = sd;
    __syncthreads();
    double tot = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += redl[i];
    const double u0 = tot / ntau;
    for (int i = threadIdx.x; i < nu; i += blockDim.x) u[lsk<R1>(i)] = i < ntau ? u0 : 0.0;
    for (int i = threadIdx.x; i < nrp; i += blockDim.x) rp[lsk<R2>(i)] = 0.0;
    __syncthreads();
    for (int it = 0; it < a.n_iter; ++it) {
      // w^r and the ratio d / w^r (0 where w^r is not positive).  The writes need no
      // bounds: d is zero past L_w, so the ratios written past the window stay 0
      for (int c0 = threadIdx.x * R1; c0 < Lw; c0 += blockDim.x * R1) {
        double acc[R1];
        lucy_corr<R1>(u, Kr, LVp, c0, acc);
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          // exact division: w^r decays to denormals where d is 0 (0 / w^r must stay 0)
          const double v = acc[j];
          const double q = d[c0 + j] / v;
          rp[lsk<R2>(LV - 1 + c0 + j)] = v > 0.0 ? q : 0.0;
        }
      }
      __syncthreads();
      // u(tau) *= sum_t ratio(t) K(t - tau); u stays 0 past tau = L_w - 1 (a select, no branch)
      for (int c0 = threadIdx.x * R2; c0 < ntau; c0 += blockDim.x * R2) {
        double acc[R2];
        lucy_corr<R2>(rp, K, LVp, c0, acc);
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          double *ue = u + lsk<R1>(c0 + j);
          *ue = c0 + j < ntau ? *ue * acc[j] : 0.0;
        }
      }
      __syncthreads();
    }
    // qhat in PE-charge units (back into a plain layout in rp); candidates tau >= 0 above the
    // threshold (flags in d)
    double lam = 0.0;
    int cnt = 0;
    for (int i = threadIdx.x; i < ntau; i += blockDim.x) {
      const double q = u[lsk<R1>(i)] * a.inv_area;
      rp[i] = q;
      lam += q;
      if (a.qhat) a.qhat[a.woff[w] + w * (int64_t)(LV - 1) + i] = q;
    }
    __syncthreads();
    const double *qh = rp;
    double *flag = u;  // plain layout from here on
    for (int i = threadIdx.x; i < Lw; i += blockDim.x) {
      const bool c = qh[i + LV - 1] > a.threshold;   // tau = i >= 0
      d[i] = c ? 1.0 : 0.0;
      cnt += c;
    }
    for (int o = 32; o > 0; o >>= 1) {
      lam += __shfl_xor(lam, o);
      cnt += __shfl_xor(cnt, o);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      redl[threadIdx.x >> 6] = lam;
      redc[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    lam = 0.0;
    cnt = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      lam += redl[i];
      cnt += redc[i];
    }
    const int kmax = a.kmax[w];
    if (cnt > kmax) {
      // keep the kmax largest qhat (ties: earlier tau): rank every candidate
      for (int i = threadIdx.x; i < Lw; i += blockDim.x) {
        if (d[i] == 0.0) {
          flag[i] = 0.0;
          continue;
        }
        const double qi = qh[i + LV - 1];
        int rank = 0;
        for (int j = 0; j < Lw; ++j) {
          const double qj = qh[j + LV - 1];
          rank += (qj > a.threshold) && (qj > qi || (qj == qi && j < i));
        }
        flag[i] = rank < kmax ? 1.0 : 0.0;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < Lw; i += blockDim.x) d[i] = flag[i];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      int t_min = -1, t_max = -1;
      for (int i = 0; i < Lw; ++i)
        if (d[i] != 0.0) {
          if (t_min < 0) t_min = i;
          t_max = i;
        }
      int n = 0;
      double t0 = 0.5 * (a.t0_min + a.t0_max);
      const int sub = a.sub;
      if (t_min < 0) {
        a.g_range[2 * w] = 1;
        a.g_range[2 * w + 1] = 0;
        a.cut[2 * w] = 0;
        a.cut[2 * w + 1] = Lw - 1;
      } else {
        t0 = fmin(fmax(t_min - 0.5 / sub, a.t0_min), a.t0_max);
        for (int i = t_min; i <= t_max; ++i)
          if (d[i] != 0.0 && i - t0 > 0.0 && n < a.kz) a.z[w * (int64_t)a.kz + n++] = sub * i;
        a.g_range[2 * w] = max(0, sub * (t_min - a.margin));
        a.g_range[2 * w + 1] = min(sub * Lw - 1, sub * (t_max + a.margin));
        a.cut[2 * w] = max(0, t_min - a.margin);
        a.cut[2 * w + 1] = min(Lw - 1, t_max + a.margin + LV);
      }
      for (int k = n; k < a.kz; ++k) a.z[w * (int64_t)a.kz + k] = -1;
      a.n_pe[w] = n;
      a.t0[w] = t0;
      a.lam[w] = lam;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_prologue(const PrologueArgs &a, hipStream_t st) {
  if (a.n_wave == 0) return hipSuccess;
  const int64_t nb = a.n_wave < 65535 * 8 ? a.n_wave : 65535 * 8;
  hipLaunchKernelGGL(prologue_kernel, dim3((unsigned)nb), dim3(256), sizeof(double) * a.md.M, st, a);
  return hipGetLastError();
}

size_t lucy_lds_bytes(int64_t Lw, int LVp) {
  const int64_t R1 = kLucyR1, R2 = kLucyR2;
  const int64_t ntau = Lw + LVp - 1;
  const int64_t nd = (Lw + R1 - 1) / R1 * R1, n2 = (ntau + R2 - 1) / R2 * R2;
  const int64_t nu = n2 + LVp + R1, nrp = n2 + LVp + R2;
  // d, then u and rp, each skewed by one pad element per window width
  return sizeof(double) * (size_t)(nd + (nu + nu / R1 + 1) + (nrp + nrp / R2 + 1));
}

hipError_t launch_lucy(const LucyArgs &a, int64_t max_len, hipStream_t st) {
  if (a.n_wave == 0) return hipSuccess;
  const size_t lds = lucy_lds_bytes(max_len, a.LVp);
  // enough threads for the longer pass of the longest window, in whole wavefronts
  const int64_t chunks = std::max((max_len + kLucyR1 - 1) / kLucyR1, (max_len + a.LV - 1 + kLucyR2 - 1) / kLucyR2);
  int threads = (int)((chunks + 63) / 64 * 64);
  threads = threads < 64 ? 64 : (threads > 256 ? 256 : threads);
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute((const void *)lucy_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
  }
  const int64_t nb = a.n_wave < 65535 * 8 ? a.n_wave : 65535 * 8;
  hipLaunchKernelGGL(lucy_kernel, dim3((unsigned)nb), dim3(threads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_posterior(const PosteriorArgs &a, hipStream_t st) {
  if (a.n_wave == 0) return hipSuccess;
  const int64_t nb = (a.n_wave + 255) / 256;
  hipLaunchKernelGGL(posterior_kernel, dim3((unsigned)nb), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && (a.rhat || a.mcse_chains || a.lambda_hat)) {
    hipLaunchKernelGGL(posterior_extra_kernel, dim3((unsigned)nb), dim3(256), 0, st, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess && a.occupancy) {
    const int64_t nw = a.n_wave < 65535 * 8 ? a.n_wave : 65535 * 8;
    hipLaunchKernelGGL(occupancy_kernel, dim3((unsigned)nw), dim3(256), 0, st, a);
    e = hipGetLastError();
  }
  return e;
}

int chain_kcap_for(int kmax) {
  for (int b = 0; b < kNumCaps; ++b)
    if (kmax <= kCaps[b]) return kCaps[b];
  return 0;
}

// lane-group instances: PE capacity, lanes per chain, wavefronts per workgroup.  With H
// in LDS the LDS bounds the chains per CU (one chain per wavefront at capacity 64); with H
// in device memory each chain keeps only its vectors in LDS, so groups can be narrow and a
// CU holds 8-16x more chains: the narrow table, for launches that throughput bounds (chains
// of equal length).  The wide table (FSMP_DESIGN_GROUP_DEVMEM_WIDE) gives each chain 2-4x the
// lanes, a whole wavefront from capacity 64 up: for launches whose longest chains set their
// duration (per-waveform sweep counts up to 8x the shortest), where a wider group shortens
// each of their sweeps (measured on the uneven-window workload: 1.38 s per step narrow, 0.92 s
// wide from capacity 96 up).
struct GroupCfg {
  int kcap, lpc, wpb;
};
static const GroupCfg kGroup[] = {{16, 16, 4}, {32, 32, 4}, {48, 64, 3}, {64, 64, 4}};
static const GroupCfg kGroupDM[] = {{16, 4, 4},  {32, 4, 4},   {48, 16, 2},  {64, 32, 4},
                                    {96, 16, 2}, {128, 32, 4}, {160, 32, 4}, {192, 32, 2}};
static const GroupCfg kGroupDMWide[] = {{32, 16, 4}, {48, 32, 4},  {64, 64, 4},  {96, 64, 4},
                                        {128, 64, 4}, {160, 64, 4}, {192, 64, 2}};
// the FP32 form keeps eight vectors per chain in LDS: two wavefronts per workgroup at the
// capacities of 4-lane groups (at four, capacity 32 would need 168 KB)
static const GroupCfg kGroupDMF32[] = {{16, 4, 2},  {32, 4, 2},   {64, 32, 4},  {96, 64, 4},
                                       {128, 64, 4}, {160, 64, 4}, {192, 64, 2}};
// its wide groups: 16 lanes per chain at the two smallest capacities (a quarter of the sweep
// latency of the 4-lane groups, which matters where one event's chains finish together);
// from capacity 64 up its groups are already 32-64 lanes wide
static const GroupCfg kGroupDMF32Wide[] = {{16, 16, 4}, {32, 16, 4}};

// the vectors of a chain's LDS block (ChainLayout::kVec); the corrected FP64 form (and with it
// group_dm_ws_doubles' exact G) from capacity 48 up
static_assert(ChainLayout<48, true>::kCorr && !ChainLayout<32, true>::kCorr && ChainLayout<64, true, false, true>::kCorr,
              "the host's sizes assume the corrected FP64 form at capacities 48 and up");
static int chain_vectors(int kcap, bool hg, bool f32, bool mcp) {
  if (f32) return ChainLayout<64, true, true>::kVec;
  return (hg && kcap >= 48) ? ChainLayout<64, true>::kVec : ChainLayout<16, true>::kVec;
}

static size_t chain_lds_bytes(const GroupCfg &g, int M, int sub, bool hg, bool f32 = false, bool mcp = false) {
  const int cpb = g.wpb * (64 / g.lpc);
  const size_t per = (hg ? 0 : (size_t)g.kcap * g.kcap) + (size_t)ChainLayout<16, true, false, false>::kAcc +
                     (size_t)chain_vectors(g.kcap, hg, f32, mcp) * (size_t)g.kcap +
                     ((size_t)g.kcap + 1) / 2 * (mcp ? 2 : 1);
  return sizeof(double) * ((size_t)M * (1 + sub) + (size_t)g.kcap + 2 + (size_t)cpb * per);
}

bool chain_kcap_supported(int kcap, int M, int sub) {
  for (const GroupCfg &g : kGroup)
    if (g.kcap == kcap) return chain_lds_bytes(g, M, sub, false) <= 160 * 1024;
  return false;
}

bool chain_dm_supported(int kcap, int M, int sub, bool f32, bool mcp, bool wide) {
  if (f32 && mcp) return false;
  if (wide && f32) {
    for (const GroupCfg &g : kGroupDMF32Wide)
      if (g.kcap == kcap) return chain_lds_bytes(g, M, sub, true, true, false) <= 160 * 1024;
    return false;
  }
  if (wide) {
    if (mcp) return false;
    for (const GroupCfg &g : kGroupDMWide)
      if (g.kcap == kcap) return chain_lds_bytes(g, M, sub, true, false, false) <= 160 * 1024;
    return false;
  }
  if (f32) {
    // no capacity 48: the precision form runs it at 64
    for (const GroupCfg &g : kGroupDMF32)
      if (g.kcap == kcap) return chain_lds_bytes(g, M, sub, true, true, false) <= 160 * 1024;
    return false;
  }
  for (const GroupCfg &g : kGroupDM)
    if (g.kcap == kcap) return chain_lds_bytes(g, M, sub, true, false, mcp) <= 160 * 1024;
  return false;
}

// H (FP64, with the exact G from capacity 48 up; or FP32 plus the FP64 refresh matrix and the
// exact G) of every chain, in tiles of a wavefront
size_t group_dm_ws_doubles(int kcap, int64_t n_list, bool f32, bool wide) {
  const GroupCfg *t = f32 ? (wide ? kGroupDMF32Wide : kGroupDMF32) : wide ? kGroupDMWide : kGroupDM;
  const int nt = f32    ? (wide ? (int)(sizeof kGroupDMF32Wide / sizeof *kGroupDMF32Wide)
                                : (int)(sizeof kGroupDMF32 / sizeof *kGroupDMF32))
                 : wide ? (int)(sizeof kGroupDMWide / sizeof *kGroupDMWide)
                        : (int)(sizeof kGroupDM / sizeof *kGroupDM);
  for (int q = 0; q < nt; ++q)
    if (t[q].kcap == kcap) {
      const int64_t cpw = 64 / t[q].lpc;
      const size_t k2 = (size_t)kcap * kcap;
      return (size_t)((n_list + cpw - 1) / cpw) * cpw * (f32 ? k2 / 2 + 2 * k2 : kcap >= 48 ? 2 * k2 : k2);
    }
  return 0;
}

size_t lane_ws_doubles(int kcap, int64_t n_list) {
  const size_t tiles = (size_t)((n_list + 63) / 64);
  return tiles * 64 * ((size_t)kcap * kcap + 5 * (size_t)kcap);
}

size_t lane_ws_ints(int kcap, int64_t n_list) {
  const size_t tiles = (size_t)((n_list + 63) / 64);
  return tiles * 64 * (2 * (size_t)kcap + 1);
}

hipError_t launch_chain_lane(int kcap, const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks) {
  // one lane per chain pays off only for small PE counts: instances at capacities 16 and 32
  switch (kcap) {
    case 16: return launch_chain_lane_t<16>(a, st, lanes, blocks);
    case 32: return launch_chain_lane_t<32>(a, st, lanes, blocks);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_chain(int kcap, const ChainArgs &a, hipStream_t st, int32_t *lanes, int64_t *blocks) {
  switch (kcap) {
    case 16: return launch_chain_t<16, 16, 4, false>(a, st, lanes, blocks);
    case 32: return launch_chain_t<32, 32, 4, false>(a, st, lanes, blocks);
    case 48: return launch_chain_t<48, 64, 3, false>(a, st, lanes, blocks);
    case 64: return launch_chain_t<64, 64, 4, false>(a, st, lanes, blocks);
    default: return hipErrorInvalidValue;
  }
}

// instances must match kGroupDM (kGroupDMWide for `wide`, kGroupDMF32 and kGroupDMF32Wide for
// the FP32 form; no wide groups for the mixture law)
hipError_t launch_chain_dm(int kcap, bool fp32, bool wide, const ChainArgs &a, hipStream_t st, int32_t *lanes,
                           int64_t *blocks) {
  if (wide && fp32) {
    if (a.md.n_mix > 0 || a.force) return hipErrorInvalidValue;
    switch (kcap) {
      case 16: return launch_chain_t<16, 16, 4, true, false, true>(a, st, lanes, blocks);
      case 32: return launch_chain_t<32, 16, 4, true, false, true>(a, st, lanes, blocks);
      default: return hipErrorInvalidValue;
    }
  }
  if (wide) {
    if (a.md.n_mix > 0) return hipErrorInvalidValue;
    if (a.force) {
      // replay with the wide groups, capacities from 64 up
      switch (kcap) {
        case 64: return launch_chain_t<64, 64, 4, true, true>(a, st, lanes, blocks);
        case 96: return launch_chain_t<96, 64, 4, true, true>(a, st, lanes, blocks);
        case 128: return launch_chain_t<128, 64, 4, true, true>(a, st, lanes, blocks);
        case 160: return launch_chain_t<160, 64, 4, true, true>(a, st, lanes, blocks);
        case 192: return launch_chain_t<192, 64, 2, true, true>(a, st, lanes, blocks);
        default: return hipErrorInvalidValue;
      }
    }
    switch (kcap) {
      case 32: return launch_chain_t<32, 16, 4, true>(a, st, lanes, blocks);
      case 48: return launch_chain_t<48, 32, 4, true>(a, st, lanes, blocks);
      case 64: return launch_chain_t<64, 64, 4, true>(a, st, lanes, blocks);
      case 96: return launch_chain_t<96, 64, 4, true>(a, st, lanes, blocks);
      case 128: return launch_chain_t<128, 64, 4, true>(a, st, lanes, blocks);
      case 160: return launch_chain_t<160, 64, 4, true>(a, st, lanes, blocks);
      case 192: return launch_chain_t<192, 64, 2, true>(a, st, lanes, blocks);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.md.n_mix > 0) {
    if (a.force || fp32) return hipErrorInvalidValue;
    switch (kcap) {
      case 16: return launch_chain_t<16, 4, 4, true, false, false, true>(a, st, lanes, blocks);
      case 32: return launch_chain_t<32, 4, 4, true, false, false, true>(a, st, lanes, blocks);
      case 48: return launch_chain_t<48, 16, 2, true, false, false, true>(a, st, lanes, blocks);
      case 64: return launch_chain_t<64, 32, 4, true, false, false, true>(a, st, lanes, blocks);
      case 96: return launch_chain_t<96, 16, 2, true, false, false, true>(a, st, lanes, blocks);
      case 128: return launch_chain_t<128, 32, 4, true, false, false, true>(a, st, lanes, blocks);
      case 160: return launch_chain_t<160, 32, 4, true, false, false, true>(a, st, lanes, blocks);
      case 192: return launch_chain_t<192, 32, 2, true, false, false, true>(a, st, lanes, blocks);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.force) {
    switch (kcap) {
      case 16: return launch_chain_t<16, 4, 4, true, true>(a, st, lanes, blocks);
      case 32: return launch_chain_t<32, 4, 4, true, true>(a, st, lanes, blocks);
      case 48: return launch_chain_t<48, 16, 2, true, true>(a, st, lanes, blocks);
      case 64: return launch_chain_t<64, 32, 4, true, true>(a, st, lanes, blocks);
      case 96: return launch_chain_t<96, 16, 2, true, true>(a, st, lanes, blocks);
      case 128: return launch_chain_t<128, 32, 4, true, true>(a, st, lanes, blocks);
      case 160: return launch_chain_t<160, 32, 4, true, true>(a, st, lanes, blocks);
      case 192: return launch_chain_t<192, 32, 2, true, true>(a, st, lanes, blocks);
      default: return hipErrorInvalidValue;
    }
  }
  if (fp32) {
    // instances must match kGroupDMF32
    switch (kcap) {
      case 16: return launch_chain_t<16, 4, 2, true, false, true>(a, st, lanes, blocks);
      case 32: return launch_chain_t<32, 4, 2, true, false, true>(a, st, lanes, blocks);
      case 64: return launch_chain_t<64, 32, 4, true, false, true>(a, st, lanes, blocks);
      case 96: return launch_chain_t<96, 64, 4, true, false, true>(a, st, lanes, blocks);
      case 128: return launch_chain_t<128, 64, 4, true, false, true>(a, st, lanes, blocks);
      case 160: return launch_chain_t<160, 64, 4, true, false, true>(a, st, lanes, blocks);
      case 192: return launch_chain_t<192, 64, 2, true, false, true>(a, st, lanes, blocks);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kcap) {
    case 16: return launch_chain_t<16, 4, 4, true>(a, st, lanes, blocks);
    case 32: return launch_chain_t<32, 4, 4, true>(a, st, lanes, blocks);
    case 48: return launch_chain_t<48, 16, 2, true>(a, st, lanes, blocks);
    case 64: return launch_chain_t<64, 32, 4, true>(a, st, lanes, blocks);
    case 96: return launch_chain_t<96, 16, 2, true>(a, st, lanes, blocks);
    case 128: return launch_chain_t<128, 32, 4, true>(a, st, lanes, blocks);
    case 160: return launch_chain_t<160, 32, 4, true>(a, st, lanes, blocks);
    case 192: return launch_chain_t<192, 32, 2, true>(a, st, lanes, blocks);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fsmp
