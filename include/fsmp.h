/*
 * fsmp.h -- C ABI of libfsmp.so: batched reversible-jump MCMC over the photo-electron
 * (PE) sequences of PMT waveforms, the Fast Stochastic Matching Pursuit (FSMP) of
 * Xu et al., "The Fast Stochastic Matching Pursuit for Neutrino and Dark Matter
 * Experiments", run in HIP kernels on one MI355X (gfx950).
 *
 * Problem (Sec. 1 eq. waveform; Sec. 2.1-2.2): a waveform w of L_w samples at
 * 1 sample per ns is  w(t) = sum_i q_i V(t - t_i) + eps(t),  eps ~ N(0, sigma_eps^2)
 * white; V is an ex-Gaussian single-electron response (Sec. 3); the charges are
 * q_i ~ N(mu_q, sigma_q^2) and are integrated out (App. A, eq. mgauss); the PE times
 * z = {t_i} follow a Poisson point process of intensity lambda0 * phi(t - t0)
 * (eq. pzmu).  The library samples z and t0 by a Gibbs sweep: t0 by
 * Metropolis-Hastings, then one birth / death / update jump of z (Sec. 2.4,
 * eqs. birth, death, update, delta-nu), with J = 1/4 and the empty-sequence rule.
 *
 * Conventions shared by every entry point
 *   - times are in samples (ns at 1 GS/s); PE times live on the grid t = g / grid_sub
 *     with integer g; the solution space T of a waveform is a range [g_lo, g_hi]
 *     inside [0, grid_sub * L_w - 1] (default: the whole window).
 *   - the target is the grid-binned Poisson process on T with normaliser
 *     exp(-Lambda_T(t0)), Lambda_T(t0) = lambda0 / grid_sub * sum_{g in T} phi(g / grid_sub - t0),
 *     truncated at K_max PEs (a birth at K_max is rejected and flagged).
 *   - the t0 prior is uniform on [t0_min, t0_max].
 *   - every chain draws its random numbers from Philox4x32-10 (Salmon et al., SC'11)
 *     with key (seed lo, seed hi) and counter (step, block, uid lo, uid hi),
 *     uid = wave_id * n_chains + chain: a chain's result does not depend on the batch
 *     it runs in, on the launch shape or on the other chains.
 *   - pointers marked "device" are HIP device memory of the context's device; pointers
 *     marked "host" are ordinary host memory read during the call.  The caller owns every
 *     buffer it passes; the context owns its tables and workspace.
 *   - work is enqueued on the HIP stream passed as `hip_stream` (NULL = the null stream);
 *     outputs are valid once that stream has reached the end of the call's work.
 *   - a function that fails returns a negative fsmp_status and leaves a message for
 *     fsmp_last_error(); problems of single waveforms do not fail a call: they set bits in
 *     that chain's status word (FSMP_ST_*).
 *   - one context serves one host thread at a time.
 */
#ifndef FSMP_H
#define FSMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSMP_OK = 0,
  FSMP_EINVAL = -1,   /* invalid argument (message in fsmp_last_error) */
  FSMP_ENOMEM = -2,   /* device or host allocation failed */
  FSMP_EDEVICE = -3,  /* HIP runtime error or no usable gfx950 device */
  FSMP_ENOTSUP = -4,  /* valid request this build does not provide (e.g. K_max above the largest kernel) */
  FSMP_EBUSY = -5     /* reserved */
} fsmp_status;

enum { FSMP_PHI_EXP = 0, FSMP_PHI_BIEXP = 1 };
enum { FSMP_FP64 = 0, FSMP_FP32_REFRESH = 1 };

/* record_flags */
enum {
  FSMP_REC_TRACE = 1u,  /* per recorded step (N, t0, Q) into fsmp_samples.trace */
  FSMP_REC_LOG = 2u,    /* one fsmp_logrec per step into fsmp_samples.log (for replay checks) */
  FSMP_REC_CHARGE = 4u  /* per recorded step the PE list and one charge draw into
                           fsmp_samples.zdraw / qdraw (needs thin > 0) */
};

/* per-chain status bits */
enum {
  FSMP_ST_KMAX = 1u,      /* a birth was rejected because N reached K_max */
  FSMP_ST_NONFINITE = 2u, /* the waveform holds a NaN or an infinity: the chain did not run */
  FSMP_ST_DRIFT = 4u,     /* FP32 form: refresh found drift above the bound */
  FSMP_ST_EMPTY_T = 8u,   /* empty solution space: no birth is possible */
  FSMP_ST_FACTOR = 16u    /* a Schur complement was not positive: proposal rejected */
};

/* Single-electron response (Sec. 3, ex-Gaussian): V(t) = A f(t) / max f, with f the
 * ex-Gaussian density of a N(mu, sigma^2) shifted by an Exp(mean tau) (the paper's form
 * has mu = 4 sigma); V = 0 outside [0, support).  support = 0 picks the smallest multiple
 * of 16 samples beyond which V / A < 1e-6.  amplitude = 0 switches the data term off
 * (every delta-nu is exactly 0: the sampler then draws from the prior). */
typedef struct {
  double mu, sigma, tau; /* ns, sigma > 0, tau > 0 */
  double amplitude;      /* peak height; 1 = peak normalised */
  int32_t support;       /* samples, 0 = automatic, at most 512 */
} fsmp_ser;

/* Light curve phi (Sec. 3): EXP  phi(t) = e^{-t/tau_decay} / tau_decay;
 * BIEXP phi(t) = (tau_rise + tau_decay) / tau_decay^2 (1 - e^{-t/tau_rise}) e^{-t/tau_decay};
 * phi(t) = 0 for t < 0.  t0 has the uniform prior [t0_min, t0_max] (eq. t0prior);
 * t0_min == t0_max fixes t0. */
typedef struct {
  int32_t kind;
  double tau_rise, tau_decay;
  double t0_min, t0_max;
} fsmp_intensity;

/* Sampler settings.  Charge model N(mu_q, sigma_q^2) (Sec. 2.1); noise sigma_eps; grid
 * step 1 / grid_sub samples; jump probabilities J, J, 1 - 2J (Sec. 2.4); t0 random-walk
 * step N(0, t0_step_sd^2) and update shift N(0, shift_sd^2) rounded to the grid.
 * Steps [0, burn_in) are not recorded; accumulators use floor(sqrt(n_steps - burn_in))
 * batches for the batch-means MCSE.  Both forms rebuild G^-1 = (A^T A + rho I)^-1 and the
 * charge means x = G^-1 b from scratch in FP64 every refresh_M sweeps (0: never), except the
 * FP64 form's corrected kernels below, which need no rebuild.
 * precision: FSMP_FP64 (all FP64; from PE capacity 48 up, in the device-memory design the
 * kernels run there, with the exact G kept beside G^-1 and the residual s = b - G x of the
 * charge means recomputed after every accepted move, so that gamma^T G^-1 b and x_j enter
 * delta-nu as gamma^T x + eta^T s and x_j + h^T s, eta = G^-1 gamma, h = row j of G^-1:
 * FP64 through an explicit inverse alone leaves x with an error of about kappa(G) eps,
 * about 1e-8 of delta-nu on pile-up windows at K ~ 100) or
 * FSMP_FP32_REFRESH: G^-1 stored in FP32 and updated by its edits (computed in FP64, stored
 * rounded), with the exact G kept in FP64; each proposal's delta-nu is evaluated from the
 * FP32 G^-1 with a two-term residual correction against G (App. A, eqs. 11-18: the quantities
 * delta^2, u+, omega and x_j of the PE-space form), whose last term bounds the error left; the
 * proposal is re-evaluated from an FP64 rebuild of G^-1 when that bound exceeds
 * 1e-5 max(1, |delta-nu|) or could turn the accept decision, and at every recorded charge
 * draw. */
typedef struct {
  double sigma_eps, mu_q, sigma_q;
  int32_t grid_sub;      /* 1..16 */
  double jump_J;         /* 0 < J < 1/2 */
  double t0_step_sd, shift_sd;
  int32_t k_max;         /* default PE cap when fsmp_batch.kmax is NULL */
  int32_t n_steps, n_chains, burn_in, thin;
  int32_t precision, refresh_M;
  uint32_t record_flags;
  uint64_t seed;
  /* MCP-PMT charge model (Sec. 2.1, eq. mcp-multi-norm; Sec. 2.4, eq. mcp; App. A for
   * MCP-PMTs): n_mix = 0 uses N(mu_q, sigma_q^2); 1..8 a Gaussian mixture in which every PE
   * carries a component e with probability mix_weight[e] (positive, summing to 1 within
   * 1e-9), charge mean mix_mu[e] and standard deviation mix_sigma[e] > 0.  A born PE's
   * component, and an updated PE's new one, are drawn from the mixture weights (Philox
   * word 7 of the step, inverse CDF with the weights accumulated in index order); the
   * weights cancel from every acceptance, which keeps the dynode form with delta-nu of the
   * per-PE charge law (G = A^T A + diag(rho_e), b = A^T w + rho_e mu_e, rho_e =
   * sigma_eps^2 / sigma_e^2).  The mixture form runs the FP64 lane-group kernels with G^-1 in
   * device memory at every capacity; FP32 storage, replay and start lists are not offered
   * with it (FSMP_ENOTSUP). */
  int32_t n_mix;
  double mix_weight[8], mix_mu[8], mix_sigma[8];
} fsmp_config;

/* One batch of waveforms (ragged).  wave: device, float32, the concatenated samples;
 * offsets: host, n_wave + 1 int64 sample offsets (offsets[0] = 0, non-decreasing, every
 * window 1..65536 samples); lambda: host, lambda0 >= 0 per waveform (the intensity's
 * scale, eq. pzmu); kmax: host or NULL, PE cap per waveform (1..192); g_range: host or
 * NULL, [g_lo, g_hi] per waveform inside [0, grid_sub * L_w - 1] (g_lo > g_hi = empty T);
 * t0_init: host or NULL (default (t0_min + t0_max) / 2); wave_id: host or NULL, the
 * identity that keys the random stream (default: the index in the batch); n_steps: host
 * or NULL, sweeps per waveform (1..cfg.n_steps; NULL = cfg.n_steps for all), each with
 * burn-in floor(n_steps * cfg.burn_in / cfg.n_steps) -- it needs fsmp_samples.rec_steps
 * so that fsmp_posterior divides by each chain's own number of recorded sweeps.
 * z_init, z_init_offsets: host or NULL (every chain starts from the empty list), the initial
 * PE sequence of every chain (Sec. 2.3: an initial guess of z, e.g. from a deconvolution;
 * Sec. 3.2: chains started from different sequences): chain c = i * n_chains + k starts
 * from the grid indices z_init[z_init_offsets[c] .. z_init_offsets[c + 1]), n_wave *
 * n_chains + 1 offsets from 0.  Each list holds at most the waveform's kmax PEs, each inside
 * the waveform's T where phi(g / grid_sub - t0_init) > 0, and needs lambda > 0; G^-1 and
 * the charges of the list are built before the first sweep, which draws no random numbers
 * for it (a chain's stream is the same as from the empty list).
 * Why the per-waveform metadata is host memory (the waveforms are device memory): the host
 * validates it (ranges, T inside the window, start lists against the prior) and uses it to
 * plan the call -- the capacity bucket of every waveform, the chain order within a bucket
 * (sweep-count bins, then lambda), the workspace size -- before any launch, so it would
 * read it back from the device otherwise.  fsmp_sample copies the planned arrays (24-40
 * bytes per waveform, 12 MB for 250,000 waveforms) to the device on the caller's stream
 * through the context's pinned staging buffer: that copy is part of the call and of any
 * time measured around it (its stream order keeps it ahead of the kernels; the call does
 * not wait for it, but reuses the staging buffer only once the previous call's copy has
 * finished).  fsmp_sample_noalloc copies from the caller's host memory directly. */
typedef struct {
  int64_t n_wave;
  const float *wave;
  const int64_t *offsets;
  const double *lambda;
  const int32_t *kmax;
  const int32_t *g_range;
  const double *t0_init;
  const uint64_t *wave_id;
  const int32_t *n_steps;
  const int32_t *z_init;
  const int64_t *z_init_offsets;
} fsmp_batch;

/* One record per step of one chain (FSMP_REC_LOG). */
typedef struct {
  int32_t move;     /* 1 birth, 2 death, 3 update */
  int32_t flags;    /* bit0 proposal valid (delta-nu computed), bit1 jump accepted, bit2 t0 accepted */
  int32_t j;        /* index of the removed / moved PE, -1 for a birth */
  int32_t g;        /* grid index of the new PE, -1 for a death */
  double t0;        /* t0 after the Metropolis-Hastings half-step */
  double dnu;       /* delta-nu = log p(w|z') - log p(w|z) of the proposal (0 if not valid) */
  double log_alpha; /* log of the acceptance (-inf if not valid) */
} fsmp_logrec;

/* Outputs of fsmp_sample, caller-allocated device buffers; chain c of waveform i is row
 * i * n_chains + c.  kz >= every waveform's kmax is the row length of z and charge.
 *   n_pe[chain]           final N
 *   t0[chain]             final t0
 *   z[chain][kz]          final PE grid indices (list order), -1 beyond N
 *   charge[chain][kz]     E[q | z, w] of the final z (Bayesian linear regression), 0 beyond N
 *   acc[chain][12]        after burn-in: sum N, N^2, Q, Q^2, t0, t0^2, then sum_b S_b and
 *                         sum_b S_b^2 of the batch sums S_b of N, Q and t0 (Q = sum of E[q|z,w])
 *   nhist[chain][kz + 1]  after burn-in: steps with N = k
 *   counts[chain][8]      proposals / accepts of t0, birth, death, update (all steps)
 *   status[chain]         FSMP_ST_* bits
 *   log                   NULL, or [chain][n_steps] fsmp_logrec when FSMP_REC_LOG
 *   trace                 NULL, or [chain][n_rec][3] (N, t0, Q) every `thin` recorded steps
 *                         when FSMP_REC_TRACE, n_rec = ceil((n_steps - burn_in) / thin)
 *   work                  NULL, or [chain][5] work counters over all steps, K the PE count
 *                         before the move, j the removed or moved PE's index (from 0):
 *                         [0] the words of a packed Cholesky factor a proposal must read
 *                             (birth K(K+1)/2 + 2K + 3, death (K-j)(K-j+1)/2 + 1, update both
 *                             with the birth on K - 1 PEs), [1] the words an accepted move
 *                             must edit (birth K + 3, death (K-1-j)(K-j) + K(K+1)/2, update
 *                             both), [2] the G^-1 elements this library's proposals read
 *                             (K^2 per K x K mat-vec, K for a row), [3] the G^-1 and G elements
 *                             its accepted edits read and write (2 K^2 per edit, K^2 more for
 *                             the residual of the corrected FP64 form), [4] FP64
 *                             re-evaluations of the FP32 form
 *   rec_steps             NULL, or [chain] the number of recorded sweeps (after burn-in) of
 *                         the chain; required with per-waveform sweep counts, read by
 *                         fsmp_posterior when present
 *   qdraw, zdraw          NULL, or [chain][n_rec][kz] when FSMP_REC_CHARGE: at every recorded
 *                         step (the steps of `trace`) the PE grid indices (-1 beyond N) and one
 *                         draw of the charges from their conditional law given z (Sec. 2.1
 *                         charge model, App. A eq. mgauss), q ~ N(x, sigma_eps^2 G^-1), as
 *                         q = x + sigma_eps R xi with R the upper-triangular factor of
 *                         G^-1 = R R^T (R = L^-T for G = L L^T) and xi standard normals, PE k
 *                         of the list from Philox block 2 + k/2 of that step (Box-Muller of
 *                         words 0 and 1: cosine for even k, sine for odd k); 0 beyond N, NaN
 *                         (with FSMP_ST_FACTOR) if the factorisation fails.  The draw reads
 *                         the maintained G^-1 (its FP64 rebuild in the precision form).  Costs O(K^3)
 *                         per record; FP64 scratch of kcap (kcap + 1) words per chain is allocated
 *                         by fsmp_sample while the flag is set.
 *   occ                   NULL, or the grid occupancy (Sec. 2.2: the PE sequence as a point
 *                         pattern on the grid of T): per waveform one int32 per grid point of its
 *                         window, the row of waveform i at occ + grid_sub * offsets[i] with
 *                         grid_sub * L_i entries (grid_sub * offsets[n_wave] in all), counting
 *                         over the waveform's chains and recorded sweeps the PEs at each grid
 *                         point (with multiplicity; a row sums to the sum of N over the recorded
 *                         steps).  fsmp_sample zeroes the rows; FSMP_EINVAL if n_chains x
 *                         (n_steps - burn_in) x kmax could overflow a count. */
typedef struct {
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
  double *work;
  double *qdraw;
  int32_t *zdraw;
  int32_t *rec_steps;
  int32_t *occ;
  int32_t *comp;   /* NULL, or [chain][kz] with a mixture: the final PEs' components, -1 beyond N */
} fsmp_samples;

/* Posterior summaries per waveform (device buffers, caller-allocated): for (N, Q, t0)
 * the mean, variance and batch-means MCSE pooled over the waveform's chains; P(N = k)
 * for k <= kz (NULL to skip); acceptance rates of t0, birth, death, update; the OR of
 * the chains' status words; optionally the posterior occupancy of the grid, the expected
 * number of PEs at every grid point (fsmp_samples.occ over the waveform's recorded
 * (chain, sweep) pairs, in the same layout), which needs fsmp_samples.occ and the batch's
 * host offsets.
 *
 * Convergence (Sec. 3.2): rhat is the potential scale reduction of Gelman and Rubin over the
 * waveform's C chains of S recorded sweeps, without the degrees-of-freedom factor or chain
 * splitting: with chain means m_i and unbiased chain variances s_i^2, W = mean s_i^2,
 * B = S / (C - 1) sum_i (m_i - m)^2, R = sqrt(((S - 1) / S W + B / S) / W); 1 when every chain
 * is constant at one value, inf when they are constant at different values, NaN for C < 2
 * or S < 2.  The batch-means mcse reads only within-chain correlation and underestimates
 * the error of short, slowly mixing chains; mcse_chains does not, given enough chains.
 *
 * lambda_hat (Sec. 2.2, eq. reduce-mu0): the maximiser over lambda >= 0 of
 * f(lambda) = -(lambda - lambda0) + log sum_k h_k (lambda / lambda0)^k, h the waveform's
 * N histogram over all chains (the whole-line normaliser e^-lambda of eq. pzmu).  Its
 * maxima solve lambda = m(lambda), the mean of k under the weights h_k (lambda / lambda0)^k,
 * with d = m - lambda going from + to -; all lie between the smallest and largest sampled
 * N (k_lo, k_hi).  A single sampled N is returned as is; otherwise d is evaluated on 64
 * evenly spaced points of [k_lo, k_hi], every interval where d goes from > 0 to <= 0 is
 * bisected to the root, lambda = 0 is a candidate when k_lo = 0 and d <= 0 at the second
 * point, and the candidate with the largest f wins (the smallest of equals). */
typedef struct {
  double *mean;      /* [n_wave][3] */
  double *var;       /* [n_wave][3] */
  double *mcse;      /* [n_wave][3] */
  double *p_n;       /* [n_wave][kz + 1] or NULL */
  double *accept;    /* [n_wave][4] */
  uint32_t *status;  /* [n_wave] */
  double *occupancy; /* NULL, or grid_sub * offsets[n_wave] doubles, rows as fsmp_samples.occ */
  const int64_t *offsets; /* host, n_wave + 1: the batch's sample offsets (with occupancy) */
  double *rhat;        /* NULL, or [n_wave][3]: Gelman-Rubin R of N, Q, t0 (see below) */
  double *mcse_chains; /* NULL, or [n_wave][3]: MCSE of the pooled means from the spread of the
                          chain means, sqrt(sum_i (m_i - m)^2 / (C (C - 1))); NaN for C < 2 */
  double *lambda_hat;  /* NULL, or [n_wave][2]: lambda-hat_FSMP (eq. reduce-mu0) and
                          lambda-hat_Q = E[Q] / mu_q */
  const double *lambda; /* host, n_wave: the batch's lambda0 (with lambda_hat) */
} fsmp_posterior_out;

/* Timing of the kernels of the last fsmp_sample call (HIP events on its stream). */
typedef struct {
  char name[32];     /* kernel */
  int32_t kcap;      /* PE capacity of the instance (0 for non-chain kernels) */
  int32_t lanes;     /* lanes per chain */
  int64_t chains;    /* chains the launch ran */
  int64_t blocks;    /* workgroups */
  double ms;         /* duration between the events around the launch */
} fsmp_timing;

typedef struct fsmp_ctx fsmp_ctx;

/* Create a context on HIP device `device`: validates the model, builds the SER table
 * V(m / grid_sub) and the stationary overlap table sum_n V(n - g1/sub) V(n - g2/sub) in
 * FP64 on the host, and uploads them.  Returns FSMP_EINVAL for a bad model,
 * FSMP_EDEVICE if the device is missing or not gfx950.  *out is NULL on failure. */
fsmp_status fsmp_create(fsmp_ctx **out, const fsmp_ser *ser, const fsmp_intensity *phi, const fsmp_config *cfg,
                        int device);

/* Device workspace (bytes) fsmp_sample would hold for this batch with the context's current
 * designs and configuration: batch metadata, the matched filter over every solution space,
 * the chain state of each PE-capacity bucket (K_cap^2 words of G^-1 per chain in the
 * device-memory designs, nothing for G^-1 in LDS), charge-draw scratch when recorded, and
 * the light-curve table.  The context grows its workspace to this on demand and keeps it.
 * Host arrays of `batch` are read (wave is not); 0 for an invalid batch. */
size_t fsmp_workspace_bytes(const fsmp_ctx *ctx, const fsmp_batch *batch);

/* Run cfg.n_chains chains of cfg.n_steps Gibbs sweeps for every waveform of the batch and
 * write `out`.  Validates every host array first (FSMP_EINVAL, nothing enqueued); returns
 * FSMP_ENOTSUP if a kmax exceeds 192 or the SER support does not fit a kernel.  The work is
 * enqueued on `hip_stream` (a hipStream_t; NULL = the null stream) and is complete when that
 * stream is: the PE-capacity buckets of the batch run concurrently, on `hip_stream` and on
 * the context's own side streams (GPU_MAX_HW_QUEUES lanes in all, default 4, read at each
 * call; HIP reads the same variable once when it starts, and each lane needs a hardware queue
 * of its own, so a process that sets it to 8 before HIP starts runs every bucket on a lane of
 * its own), forked from and joined back into `hip_stream` with events; with fewer lanes than
 * buckets, buckets are dealt to the lanes by estimated cost (after fsmp_autotune, its trial
 * times of the chosen designs).  The calls of one context share its workspace: give them
 * one stream, or order their streams, so that two calls never run on the device at once. */
fsmp_status fsmp_sample(fsmp_ctx *ctx, const fsmp_batch *batch, const fsmp_samples *out, void *hip_stream);

/* fsmp_sample for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same validation, kernels and outputs
 * as fsmp_sample (identical results for the same context and batch), but the call allocates
 * nothing -- no device, pinned or host memory, streams or events.  Its device workspace
 * (batch metadata, matched filter, chain lists, chain state, charge-draw scratch) is one
 * static array of 256 MiB per GPU in the library's code object, held until the process
 * ends, whose address fsmp_create takes on the context's device; its host-side arrays are
 * static too.  Limits: at most 65,536 waveforms and 262,144 chains, a workspace within the
 * 256 MiB (fsmp_workspace_bytes gives it, to within alignment), and solution spaces no longer
 * than the context's light-curve table (16,384 grid points at creation; a longer batch
 * through fsmp_sample grows it); FSMP_EINVAL / FSMP_ENOTSUP beyond them, with the reason in
 * fsmp_last_error.  The PE-capacity buckets run one after the other on `hip_stream` (no side
 * streams), no kernel timings are taken, and the batch's host arrays are uploaded with
 * hipMemcpyAsync from the caller's (pageable) memory, which the copies have read when the
 * call returns.  Every call in the process shares the host arrays and every call on a GPU
 * shares that GPU's scratch array, whose contents the previous call leaves: calls are
 * serialised on the host, and the caller must not let the device work of two calls on one
 * GPU overlap (one stream, or streams ordered by events); nothing in the scratch needs to
 * start at zero. */
fsmp_status fsmp_sample_noalloc(fsmp_ctx *ctx, const fsmp_batch *batch, const fsmp_samples *out, void *hip_stream);

/* Replay (a check of the sampler's delta-nu along a given path; Sec. 2.4 moves, App. A
 * delta-nu): like fsmp_sample, but every chain follows the recorded proposals of `log`
 * (device, [chain][cfg.n_steps] fsmp_logrec, the FSMP_REC_LOG layout, from this library
 * or written elsewhere) instead of its own draws: at each step t0 is set to the record's
 * t0, the record's move, index and grid point are proposed if the record is flagged
 * valid (bit 0), and the record's accept bit (bit 1) decides.  dnu and log_alpha (device,
 * [chain][cfg.n_steps]) receive what the kernel computes for each evaluated proposal; 0
 * and -inf for steps not evaluated (not flagged valid, malformed, or invalid here, e.g. a
 * Schur complement that is not positive).  Runs the lane-group kernels with G^-1 in
 * device memory at every capacity (the wide ones where the context has chosen them at
 * capacity 64 and up), FP64 form only (FSMP_ENOTSUP otherwise).  `out`
 * receives the final state and accumulators as in fsmp_sample.  Errors as fsmp_sample. */
fsmp_status fsmp_replay(fsmp_ctx *ctx, const fsmp_batch *batch, const fsmp_logrec *log, double *dnu,
                        double *log_alpha, const fsmp_samples *out, void *hip_stream);

/* Reduce the per-chain accumulators of fsmp_sample's output into per-waveform summaries
 * (device kernel on `hip_stream`). */
fsmp_status fsmp_posterior(fsmp_ctx *ctx, int64_t n_wave, const fsmp_samples *in, fsmp_posterior_out *out,
                           void *hip_stream);

/* Initial state by deconvolution (Sec. 2.3), for fsmp_batch's z_init, g_range, t0_init and
 * lambda: n_iter iterations of Lucy's multiplicative update of qhat over tau = -L_V + 1 ..
 * L_w - 1 (whole samples), with the SER sampled at whole samples and normalised to unit
 * sum (so that qhat is in units of one PE's charge), the data clipped at 0 and a uniform
 * start with the data's total; then
 *   z         {tau >= 0 : qhat(tau) > threshold} (the paper takes 0.1), the kmax largest
 *             when more pass (ties: earlier tau), in time order, as grid indices
 *             grid_sub * tau, without PEs at or before t0;
 *   t0        the first PE time minus half a grid step, held inside [t0_min, t0_max];
 *   g_range   T = [t_min - margin, t_max + margin] (the paper takes 4 ns) on the grid,
 *             clipped to the window; g_lo > g_hi (an empty T: the waveform is taken as
 *             no PE) when no point passes;
 *   cut       the sample range [t_min - margin, t_max + margin + L_V] of the waveform
 *             that the paper keeps (clipped; the whole window when no point passes);
 *   lambda    the total of qhat, the initial intensity scale.
 * Outputs are device buffers; qhat (NULL to skip) holds row i at offsets[i] + i (L_V - 1),
 * L_i + L_V - 1 entries.  FP64 throughout.  Windows are held in LDS: FSMP_ENOTSUP when the
 * longest does not fit (about 6,000 samples at L_V = 96).  kz >= every kmax. */
typedef struct {
  int32_t *z;       /* [n_wave][kz], -1 beyond n_pe */
  int32_t *n_pe;    /* [n_wave] */
  int32_t *g_range; /* [n_wave][2] */
  double *t0;       /* [n_wave] */
  double *lambda;   /* [n_wave] */
  int32_t *cut;     /* [n_wave][2] */
  double *qhat;     /* NULL or see above */
  int32_t kz;
} fsmp_lucy_out;

fsmp_status fsmp_lucy(fsmp_ctx *ctx, const fsmp_batch *batch, int32_t n_iter, double threshold, int32_t margin,
                      fsmp_lucy_out *out, void *hip_stream);

/* L_V, the SER support in samples of the context (the row length of the response the
 * deconvolution uses); -1 for a NULL context. */
int32_t fsmp_ser_support(const fsmp_ctx *ctx);

/* Kernel timings of the last fsmp_sample: waits for its kernels, writes up to `cap`
 * entries and returns how many kernels ran.  Timings are taken (HIP events recorded on
 * the call's stream around each launch, no synchronisation inside fsmp_sample) only
 * while fsmp_set_timing(ctx, 1) is in effect. */
int32_t fsmp_last_timings(const fsmp_ctx *ctx, fsmp_timing *out, int32_t cap);
fsmp_status fsmp_set_timing(fsmp_ctx *ctx, int32_t enable);

/* ------------------------------------------------------------------ kernel designs
 * Four implementations of the same chains (identical results up to rounding order):
 * FSMP_DESIGN_GROUP runs one chain per group of lanes with G^{-1} in LDS (PE capacities up
 * to 64); FSMP_DESIGN_LANE runs one chain per lane with G^{-1} interleaved in device
 * memory (capacities 16 and 32); FSMP_DESIGN_GROUP_DEVMEM runs one chain per (narrower)
 * group of lanes with G^{-1} in device memory, interleaved across the chains of a
 * wavefront, and only the vectors in LDS (every capacity, while the SER tables leave room
 * in LDS); FSMP_DESIGN_GROUP_DEVMEM_WIDE the same with 2-4x the lanes per chain (a whole
 * wavefront from capacity 64 up; capacities 32-192 in FP64 with the single charge law, 16
 * and 32 in the FP32-refresh form, 16 lanes per chain), for batches whose longest chains
 * set the launch's duration.  Capacities are 16, 32, 48, 64, 96, 128, 160, 192; a waveform
 * runs in the smallest one >= its kmax.  capacity 0 = every capacity that has the design.
 * FSMP_ENOTSUP if the requested pair does not exist.  The FP32-refresh form runs
 * FSMP_DESIGN_GROUP_DEVMEM and its wide groups (capacity 48 at 64); the mixture charge law
 * FSMP_DESIGN_GROUP_DEVMEM only; replays run FSMP_DESIGN_GROUP_DEVMEM, or
 * FSMP_DESIGN_GROUP_DEVMEM_WIDE where the context has it at capacity 64 and up. */
enum { FSMP_DESIGN_GROUP = 0, FSMP_DESIGN_LANE = 1, FSMP_DESIGN_GROUP_DEVMEM = 2, FSMP_DESIGN_GROUP_DEVMEM_WIDE = 3 };
fsmp_status fsmp_set_design(fsmp_ctx *ctx, int32_t capacity, int32_t design);
int32_t fsmp_get_design(const fsmp_ctx *ctx, int32_t capacity);

/* Autotuner: runs the whole batch for trial_steps sweeps once per design, each capacity
 * in that design where it exists (outputs discarded, HIP-event timings of each capacity's
 * launch, the capacities one after the other so that each time is the launch's own), then
 * keeps the fastest design per capacity in the context.  With per-waveform
 * sweep counts (batch->n_steps) every waveform's trial keeps its share of them, scaled to a
 * mean of trial_steps (at least 1), so that the trial weighs a launch's longest chains
 * against its total work as the full run does.
 * Allocates scratch outputs for the trial and synchronises `hip_stream`.  The FP32-refresh
 * form and the mixture law have one design, which it keeps. */
fsmp_status fsmp_autotune(fsmp_ctx *ctx, const fsmp_batch *batch, int32_t trial_steps, void *hip_stream);

/* Chain-length autotuner: runs the batch once for pilot_steps sweeps (the configured
 * burn-in fraction, outputs discarded), takes each waveform's batch-means MCSE of N from
 * the pilot and writes to steps_out (host, n_wave) the sweeps that bring it to
 * target_rel_mcse * max(1, mean N) under MCSE ~ 1 / sqrt(recorded sweeps), clamped to
 * [min_steps, min(max_steps, cfg.n_steps)] (a waveform whose pilot shows no variation gets
 * min_steps).  Pass the result as fsmp_batch.n_steps.  Allocates scratch and
 * synchronises `hip_stream`.  The MCSE of a short pilot is itself noisy: the result is a
 * budget, not a guarantee. */
fsmp_status fsmp_autotune_steps(fsmp_ctx *ctx, const fsmp_batch *batch, int32_t pilot_steps, double target_rel_mcse,
                                int32_t min_steps, int32_t max_steps, int32_t *steps_out, void *hip_stream);

/* HIP graph of one batch: makes a private context with ctx's model, configuration and
 * designs, uploads the batch's metadata into it (synchronising `hip_stream`), records the
 * prologue and chain kernels of fsmp_sample(batch, out) into a graph and instantiates it.
 * Each fsmp_graph_launch replays exactly that work (same results as the eager call): it
 * reads batch->wave and writes `out`'s buffers, which the caller keeps allocated until
 * fsmp_graph_destroy; the host arrays of `batch` may be freed after creation.  Calls on
 * ctx afterwards do not affect the graph.  Replays of one graph must not overlap in time
 * (they share the private workspace and `out`).  No memset nodes are recorded.  Errors
 * are reported on ctx. */
typedef struct fsmp_graph fsmp_graph;
fsmp_status fsmp_graph_create(fsmp_ctx *ctx, const fsmp_batch *batch, const fsmp_samples *out, void *hip_stream,
                              fsmp_graph **graph);
fsmp_status fsmp_graph_launch(fsmp_graph *graph, void *hip_stream);
void fsmp_graph_destroy(fsmp_graph *graph);

/* Message of the last failure on this context (or of the last failed fsmp_create when ctx
 * is NULL); never NULL. */
const char *fsmp_last_error(const fsmp_ctx *ctx);

/* Release the context's device memory; NULL is ignored. */
void fsmp_destroy(fsmp_ctx *ctx);

/* Library version string. */
const char *fsmp_version(void);

/* ------------------------------------------------------------------ serving
 * A continuous-batching request loop over one device.  Trigger events (each a ragged set
 * of channel waveforms, host memory) are submitted as they arrive; fsmp_server_progress
 * admits queued events, in arrival order, into micro-batches while the device-memory
 * budget allows, launches each micro-batch on one of n_streams HIP streams (its own
 * context and workspace, so micro-batches overlap on the device), and retires finished
 * ones.  Every chain of an event runs start to finish on the device.  Random streams are
 * keyed by the waveform identity (event_id * 65536 + channel), so an event's results are
 * the same whether it runs alone or mixed with others.  Buffers grow to the largest
 * micro-batch seen and are then reused: in steady state the server allocates nothing.
 * Latency of an event = completion seen by fsmp_server_progress - fsmp_server_submit. */
typedef struct {
  int32_t n_streams;       /* micro-batches in flight (1..16) */
  int64_t max_batch_wave;  /* waveforms per micro-batch */
  size_t memory_budget;    /* device bytes the admitted, unfinished micro-batches may hold */
} fsmp_server_config;

typedef struct fsmp_server fsmp_server;

/* The server returns posterior summaries per channel (fsmp_server_result): cfg.record_flags
 * must be 0 (FSMP_EINVAL otherwise). */
fsmp_status fsmp_server_create(fsmp_server **out, const fsmp_ser *ser, const fsmp_intensity *phi,
                               const fsmp_config *cfg, int device, const fsmp_server_config *scfg);
/* Queue one event: n_wave channels, samples concatenated in wave (host, copied now),
 * offsets (host, n_wave + 1), lambda and kmax (host; kmax NULL = cfg.k_max).  event_id
 * must be unique among unfinished events and below 2^48; n_wave <= 65536. */
fsmp_status fsmp_server_submit(fsmp_server *srv, uint64_t event_id, int64_t n_wave, const float *wave,
                               const int64_t *offsets, const double *lambda, const int32_t *kmax);
/* Admit, launch and retire; with wait != 0 blocks until at least one micro-batch finishes
 * (if any is in flight).  Returns the number of events completed by this call, or a
 * negative fsmp_status. */
int32_t fsmp_server_progress(fsmp_server *srv, int32_t wait);
/* Results of a completed event (host buffers of n_wave rows): posterior mean and MCSE of
 * (N, Q, t0) per channel, OR of the chains' status words, latency in seconds.  The event
 * is forgotten afterwards.  FSMP_EBUSY if it has not completed. */
fsmp_status fsmp_server_result(fsmp_server *srv, uint64_t event_id, double *mean, double *mcse, uint32_t *status,
                               double *latency_s);
/* Events queued, in flight, completed-but-not-collected; device bytes held. */
fsmp_status fsmp_server_stats(const fsmp_server *srv, int64_t *queued, int64_t *in_flight, int64_t *done,
                              size_t *bytes_held);
const char *fsmp_server_last_error(const fsmp_server *srv);
/* Waits for in-flight work, then releases everything; NULL is ignored. */
void fsmp_server_destroy(fsmp_server *srv);


#ifdef __cplusplus
}
#endif

#endif /* FSMP_H */
