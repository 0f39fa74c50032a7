/*
 * fsmp_oracle.c -- plain FP64 CPU reference of the FSMP sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP path: it has its own SER evaluation, its own overlap sums, its own
 * dense Cholesky, its own Philox generator and its own chain driver.
 *
 * What it computes (Xu et al., "The Fast Stochastic Matching Pursuit for
 * Neutrino and Dark Matter Experiments"):
 *   - waveform model w = sum_i q_i V(t - t_i) + eps           (Sec. 1, eq. waveform)
 *   - ex-Gaussian SER V, peak normalised                      (Sec. 3, SER formula)
 *   - charges q ~ N(mu_q, sigma_q^2)                          (Sec. 2.1)
 *   - Poisson point-process prior with intensity lambda*phi(t-t0) (Sec. 2.2, eq. pzmu)
 *   - p(w|z) as the multivariate normal of App. A (eq. mgauss), evaluated
 *     from scratch for every proposal (no incremental update at all)
 *   - Gibbs sweep: t0 by Metropolis-Hastings, then one RJMCMC jump
 *     (birth / death / update) with J = 1/4 and the empty-sequence rule
 *     (Sec. 2.4, eqs. birth, death, update, delta-nu)
 *   - MCP-PMT form: each PE's charge from a Gaussian mixture component e
 *     (Sec. 2.1, eq. mcp-multi-norm; Sec. 2.4, eq. mcp; App. A for MCP-PMTs)
 *
 * Readings where the paper leaves a choice (each is listed in the design notes):
 *   - PE times live on a grid t = g * dt with dt = 1/sub samples; the prior is
 *     the Poisson process binned on that grid, so the target carries a factor
 *     1/prod_g n_g! and the normaliser is exp(-Lambda_T(t0)),
 *     Lambda_T(t0) = lambda0 * dt * sum_{g in T} phi(g dt - t0).  With it the
 *     paper's acceptance ratios are exact.
 *   - the density on the grid is point evaluation (midpoint rule) times dt.
 *   - update shift = nearest grid step of a N(0, shift_sd^2) draw; a shift that
 *     leaves T, or lands where phi = 0, is rejected.
 *   - the updated PE keeps its list position; a death moves the last PE of the
 *     list into the freed position; a birth appends.  (Order does not enter
 *     the target; it fixes which index a uniform draw names.)
 *   - K_max truncates the target: a birth at N = K_max is rejected.
 *   - t0 prior uniform on [t0_min, t0_max].
 *   - the SER support is cut at L_V samples; a column is cut at the window end.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 * (seed lo, seed hi), counter = (step, block, uid lo, uid hi) with
 * uid = wave_id * n_chains + chain; block 0 gives r0..r3, block 1 r4..r7:
 *   r0,r1 -> Box-Muller pair (t0 step, update shift); r2 -> t0 accept;
 *   r3 -> move choice; r4 (and r5) -> index / birth position; r6 -> jump accept;
 *   r7 -> the mixture component of a born or updated PE (MCP-PMT form only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PHI_EXP 0
#define ORA_PHI_BIEXP 1

#define MOVE_BIRTH 1
#define MOVE_DEATH 2
#define MOVE_UPDATE 3

typedef struct {
  double ser_mu, ser_sigma, ser_tau, ser_amp;
  int32_t ser_support; /* L_V in samples; 0 = automatic */
  int32_t sub;         /* grid points per sample (dt = 1/sub) */
  double sigma_eps, mu_q, sigma_q;
  int32_t phi_kind;
  double tau_rise, tau_decay, t0_min, t0_max;
  double J, t0_sd, shift_sd;
  /* MCP-PMT charge model (Sec. 2.1, eq. mcp-multi-norm): n_mix > 0 components with
   * probabilities mix_w, means mix_mu and standard deviations mix_sigma; every PE carries
   * its component index e.  n_mix = 0: the single normal N(mu_q, sigma_q^2). */
  int32_t n_mix;
  double mix_w[8], mix_mu[8], mix_sigma[8];
} ora_params;

/* charge law of a PE: ridge rho = sigma_eps^2 / sigma^2 and mean mu of its component */
static void pe_law(const ora_params *p, const int32_t *ez, int k, double *rho, double *mu) {
  double s = p->sigma_eps * p->sigma_eps;
  if (p->n_mix > 0 && ez) {
    double sg = p->mix_sigma[ez[k]];
    *rho = s / (sg * sg);
    *mu = p->mix_mu[ez[k]];
  } else {
    *rho = s / (p->sigma_q * p->sigma_q);
    *mu = p->mu_q;
  }
}

/* component of a new PE: the inverse CDF of the mixture probabilities at u (Sec. 2.4: the
 * proposal of e is G(e) itself) */
static int32_t mix_draw(const ora_params *p, double u) {
  double c = 0.0;
  for (int32_t e = 0; e < p->n_mix - 1; ++e) {
    c += p->mix_w[e];
    if (u < c) return e;
  }
  return p->n_mix - 1;
}

/* one record per step of one chain; same layout as the library's log */
typedef struct {
  int32_t move;     /* 1 birth, 2 death, 3 update */
  int32_t flags;    /* bit0 proposal valid (delta-nu computed), bit1 jump accepted, bit2 t0 accepted */
  int32_t j;        /* index of the removed / moved PE, -1 for birth */
  int32_t g;        /* grid index of the new PE, -1 for death */
  double t0;        /* t0 after the MH half-step */
  double dnu;       /* delta-nu of the proposal (0 if not valid) */
  double log_alpha; /* log acceptance (-inf if not valid) */
} ora_logrec;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 S-box     */
/* with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments     */
/* 0x9E3779B9, 0xBB67AE85.                                             */
/* ------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01_open(uint32_t r) { return ((double)r + 0.5) * 2.3283064365386963e-10; /* 2^-32 */ }

static double u53_open(uint32_t lo, uint32_t hi) {
  uint64_t v = ((uint64_t)hi << 32) | lo;
  return (double)(v >> 11) * 1.1102230246251565e-16 /* 2^-53 */ + 5.551115123125783e-17 /* 2^-54 */;
}

/* ------------------------------------------------------------------ */
/* SER: ex-Gaussian (Sec. 3, SER formula with the Gaussian mean 4 sigma */
/* generalised to mu), divided by its maximum, times the amplitude.     */
/* ------------------------------------------------------------------ */
static double exg_pdf(double t, double mu, double sigma, double tau) {
  double s2t = sigma * sigma / tau;
  return 0.5 / tau * exp((2.0 * mu + s2t - 2.0 * t) / (2.0 * tau)) * erfc((mu + s2t - t) / (M_SQRT2 * sigma));
}

double ora_ser_peak_time(double mu, double sigma, double tau) {
  /* the ex-Gaussian density is unimodal: coarse scan, then golden section */
  double hi = mu + 10.0 * sigma + 10.0 * tau, step = 1e-3;
  double best_t = 0.0, best_f = -1.0;
  for (double t = 0.0; t <= hi; t += step) {
    double f = exg_pdf(t, mu, sigma, tau);
    if (f > best_f) { best_f = f; best_t = t; }
  }
  double a = best_t - step, b = best_t + step;
  const double gr = 0.6180339887498949;
  double c = b - gr * (b - a), d = a + gr * (b - a);
  for (int it = 0; it < 200; ++it) {
    if (exg_pdf(c, mu, sigma, tau) > exg_pdf(d, mu, sigma, tau)) b = d; else a = c;
    c = b - gr * (b - a);
    d = a + gr * (b - a);
  }
  return 0.5 * (a + b);
}

int ora_ser_support_auto(double mu, double sigma, double tau) {
  /* smallest multiple of 16 samples beyond which V / peak < 1e-6 */
  double tp = ora_ser_peak_time(mu, sigma, tau);
  double fp = exg_pdf(tp, mu, sigma, tau);
  for (int L = 16; L <= 8192; L += 16) {
    if ((double)L > tp && exg_pdf((double)L, mu, sigma, tau) / fp < 1e-6) return L;
  }
  return 8192;
}

/* V(t) for t in samples; zero outside [0, L_V) */
double ora_ser_value(const ora_params *p, double t) {
  int LV = p->ser_support > 0 ? p->ser_support : ora_ser_support_auto(p->ser_mu, p->ser_sigma, p->ser_tau);
  if (t < 0.0 || t >= (double)LV) return 0.0;
  double tp = ora_ser_peak_time(p->ser_mu, p->ser_sigma, p->ser_tau);
  double fp = exg_pdf(tp, p->ser_mu, p->ser_sigma, p->ser_tau);
  return p->ser_amp * exg_pdf(t, p->ser_mu, p->ser_sigma, p->ser_tau) / fp;
}

/* ------------------------------------------------------------------ */
/* Light curve phi (Sec. 3, eq. for phi): EXP is the single exponential */
/* (1/tau) e^{-t/tau}; BIEXP is (tau1+tau2)/tau2^2 (1-e^{-t/tau1}) e^{-t/tau2}. */
/* phi(t) = 0 for t < 0.                                                */
/* ------------------------------------------------------------------ */
double ora_phi(const ora_params *p, double t) {
  if (t < 0.0) return 0.0;
  if (p->phi_kind == ORA_PHI_EXP) return exp(-t / p->tau_decay) / p->tau_decay;
  double t1 = p->tau_rise, t2 = p->tau_decay;
  return (t1 + t2) / (t2 * t2) * (-expm1(-t / t1)) * exp(-t / t2);
}

double ora_log_phi(const ora_params *p, double t) {
  double f = ora_phi(p, t);
  return f > 0.0 ? log(f) : -INFINITY;
}

/* Sum over the grid points g = glo..ghi of phi(g dt - t0), as a closed-form
 * geometric series: with x_s = g_s dt - t0 >= 0 the first point where phi is
 * non-zero and r = e^{-dt/tau}, sum_{k<n} e^{-(x_s + k dt)/tau}
 * = e^{-x_s/tau} (1 - r^n) / (1 - r).  BIEXP is the difference of two such
 * series because (1 - e^{-t/tau1}) e^{-t/tau2} = e^{-t/tau2} - e^{-t/tau12},
 * 1/tau12 = 1/tau1 + 1/tau2.  A direct grid sum pins it in the tests. */
static double geo_sum(double xs, double dt, int64_t n, double tau) {
  return exp(-xs / tau) * (-expm1(-(double)n * dt / tau)) / (-expm1(-dt / tau));
}

double ora_phi_sum(const ora_params *p, double t0, int32_t glo, int32_t ghi) {
  double dt = 1.0 / p->sub;
  int64_t gs = (int64_t)ceil(t0 / dt);
  if (gs < glo) gs = glo;
  if (gs > ghi) return 0.0;
  double xs = gs * dt - t0;
  int64_t n = (int64_t)ghi - gs + 1;
  if (p->phi_kind == ORA_PHI_EXP) return geo_sum(xs, dt, n, p->tau_decay) / p->tau_decay;
  double t1 = p->tau_rise, t2 = p->tau_decay;
  double t12 = 1.0 / (1.0 / t1 + 1.0 / t2);
  return (t1 + t2) / (t2 * t2) * (geo_sum(xs, dt, n, t2) - geo_sum(xs, dt, n, t12));
}

/* Lambda_T(t0): expected PE count inside T (reading of eq. pzmu on the grid) */
double ora_lambda_T(const ora_params *p, double lambda0, double t0, int32_t glo, int32_t ghi) {
  return lambda0 * (1.0 / p->sub) * ora_phi_sum(p, t0, glo, ghi);
}

/* Birth position from h(t) = phi(t - t0) / sum_T phi (Sec. 2.4, eq. for h):
 * the smallest g whose running sum exceeds u * total, by a plain scan. */
int32_t ora_birth_draw(const ora_params *p, double t0, int32_t glo, int32_t ghi, double u) {
  double total = ora_phi_sum(p, t0, glo, ghi);
  double target = u * total, run = 0.0;
  double dt = 1.0 / p->sub;
  int32_t last_pos = -1;
  for (int32_t g = glo; g <= ghi; ++g) {
    double f = ora_phi(p, g * dt - t0);
    if (f > 0.0) last_pos = g;
    run += f;
    if (run > target && f > 0.0) return g;
    if (f == 0.0 && g * dt > t0) break; /* beyond the support only through underflow */
  }
  return last_pos;
}

/* ------------------------------------------------------------------ */
/* Likelihood (App. A, eq. mgauss): w ~ N(mu_q A 1, sigma_q^2 A A^T +  */
/* sigma_eps^2 I) where column k of A is the SER placed at t_k.  In PE  */
/* space, with s = sigma_eps^2, rho = s / sigma_q^2, G = A^T A + rho I, */
/* b = A^T w + rho mu_q 1 (determinant lemma and Woodbury identity):     */
/*   log p(w|z) = -1/2 [ Lw log(2 pi s) + w^T w / s ]                   */
/*                -1/2 [ -K log rho + log|G| + (rho mu_q^2 K - b^T G^-1 b)/s ] */
/* The second line is nu(z); delta-nu (eq. delta-nu) is a difference of  */
/* nu's.  Dense MVN and the paper's Woodbury form pin it in the tests.   */
/* ------------------------------------------------------------------ */
typedef struct {
  int LV, sub, M; /* M = sub * LV table entries */
  double *vtab;   /* V(m / sub), m < M */
} ora_table;

static void table_init(ora_table *t, const ora_params *p) {
  t->LV = p->ser_support > 0 ? p->ser_support : ora_ser_support_auto(p->ser_mu, p->ser_sigma, p->ser_tau);
  t->sub = p->sub;
  t->M = t->sub * t->LV;
  t->vtab = (double *)malloc(sizeof(double) * t->M);
  double tp = ora_ser_peak_time(p->ser_mu, p->ser_sigma, p->ser_tau);
  double fp = exg_pdf(tp, p->ser_mu, p->ser_sigma, p->ser_tau);
  for (int m = 0; m < t->M; ++m)
    t->vtab[m] = p->ser_amp * exg_pdf((double)m / t->sub, p->ser_mu, p->ser_sigma, p->ser_tau) / fp;
}

static void table_free(ora_table *t) { free(t->vtab); }

/* fill V(m / sub) for m < sub * L_V; returns L_V */
int32_t ora_ser_table(const ora_params *p, double *out, int32_t cap) {
  ora_table t;
  table_init(&t, p);
  for (int m = 0; m < t.M && m < cap; ++m) out[m] = t.vtab[m];
  int32_t LV = t.LV;
  table_free(&t);
  return LV;
}

typedef struct {
  const ora_params *p;
  int LV, sub, M;
  const double *vtab;
  const float *w;
  int32_t Lw;
} ora_ctx;

static void ctx_init(ora_ctx *c, const ora_params *p, const ora_table *t, const float *w, int32_t Lw) {
  c->p = p;
  c->LV = t->LV;
  c->sub = t->sub;
  c->M = t->M;
  c->vtab = t->vtab;
  c->w = w;
  c->Lw = Lw;
}

/* column of grid point g at sample n: V(n - g/sub) */
static double col(const ora_ctx *c, int32_t g, int32_t n) {
  int64_t m = (int64_t)c->sub * n - g;
  return (m >= 0 && m < c->M) ? c->vtab[m] : 0.0;
}

/* samples where column g can be non-zero, clipped to the window */
static void col_span(const ora_ctx *c, int32_t g, int32_t *n0, int32_t *n1) {
  int64_t lo = (g + c->sub - 1) / c->sub; /* g >= 0 */
  if (g < 0) lo = -((-(int64_t)g) / c->sub);
  int64_t hi = ((int64_t)g + c->M - 1) / c->sub;
  if (lo < 0) lo = 0;
  if (hi > c->Lw - 1) hi = c->Lw - 1;
  *n0 = (int32_t)lo;
  *n1 = (int32_t)hi;
}

static double overlap(const ora_ctx *c, int32_t g1, int32_t g2) {
  int32_t a0, a1, b0, b1;
  col_span(c, g1, &a0, &a1);
  col_span(c, g2, &b0, &b1);
  int32_t lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  double s = 0.0;
  for (int32_t n = lo; n <= hi; ++n) s += col(c, g1, n) * col(c, g2, n);
  return s;
}

static double matched(const ora_ctx *c, int32_t g) {
  int32_t a0, a1;
  col_span(c, g, &a0, &a1);
  double s = 0.0;
  for (int32_t n = a0; n <= a1; ++n) s += col(c, g, n) * (double)c->w[n];
  return s;
}

/* nu(z) from scratch; x (if not NULL) receives G^-1 b, the charges' posterior
 * mean given z.  Returns 0 on success, -1 if G is not positive definite. */
static int nu_of(const ora_ctx *c, const int32_t *z, const int32_t *ez, int K, double *nu, double *x) {
  const ora_params *p = c->p;
  double s = p->sigma_eps * p->sigma_eps;
  if (K == 0) { *nu = 0.0; return 0; }
  /* per PE: sum log rho_k and sum rho_k mu_k^2 (App. A; for MCP-PMTs every PE has its
   * component's mean and variance, App. A for MCP-PMTs) */
  double slr = 0.0, srm = 0.0;
  double *G = (double *)malloc(sizeof(double) * K * K);
  double *L = (double *)calloc((size_t)K * K, sizeof(double));
  double *b = (double *)malloc(sizeof(double) * K);
  double *u = (double *)malloc(sizeof(double) * K);
  for (int i = 0; i < K; ++i) {
    for (int k = 0; k <= i; ++k) {
      double o = overlap(c, z[i], z[k]);
      G[i * K + k] = o;
      G[k * K + i] = o;
    }
    double rho, m;
    pe_law(p, ez, i, &rho, &m);
    G[i * K + i] += rho;
    b[i] = matched(c, z[i]) + rho * m;
    slr += log(rho);
    srm += rho * m * m;
  }
  /* Cholesky G = L L^T */
  int fail = 0;
  for (int j = 0; j < K && !fail; ++j) {
    double d = G[j * K + j];
    for (int k = 0; k < j; ++k) d -= L[j * K + k] * L[j * K + k];
    if (!(d > 0.0)) { fail = 1; break; }
    L[j * K + j] = sqrt(d);
    for (int i = j + 1; i < K; ++i) {
      double v = G[i * K + j];
      for (int k = 0; k < j; ++k) v -= L[i * K + k] * L[j * K + k];
      L[i * K + j] = v / L[j * K + j];
    }
  }
  if (!fail) {
    double logdet = 0.0, uu = 0.0;
    for (int i = 0; i < K; ++i) {
      double v = b[i];
      for (int k = 0; k < i; ++k) v -= L[i * K + k] * u[k];
      u[i] = v / L[i * K + i];
      uu += u[i] * u[i];
      logdet += 2.0 * log(L[i * K + i]);
    }
    *nu = -0.5 * (-slr + logdet + (srm - uu) / s);
    if (x) {
      for (int i = K - 1; i >= 0; --i) {
        double v = u[i];
        for (int k = i + 1; k < K; ++k) v -= L[k * K + i] * x[k];
        x[i] = v / L[i * K + i];
      }
    }
  }
  free(G); free(L); free(b); free(u);
  return fail ? -1 : 0;
}

/* full log p(w|z), for the tests that pin nu against the dense normal law; ez (NULL
 * without a mixture) holds the PEs' components */
double ora_log_likelihood(const ora_params *p, const float *w, int32_t Lw, const int32_t *z, const int32_t *ez,
                          int32_t K, double *x_out) {
  ora_table t;
  table_init(&t, p);
  ora_ctx c;
  ctx_init(&c, p, &t, w, Lw);
  double nu = 0.0;
  int rc = nu_of(&c, z, ez, K, &nu, x_out);
  double s = p->sigma_eps * p->sigma_eps, ww = 0.0;
  for (int32_t n = 0; n < Lw; ++n) ww += (double)w[n] * w[n];
  table_free(&t);
  if (rc) return NAN;
  return -0.5 * (Lw * log(2.0 * M_PI * s) + ww / s) + nu;
}

/* ------------------------------------------------------------------ */
/* Charge draw given z.  With the Gaussian charge model (Sec. 2.1) the  */
/* charges' conditional law given z and w is normal (App. A, eq.        */
/* mgauss, read as Bayesian linear regression): mean x = G^-1 b and     */
/* covariance sigma_eps^2 G^-1, G = A^T A + rho I, b = A^T w + rho mu_q. */
/* A draw is q = x + sigma_eps L^-T xi with G = L L^T (lower Cholesky)  */
/* and standard normals xi, one per PE in list order: L^-T xi has       */
/* covariance L^-T L^-1 = G^-1.  Returns -1 if G is not positive        */
/* definite.                                                            */
/* ------------------------------------------------------------------ */
static int charge_draw(const ora_ctx *c, const int32_t *z, const int32_t *ez, int K, const double *xi, double *q) {
  const ora_params *p = c->p;
  if (K == 0) return 0;
  double *G = (double *)malloc(sizeof(double) * K * K);
  double *L = (double *)calloc((size_t)K * K, sizeof(double));
  double *b = (double *)malloc(sizeof(double) * K);
  double *u = (double *)malloc(sizeof(double) * K);
  double *x = (double *)malloc(sizeof(double) * K);
  double *y = (double *)malloc(sizeof(double) * K);
  for (int i = 0; i < K; ++i) {
    for (int k = 0; k <= i; ++k) {
      double o = overlap(c, z[i], z[k]);
      G[i * K + k] = o;
      G[k * K + i] = o;
    }
    double rho, m;
    pe_law(p, ez, i, &rho, &m);
    G[i * K + i] += rho;
    b[i] = matched(c, z[i]) + rho * m;
  }
  int fail = 0;
  for (int j = 0; j < K && !fail; ++j) {
    double d = G[j * K + j];
    for (int k = 0; k < j; ++k) d -= L[j * K + k] * L[j * K + k];
    if (!(d > 0.0)) { fail = 1; break; }
    L[j * K + j] = sqrt(d);
    for (int i = j + 1; i < K; ++i) {
      double v = G[i * K + j];
      for (int k = 0; k < j; ++k) v -= L[i * K + k] * L[j * K + k];
      L[i * K + j] = v / L[j * K + j];
    }
  }
  if (!fail) {
    /* x = G^-1 b: forward solve L u = b, back solve L^T x = u */
    for (int i = 0; i < K; ++i) {
      double v = b[i];
      for (int k = 0; k < i; ++k) v -= L[i * K + k] * u[k];
      u[i] = v / L[i * K + i];
    }
    for (int i = K - 1; i >= 0; --i) {
      double v = u[i];
      for (int k = i + 1; k < K; ++k) v -= L[k * K + i] * x[k];
      x[i] = v / L[i * K + i];
    }
    /* y = L^-T xi: back solve L^T y = xi */
    for (int i = K - 1; i >= 0; --i) {
      double v = xi[i];
      for (int k = i + 1; k < K; ++k) v -= L[k * K + i] * y[k];
      y[i] = v / L[i * K + i];
    }
    for (int i = 0; i < K; ++i) q[i] = x[i] + p->sigma_eps * y[i];
  }
  free(G); free(L); free(b); free(u); free(x); free(y);
  return fail ? -1 : 0;
}

/* the standard normals of the charge draw at `step` of chain `uid`: PE k of the
 * list takes Philox block 2 + k/2; the Box-Muller pair of words 0 and 1 gives
 * the cosine branch to even k and the sine branch to odd k */
static void charge_normals(uint64_t uid, uint64_t seed, int32_t step, int K, double *xi) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int k = 0; k < K; k += 2) {
    uint32_t r[4];
    uint32_t ctr[4] = {(uint32_t)step, 2u + (uint32_t)(k / 2), (uint32_t)uid, (uint32_t)(uid >> 32)};
    ora_philox4x32_10(ctr, key, r);
    double R = sqrt(-2.0 * log(u01_open(r[0])));
    double th = 2.0 * M_PI * u01_open(r[1]);
    xi[k] = R * cos(th);
    if (k + 1 < K) xi[k + 1] = R * sin(th);
  }
}

/* one charge draw for given z and normals xi (for the tests that pin it) */
int ora_charge_draw(const ora_params *p, const float *w, int32_t Lw, const int32_t *z, int32_t K, const double *xi,
                    double *q) {
  ora_table t;
  table_init(&t, p);
  ora_ctx c;
  ctx_init(&c, p, &t, w, Lw);
  int rc = charge_draw(&c, z, NULL, K, xi, q);
  table_free(&t);
  return rc;
}

void ora_charge_normals(uint64_t uid, uint64_t seed, int32_t step, int32_t K, double *xi) {
  charge_normals(uid, seed, step, K, xi);
}

/* matched filter and overlaps, exposed for the table-level pins */
double ora_overlap(const ora_params *p, int32_t Lw, int32_t g1, int32_t g2) {
  ora_table t;
  table_init(&t, p);
  ora_ctx c;
  ctx_init(&c, p, &t, NULL, Lw);
  double v = overlap(&c, g1, g2);
  table_free(&t);
  return v;
}

/* ------------------------------------------------------------------ */
/* Acceptance of one proposal (Sec. 2.4).  The posterior ratio is       */
/* e^{dnu} lambda0^{N'-N} phi(z'-t0)/phi(z-t0) (on the grid: times dt   */
/* per PE and the multiplicity factor, which cancels against the        */
/* proposal's own multiplicity), and:                                   */
/*   birth : ratio * (1/N') / h(t+)           -> dnu + log Lambda_T - log(N+1)
 *   death : ratio * h(t-) / (1/N)            -> dnu - log Lambda_T + log N
 *   update: ratio                            -> dnu + log phi(t+-t0) - log phi(t- -t0)
 * with the empty-sequence rule: a birth from N = 0 is multiplied by J and  */
/* a death to N = 0 divided by J.                                          */
/* ------------------------------------------------------------------ */
/* nu(z) from scratch in extended precision (long double: a 64-bit significand on x86-64):
 * the same overlaps, matched filter and Cholesky as nu_of with every sum and product carried
 * in long double from the double SER table and the float samples; the reference of the
 * replay check where nu(z) reaches ~1e6 (pile-up waveforms) and a difference of two FP64 nu's
 * would carry their rounding.  Single charge law only.  Returns 0, or -1 if G is not positive
 * definite. */
static long double overlap_ext(const ora_ctx *c, int32_t g1, int32_t g2) {
  int32_t a0, a1, b0, b1;
  col_span(c, g1, &a0, &a1);
  col_span(c, g2, &b0, &b1);
  int32_t lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  long double s = 0.0L;
  for (int32_t n = lo; n <= hi; ++n) s += (long double)col(c, g1, n) * (long double)col(c, g2, n);
  return s;
}

static long double matched_ext(const ora_ctx *c, int32_t g) {
  int32_t a0, a1;
  col_span(c, g, &a0, &a1);
  long double s = 0.0L;
  for (int32_t n = a0; n <= a1; ++n) s += (long double)col(c, g, n) * (long double)c->w[n];
  return s;
}

static int nu_of_ext(const ora_ctx *c, const int32_t *z, int K, long double *nu) {
  const ora_params *p = c->p;
  const long double s = (long double)p->sigma_eps * (long double)p->sigma_eps;
  const long double rho = s / ((long double)p->sigma_q * (long double)p->sigma_q), m = p->mu_q;
  if (K == 0) { *nu = 0.0L; return 0; }
  long double *G = (long double *)malloc(sizeof(long double) * K * K);
  long double *L = (long double *)calloc((size_t)K * K, sizeof(long double));
  long double *b = (long double *)malloc(sizeof(long double) * K);
  long double *u = (long double *)malloc(sizeof(long double) * K);
  for (int i = 0; i < K; ++i) {
    for (int k = 0; k <= i; ++k) {
      long double o = overlap_ext(c, z[i], z[k]);
      G[i * K + k] = o;
      G[k * K + i] = o;
    }
    G[i * K + i] += rho;
    b[i] = matched_ext(c, z[i]) + rho * m;
  }
  int fail = 0;
  for (int j = 0; j < K && !fail; ++j) {
    long double d = G[j * K + j];
    for (int k = 0; k < j; ++k) d -= L[j * K + k] * L[j * K + k];
    if (!(d > 0.0L)) { fail = 1; break; }
    L[j * K + j] = sqrtl(d);
    for (int i = j + 1; i < K; ++i) {
      long double v = G[i * K + j];
      for (int k = 0; k < j; ++k) v -= L[i * K + k] * L[j * K + k];
      L[i * K + j] = v / L[j * K + j];
    }
  }
  if (!fail) {
    long double logdet = 0.0L, uu = 0.0L;
    for (int i = 0; i < K; ++i) {
      long double v = b[i];
      for (int k = 0; k < i; ++k) v -= L[i * K + k] * u[k];
      u[i] = v / L[i * K + i];
      uu += u[i] * u[i];
      logdet += 2.0L * logl(L[i * K + i]);
    }
    *nu = -0.5L * (-(long double)K * logl(rho) + logdet + ((long double)K * rho * m * m - uu) / s);
  }
  free(G); free(L); free(b); free(u);
  return fail ? -1 : 0;
}

typedef struct {
  int valid;
  double dnu, log_alpha;
  double nu_new;
} proposal_eval;

/* The MCP form (Sec. 2.4, eq. mcp): a born PE's component e is proposed from G(e) and the
 * update moves both time and component (e_new); G(e) enters both the target (eq.
 * mcp-pzmu) and the proposal, and cancels from every acceptance, which keeps the form above
 * with delta-nu of the per-PE charge law.  ez / ebuf / e_new are unused without a mixture. */
static proposal_eval eval_proposal(const ora_ctx *c, double lambda0, int32_t glo, int32_t ghi, double t0,
                                   const int32_t *z, const int32_t *ez, int N, double nu_cur, int move, int j,
                                   int32_t gnew, int32_t e_new, int32_t *zbuf, int32_t *ebuf, double *xbuf) {
  const ora_params *p = c->p;
  double dt = 1.0 / p->sub;
  proposal_eval e;
  e.valid = 0;
  e.dnu = 0.0;
  e.log_alpha = -INFINITY;
  e.nu_new = nu_cur;
  double LamT = ora_lambda_T(p, lambda0, t0, glo, ghi);
  if (move == MOVE_BIRTH) {
    if (!(LamT > 0.0) || gnew < glo || gnew > ghi) return e;
    memcpy(zbuf, z, sizeof(int32_t) * N);
    zbuf[N] = gnew;
    if (ez) {
      memcpy(ebuf, ez, sizeof(int32_t) * N);
      ebuf[N] = e_new;
    }
    double nu;
    if (nu_of(c, zbuf, ez ? ebuf : NULL, N + 1, &nu, xbuf)) return e;
    e.valid = 1;
    e.nu_new = nu;
    e.dnu = nu - nu_cur;
    e.log_alpha = e.dnu + log(LamT) - log((double)(N + 1)) + (N == 0 ? log(p->J) : 0.0);
  } else if (move == MOVE_DEATH) {
    memcpy(zbuf, z, sizeof(int32_t) * N);
    zbuf[j] = zbuf[N - 1];
    if (ez) {
      memcpy(ebuf, ez, sizeof(int32_t) * N);
      ebuf[j] = ebuf[N - 1];
    }
    double nu;
    if (nu_of(c, zbuf, ez ? ebuf : NULL, N - 1, &nu, xbuf)) return e;
    e.valid = 1;
    e.nu_new = nu;
    e.dnu = nu - nu_cur;
    e.log_alpha = e.dnu - log(LamT) + log((double)N) - (N == 1 ? log(p->J) : 0.0);
  } else {
    if (gnew < glo || gnew > ghi) return e;
    double lpn = ora_log_phi(p, gnew * dt - t0);
    double lpo = ora_log_phi(p, z[j] * dt - t0);
    if (lpn == -INFINITY) return e;
    memcpy(zbuf, z, sizeof(int32_t) * N);
    zbuf[j] = gnew;
    if (ez) {
      memcpy(ebuf, ez, sizeof(int32_t) * N);
      ebuf[j] = e_new;
    }
    double nu;
    if (nu_of(c, zbuf, ez ? ebuf : NULL, N, &nu, xbuf)) return e;
    e.valid = 1;
    e.nu_new = nu;
    e.dnu = nu - nu_cur;
    e.log_alpha = e.dnu + lpn - lpo;
  }
  return e;
}

/* log acceptance of a given proposal from a given state (for the exact
 * stationarity test on tiny state spaces); returns -inf for an invalid one */
double ora_log_alpha(const ora_params *p, const float *w, int32_t Lw, double lambda0, int32_t glo, int32_t ghi,
                     double t0, const int32_t *z, int32_t N, int32_t move, int32_t j, int32_t gnew, double *dnu_out) {
  ora_table t;
  table_init(&t, p);
  ora_ctx c;
  ctx_init(&c, p, &t, w, Lw);
  double nu_cur = 0.0;
  nu_of(&c, z, NULL, N, &nu_cur, NULL);
  int32_t *zb = (int32_t *)malloc(sizeof(int32_t) * (N + 1));
  double *xb = (double *)malloc(sizeof(double) * (N + 1));
  proposal_eval e = eval_proposal(&c, lambda0, glo, ghi, t0, z, NULL, N, nu_cur, move, j, gnew, 0, zb, NULL, xb);
  free(zb); free(xb);
  table_free(&t);
  if (dnu_out) *dnu_out = e.dnu;
  return e.valid ? e.log_alpha : -INFINITY;
}

/* log of the t0 conditional ratio p(t0'|z) / p(t0|z) (Sec. 2.4): the product
 * of phi over PEs and the normaliser exp(-Lambda_T(t0)); -inf if t0' leaves
 * [t0_min, t0_max] or makes some phi vanish */
double ora_t0_log_alpha(const ora_params *p, double lambda0, int32_t glo, int32_t ghi, const int32_t *z, int32_t N,
                        double t0, double t0p) {
  if (t0p < p->t0_min || t0p > p->t0_max) return -INFINITY;
  double dt = 1.0 / p->sub, s = 0.0;
  for (int k = 0; k < N; ++k) {
    double a = ora_log_phi(p, z[k] * dt - t0p);
    if (a == -INFINITY) return -INFINITY;
    s += a - ora_log_phi(p, z[k] * dt - t0);
  }
  return s - (ora_lambda_T(p, lambda0, t0p, glo, ghi) - ora_lambda_T(p, lambda0, t0, glo, ghi));
}

/* ------------------------------------------------------------------ */
/* Chain driver                                                         */
/* ------------------------------------------------------------------ */
#define ORA_ST_KMAX 1u
#define ORA_ST_NONFINITE 2u
#define ORA_ST_EMPTY_T 8u
#define ORA_ST_FACTOR 16u

typedef struct {
  /* accumulators after burn-in: sum N, N^2, Q, Q^2, t0, t0^2, then the
   * batch-sum statistics sum_b S_b, sum_b S_b^2 for N, Q, t0 */
  double acc[12];
} ora_acc;

static void run_one_chain(const ora_params *p, const ora_table *tab, const float *w, int32_t Lw, double lambda0, int32_t kmax, int32_t glo,
                          int32_t ghi, double t0_init, uint64_t uid, uint64_t seed, int32_t n_steps, int32_t burn_in,
                          int32_t kz, int32_t *N_out, double *t0_out, int32_t *z_out, double *x_out, double *acc,
                          int32_t *nhist, int32_t *counts, uint32_t *status, ora_logrec *logrec, double *trace,
                          int32_t thin, double *qdraw, int32_t *zdraw, int32_t *occ, const int32_t *z0, int32_t n0,
                          int32_t *e_out) {
  ora_ctx c;
  ctx_init(&c, p, tab, w, Lw);
  double dt = 1.0 / p->sub;
  uint32_t st = 0;
  for (int32_t n = 0; n < Lw; ++n)
    if (!isfinite(w[n])) st |= ORA_ST_NONFINITE;
  if (glo > ghi) st |= ORA_ST_EMPTY_T;
  int32_t *z = (int32_t *)calloc((size_t)kmax + 1, sizeof(int32_t));
  int32_t *zb = (int32_t *)calloc((size_t)kmax + 2, sizeof(int32_t));
  double *x = (double *)calloc((size_t)kmax + 1, sizeof(double));
  double *xb = (double *)calloc((size_t)kmax + 2, sizeof(double));
  double *xi = (double *)calloc((size_t)kmax + 1, sizeof(double));
  double *qb = (double *)calloc((size_t)kmax + 1, sizeof(double));
  /* MCP form: the component of every PE, in list order */
  const int mcp = p->n_mix > 0;
  int32_t *ez = mcp ? (int32_t *)calloc((size_t)kmax + 1, sizeof(int32_t)) : NULL;
  int32_t *eb = mcp ? (int32_t *)calloc((size_t)kmax + 2, sizeof(int32_t)) : NULL;
  int N = 0;
  double t0 = t0_init, nu_cur = 0.0;
  memset(acc, 0, sizeof(double) * 12);
  memset(counts, 0, sizeof(int32_t) * 8);
  for (int k = 0; k <= kz; ++k) nhist[k] = 0;
  int64_t S = n_steps - burn_in;
  int64_t nb = (int64_t)floor(sqrt((double)(S > 0 ? S : 0)));
  int64_t lb = nb > 0 ? S / nb : 0;
  double bs[3] = {0.0, 0.0, 0.0};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  if (st & ORA_ST_NONFINITE) n_steps = 0;
  /* a given initial PE sequence (Sec. 2.3 initial guess): its nu and charges from scratch */
  if (n_steps > 0 && n0 > 0) {
    memcpy(z, z0, sizeof(int32_t) * n0);
    N = n0;
    if (nu_of(&c, z, ez, N, &nu_cur, x)) st |= ORA_ST_FACTOR;
  }
  for (int32_t step = 0; step < n_steps; ++step) {
    uint32_t r[8];
    uint32_t ctr0[4] = {(uint32_t)step, 0u, (uint32_t)uid, (uint32_t)(uid >> 32)};
    uint32_t ctr1[4] = {(uint32_t)step, 1u, (uint32_t)uid, (uint32_t)(uid >> 32)};
    ora_philox4x32_10(ctr0, key, r);
    ora_philox4x32_10(ctr1, key, r + 4);
    /* Box-Muller pair */
    double R = sqrt(-2.0 * log(u01_open(r[0])));
    double th = 2.0 * M_PI * u01_open(r[1]);
    double xi_t0 = R * cos(th), xi_sh = R * sin(th);
    /* Gibbs half-step 1: t0 by Metropolis-Hastings */
    double t0p = t0 + p->t0_sd * xi_t0;
    int t0_acc = 0;
    counts[0]++;
    double la0 = ora_t0_log_alpha(p, lambda0, glo, ghi, z, N, t0, t0p);
    if (la0 > -INFINITY && log(u01_open(r[2])) < la0) {
      t0 = t0p;
      t0_acc = 1;
      counts[1]++;
    }
    /* Gibbs half-step 2: one RJMCMC jump on z */
    double um = u01_open(r[3]);
    int move = (N == 0 || um < p->J) ? MOVE_BIRTH : (um < 2.0 * p->J ? MOVE_DEATH : MOVE_UPDATE);
    int j = -1;
    int32_t gnew = -1;
    /* MCP form: the component of a born or updated PE, from word r7 */
    const int32_t enew = mcp ? mix_draw(p, u01_open(r[7])) : 0;
    proposal_eval e;
    e.valid = 0;
    e.dnu = 0.0;
    e.log_alpha = -INFINITY;
    e.nu_new = nu_cur;
    if (move == MOVE_BIRTH) {
      counts[2]++;
      if (N >= kmax) {
        st |= ORA_ST_KMAX;
      } else if (ora_phi_sum(p, t0, glo, ghi) > 0.0) {
        gnew = ora_birth_draw(p, t0, glo, ghi, u53_open(r[4], r[5]));
        e = eval_proposal(&c, lambda0, glo, ghi, t0, z, ez, N, nu_cur, move, -1, gnew, enew, zb, eb, xb);
      }
    } else {
      j = (int)(((uint64_t)r[4] * (uint64_t)N) >> 32);
      if (move == MOVE_DEATH) {
        counts[4]++;
        e = eval_proposal(&c, lambda0, glo, ghi, t0, z, ez, N, nu_cur, move, j, -1, 0, zb, eb, xb);
      } else {
        counts[6]++;
        int32_t shift = (int32_t)rint(xi_sh * p->shift_sd / dt);
        gnew = z[j] + shift;
        e = eval_proposal(&c, lambda0, glo, ghi, t0, z, ez, N, nu_cur, move, j, gnew, enew, zb, eb, xb);
      }
    }
    int accepted = 0;
    if (e.valid && log(u01_open(r[6])) < e.log_alpha) {
      accepted = 1;
      counts[2 * move + 1]++;
      if (move == MOVE_BIRTH) {
        z[N] = gnew;
        if (mcp) ez[N] = enew;
        N++;
      } else if (move == MOVE_DEATH) {
        z[j] = z[N - 1];
        if (mcp) ez[j] = ez[N - 1];
        N--;
      } else {
        z[j] = gnew;
        if (mcp) ez[j] = enew;
      }
      nu_cur = e.nu_new;
      memcpy(x, xb, sizeof(double) * N);
    }
    if (logrec) {
      ora_logrec *lr = &logrec[step];
      lr->move = move;
      lr->flags = (e.valid ? 1 : 0) | (accepted ? 2 : 0) | (t0_acc ? 4 : 0);
      lr->j = j;
      lr->g = gnew;
      lr->t0 = t0;
      lr->dnu = e.valid ? e.dnu : 0.0;
      lr->log_alpha = e.valid ? e.log_alpha : -INFINITY;
    }
    /* record after burn-in: N, Q = 1^T x (charges' conditional mean), t0 */
    if (step >= burn_in) {
      double Q = 0.0;
      for (int k = 0; k < N; ++k) Q += x[k];
      double v[3] = {(double)N, Q, t0};
      for (int a = 0; a < 3; ++a) {
        acc[2 * a] += v[a];
        acc[2 * a + 1] += v[a] * v[a];
      }
      int64_t i = step - burn_in;
      if (nb > 0 && i < nb * lb) {
        for (int a = 0; a < 3; ++a) bs[a] += v[a];
        if ((i + 1) % lb == 0) {
          for (int a = 0; a < 3; ++a) {
            acc[6 + 2 * a] += bs[a];
            acc[7 + 2 * a] += bs[a] * bs[a];
            bs[a] = 0.0;
          }
        }
      }
      if (N <= kz) nhist[N]++;
      /* grid occupancy: every PE of the recorded state counts once at its grid point */
      if (occ)
        for (int k = 0; k < N; ++k) occ[z[k]]++;
      if (trace && thin > 0 && (i % thin) == 0) {
        double *tr = trace + 3 * (i / thin);
        tr[0] = (double)N;
        tr[1] = t0;
        tr[2] = Q;
      }
      /* charge draw of the recorded state (NaN if G is not positive definite) */
      if (qdraw && thin > 0 && (i % thin) == 0) {
        double *qr = qdraw + (size_t)kz * (i / thin);
        int32_t *zr = zdraw + (size_t)kz * (i / thin);
        charge_normals(uid, seed, step, N, xi);
        int rc = charge_draw(&c, z, ez, N, xi, qb);
        if (rc) st |= ORA_ST_FACTOR;
        for (int k = 0; k < kz; ++k) {
          zr[k] = k < N ? z[k] : -1;
          qr[k] = k < N ? (rc ? NAN : qb[k]) : 0.0;
        }
      }
    }
  }
  *N_out = N;
  *t0_out = t0;
  for (int k = 0; k < kz; ++k) {
    z_out[k] = k < N ? z[k] : -1;
    x_out[k] = k < N ? x[k] : 0.0;
  }
  *status = st;
  if (e_out)
    for (int k = 0; k < kz; ++k) e_out[k] = (mcp && k < N) ? ez[k] : -1;
  free(z); free(zb); free(x); free(xb); free(xi); free(qb); free(ez); free(eb);
}

/* Run n_chains chains for every waveform.  Chain c of waveform i writes
 * index i * n_chains + c of every output.  kz is the row length of z_out /
 * x_out (>= every kmax) and nhist rows have kz + 1 entries.  occ (NULL to
 * skip; zeroed by the caller) holds one row of sub * L_i grid points per chain,
 * chain c of waveform i at n_chains * sub * offsets[i] + c * sub * L_i: the
 * number of recorded sweeps with a PE at each grid point, PEs counted with
 * their multiplicity.  z_init / z_init_off (NULL: empty start) give chain c the
 * initial PE list z_init[z_init_off[c] .. z_init_off[c + 1]), which the caller has
 * checked (at most kmax PEs, inside T, phi > 0 at t0_init). */
int ora_run(const ora_params *p, int64_t n_wave, const float *wave, const int64_t *offsets, const double *lambda,
            const int32_t *kmax, const int32_t *g_range, const double *t0_init, const uint64_t *wave_id,
            int32_t n_chains, int32_t n_steps, int32_t burn_in, uint64_t seed, int32_t kz, int32_t *N_out,
            double *t0_out, int32_t *z_out, double *x_out, double *acc, int32_t *nhist, int32_t *counts,
            uint32_t *status, ora_logrec *logrec, double *trace, int32_t thin, double *qdraw, int32_t *zdraw,
            int32_t *occ, const int32_t *z_init, const int64_t *z_init_off, int32_t *e_out, int32_t n_threads,
            const int32_t *wsteps) {
  int64_t total = n_wave * n_chains;
  int64_t n_rec = (thin > 0 && n_steps > burn_in) ? (n_steps - burn_in + thin - 1) / thin : 0;
  ora_table tab;
  table_init(&tab, p);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t ic = 0; ic < total; ++ic) {
    int64_t i = ic / n_chains;
    int32_t ch = (int32_t)(ic % n_chains);
    int32_t Lw = (int32_t)(offsets[i + 1] - offsets[i]);
    int32_t glo = g_range ? g_range[2 * i] : 0;
    int32_t ghi = g_range ? g_range[2 * i + 1] : p->sub * Lw - 1;
    double t0i = t0_init ? t0_init[i] : 0.5 * (p->t0_min + p->t0_max);
    uint64_t wid = wave_id ? wave_id[i] : (uint64_t)i;
    uint64_t uid = wid * (uint64_t)n_chains + (uint64_t)ch;
    /* a waveform's own sweep count keeps the configured burn-in fraction, rounded down */
    int32_t ns = wsteps ? wsteps[i] : n_steps;
    int32_t bw = wsteps ? (int32_t)((int64_t)ns * burn_in / n_steps) : burn_in;
    run_one_chain(p, &tab, wave + offsets[i], Lw, lambda[i], kmax ? kmax[i] : kz, glo, ghi, t0i, uid, seed, ns,
                  bw, kz, &N_out[ic], &t0_out[ic], z_out + ic * kz, x_out + ic * kz, acc + ic * 12,
                  nhist + ic * (kz + 1), counts + ic * 8, &status[ic], logrec ? logrec + ic * n_steps : NULL,
                  trace ? trace + ic * 3 * n_rec : NULL, thin, qdraw ? qdraw + ic * kz * n_rec : NULL,
                  zdraw ? zdraw + ic * kz * n_rec : NULL,
                  occ ? occ + n_chains * p->sub * offsets[i] + (int64_t)ch * p->sub * Lw : NULL,
                  z_init_off ? z_init + z_init_off[ic] : NULL,
                  z_init_off ? (int32_t)(z_init_off[ic + 1] - z_init_off[ic]) : 0, e_out ? e_out + ic * kz : NULL);
  }
  table_free(&tab);
  return 0;
}

/* Replay: follow a recorded proposal sequence of one chain (the move, the
 * index, the new grid point, the t0 after the MH half-step and the recorded
 * accept decision), recompute delta-nu and log alpha from scratch for every
 * valid proposal, and re-derive the accept decision from this oracle's own
 * Philox stream.  z0[0 .. n0) is the chain's initial PE list (n0 = 0: empty
 * start).  Returns the number of steps whose decision differs although
 * |log U - log alpha| > tie_eps, or -1 when n0 exceeds kmax. */
int64_t ora_replay(const ora_params *p, const float *w, int32_t Lw, double lambda0, int32_t kmax, int32_t glo,
                   int32_t ghi, uint64_t uid, uint64_t seed, int32_t n_steps, const ora_logrec *rec, double *dnu_ref,
                   double *la_ref, double tie_eps, int32_t ext, const int32_t *z0, int32_t n0) {
  if (n0 < 0 || n0 > kmax) return -1;
  ora_table t;
  table_init(&t, p);
  ora_ctx c;
  ctx_init(&c, p, &t, w, Lw);
  int32_t *z = (int32_t *)calloc((size_t)kmax + 1, sizeof(int32_t));
  int32_t *zb = (int32_t *)calloc((size_t)kmax + 2, sizeof(int32_t));
  double *xb = (double *)calloc((size_t)kmax + 2, sizeof(double));
  int N = 0;
  double nu_cur = 0.0;
  long double nu_cur_ext = 0.0L, nu_new_ext = 0.0L;
  int64_t bad = 0;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  /* a chain started from a given PE sequence (as ora_run starts it): its nu from scratch */
  if (n0 > 0) {
    memcpy(z, z0, sizeof(int32_t) * n0);
    N = n0;
    if (nu_of(&c, z, NULL, N, &nu_cur, NULL)) bad++;
    if (ext && nu_of_ext(&c, z, N, &nu_cur_ext)) bad++;
  }
  for (int32_t step = 0; step < n_steps; ++step) {
    const ora_logrec *lr = &rec[step];
    double t0 = lr->t0;
    dnu_ref[step] = 0.0;
    la_ref[step] = -INFINITY;
    if (!(lr->flags & 1)) continue;
    if (lr->move == MOVE_BIRTH && N >= kmax) { bad++; continue; }
    if ((lr->move == MOVE_DEATH || lr->move == MOVE_UPDATE) && (lr->j < 0 || lr->j >= N)) { bad++; continue; }
    proposal_eval e = eval_proposal(&c, lambda0, glo, ghi, t0, z, NULL, N, nu_cur, lr->move, lr->j, lr->g, 0, zb, NULL, xb);
    if (!e.valid) { bad++; continue; }
    if (ext) {
      /* the proposed list as eval_proposal formed it, nu in extended precision */
      const int Kn = lr->move == MOVE_BIRTH ? N + 1 : lr->move == MOVE_DEATH ? N - 1 : N;
      if (nu_of_ext(&c, zb, Kn, &nu_new_ext)) { bad++; continue; }
      const double d = (double)(nu_new_ext - nu_cur_ext);
      e.log_alpha += d - e.dnu;
      e.dnu = d;
    }
    dnu_ref[step] = e.dnu;
    la_ref[step] = e.log_alpha;
    uint32_t r[4];
    uint32_t ctr1[4] = {(uint32_t)step, 1u, (uint32_t)uid, (uint32_t)(uid >> 32)};
    ora_philox4x32_10(ctr1, key, r);
    double lu = log(u01_open(r[2]));
    int mine = lu < e.log_alpha;
    int theirs = (lr->flags & 2) != 0;
    if (mine != theirs && fabs(lu - e.log_alpha) > tie_eps) bad++;
    if (theirs) {
      if (lr->move == MOVE_BIRTH) {
        z[N] = lr->g;
        N++;
      } else if (lr->move == MOVE_DEATH) {
        z[lr->j] = z[N - 1];
        N--;
      } else {
        z[lr->j] = lr->g;
      }
      nu_cur = e.nu_new;
      nu_cur_ext = nu_new_ext;
    }
  }
  free(z); free(zb); free(xb);
  table_free(&t);
  return bad;
}
