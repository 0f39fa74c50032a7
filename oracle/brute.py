"""Definitions written out densely, for pinning the oracle (and through it the HIP path).

TEST INFRASTRUCTURE ONLY.  Everything here is numpy/scipy and independent of
``fsmp_oracle.c``: its own SER (scipy's ``exponnorm``), its own light curve, a
direct grid sum for the prior normaliser, the dense normal law of App. A
(eq. mgauss) and the paper's Woodbury form of delta-nu (App. A, eqs. 11-18).

* ``dense_logp``       -- log N(w; mu_q A 1, sigma_q^2 A A^T + sigma_eps^2 I), the definition.
* ``paper_dnu``        -- delta-nu through Sigma^{-1}(z) and the rank-2 Woodbury update.
* ``charge_mean``      -- E[q | z, w] by least squares on the augmented system
                          [A/sigma_eps; I/sigma_q] q = [w/sigma_eps; mu_q 1/sigma_q].
* ``posterior_exact``  -- the grid posterior of (z, t0) by enumeration of all
                          multisets with N <= K_max (t0 fixed, or integrated by
                          Gauss-Legendre quadrature between the grid knots).
"""
import itertools
import math

import numpy as np
from scipy import stats
from scipy.special import gammaln


class Model:
    """Model constants for the dense definitions (times in samples, grid dt = 1/sub)."""

    def __init__(self, ser=(8.0, 1.5, 6.0), ser_amp=1.0, LV=96, sub=4, sigma_eps=0.1, mu_q=1.0, sigma_q=0.3,
                 phi_kind=0, tau_rise=0.0, tau_decay=20.0, t0_min=50.0, t0_max=100.0, J=0.25, shift_sd=1.0):
        self.mu, self.sigma, self.tau = ser
        self.amp = ser_amp
        self.LV = LV
        self.sub = sub
        self.sigma_eps, self.mu_q, self.sigma_q = sigma_eps, mu_q, sigma_q
        self.phi_kind, self.tau_rise, self.tau_decay = phi_kind, tau_rise, tau_decay
        self.t0_min, self.t0_max = t0_min, t0_max
        self.J, self.shift_sd = J, shift_sd
        dist = stats.exponnorm(K=self.tau / self.sigma, loc=self.mu, scale=self.sigma)
        self._dist = dist
        res = __import__("scipy.optimize", fromlist=["minimize_scalar"]).minimize_scalar(
            lambda t: -dist.pdf(t), bounds=(0.0, self.mu + 5 * self.tau), method="bounded",
            options={"xatol": 1e-12})
        self.peak = dist.pdf(res.x)

    def V(self, t):
        t = np.asarray(t, dtype=np.float64)
        v = self.amp * self._dist.pdf(t) / self.peak
        return np.where((t >= 0) & (t < self.LV), v, 0.0)

    def column(self, g, Lw):
        n = np.arange(Lw, dtype=np.float64)
        return self.V(n - g / self.sub)

    def A(self, z, Lw):
        if len(z) == 0:
            return np.zeros((Lw, 0))
        return np.stack([self.column(g, Lw) for g in z], axis=1)

    def phi(self, t):
        t = np.asarray(t, dtype=np.float64)
        if self.phi_kind == 0:
            v = np.exp(-t / self.tau_decay) / self.tau_decay
        else:
            t1, t2 = self.tau_rise, self.tau_decay
            v = (t1 + t2) / t2 ** 2 * (1 - np.exp(-t / t1)) * np.exp(-t / t2)
        return np.where(t >= 0, v, 0.0)

    def Lambda_T(self, lam, t0, glo, ghi):
        g = np.arange(glo, ghi + 1)
        return lam / self.sub * self.phi(g / self.sub - t0).sum()

    def h(self, t0, glo, ghi):
        g = np.arange(glo, ghi + 1)
        f = self.phi(g / self.sub - t0)
        return f / f.sum()


def dense_logp(m: Model, w, z):
    """log p(w|z) straight from App. A, eq. mgauss."""
    w = np.asarray(w, dtype=np.float64)
    Lw = len(w)
    A = m.A(z, Lw)
    U = m.mu_q * A.sum(axis=1)
    Sig = m.sigma_q ** 2 * A @ A.T + m.sigma_eps ** 2 * np.eye(Lw)
    return stats.multivariate_normal(mean=U, cov=Sig).logpdf(w)


def paper_dnu(m: Model, w, z, a_minus_g, a_plus_g):
    """delta-nu of App. A (eqs. 11, 14, DeltaU, 12, 16, 17, 18): the rank-2 Woodbury form on the
    N_w x N_w covariance.  ``a_minus_g`` / ``a_plus_g`` are grid indices or None (birth / death)."""
    w = np.asarray(w, dtype=np.float64)
    Lw = len(w)
    A = m.A(z, Lw)
    U = m.mu_q * A.sum(axis=1)
    Sig = m.sigma_q ** 2 * A @ A.T + m.sigma_eps ** 2 * np.eye(Lw)
    Sinv = np.linalg.inv(Sig)
    am = m.column(a_minus_g, Lw) if a_minus_g is not None else np.zeros(Lw)
    ap = m.column(a_plus_g, Lw) if a_plus_g is not None else np.zeros(Lw)
    a = np.stack([am, ap], axis=1)
    Lam = m.sigma_q ** 2 * np.diag([-1.0, 1.0])
    Laminv = np.linalg.inv(Lam)
    lamv = m.mu_q * np.array([-1.0, 1.0])
    y = w - U
    c = Sinv @ a
    B = np.linalg.inv(Laminv + a.T @ c)
    Ups = c.T @ y + Laminv @ lamv
    return 0.5 * (Ups @ B @ Ups - lamv @ Laminv @ lamv + np.log(np.linalg.det(B @ Laminv)))


def charge_mean(m: Model, w, z):
    """E[q | z, w]: Bayesian linear regression with prior N(mu_q, sigma_q^2 I), by lstsq."""
    w = np.asarray(w, dtype=np.float64)
    K = len(z)
    if K == 0:
        return np.zeros(0)
    A = m.A(z, len(w))
    M = np.vstack([A / m.sigma_eps, np.eye(K) / m.sigma_q])
    r = np.concatenate([w / m.sigma_eps, np.full(K, m.mu_q / m.sigma_q)])
    return np.linalg.lstsq(M, r, rcond=None)[0]


def multisets(glo, ghi, kmax):
    pts = range(glo, ghi + 1)
    for k in range(kmax + 1):
        for c in itertools.combinations_with_replacement(pts, k):
            yield c


def log_prior(m: Model, z, lam, t0, glo, ghi):
    """Grid Poisson process on T: exp(-Lambda_T) prod_k (lam dt phi(t_k - t0)) / prod_g n_g!."""
    dt = 1.0 / m.sub
    lp = -m.Lambda_T(lam, t0, glo, ghi)
    for g in z:
        f = float(m.phi(g * dt - t0))
        if f <= 0:
            return -np.inf
        lp += math.log(lam * dt * f)
    _, counts = np.unique(np.asarray(z, dtype=np.int64), return_counts=True) if len(z) else (None, [])
    lp -= sum(gammaln(c + 1) for c in counts)
    return lp


def posterior_exact(m: Model, w, lam, glo, ghi, kmax, t0=None, n_gl=12):
    """Exact posterior summaries by enumeration.  With ``t0`` None the uniform t0 prior on
    [t0_min, t0_max] is integrated out with Gauss-Legendre on every interval between grid knots.

    Returns dict with states, weights, P(N=k), E[N], E[Q] (Q = sum of E[q|z,w]), E[t0], occupancy."""
    states = list(multisets(glo, ghi, kmax))
    ll = np.array([dense_logp(m, w, z) for z in states])
    Qz = np.array([charge_mean(m, w, z).sum() for z in states])
    if t0 is not None:
        lp = np.array([log_prior(m, z, lam, t0, glo, ghi) for z in states])
        logw = ll + lp
        mx = logw.max()
        wt = np.exp(logw - mx)
        wt /= wt.sum()
        Et0 = t0
    else:
        dt = 1.0 / m.sub
        knots = [m.t0_min, m.t0_max]
        g = np.arange(glo, ghi + 1) * dt
        knots += [x for x in g if m.t0_min < x < m.t0_max]
        knots = np.unique(knots)
        xg, wg = np.polynomial.legendre.leggauss(n_gl)
        t_nodes, t_wts = [], []
        for a, b in zip(knots[:-1], knots[1:]):
            t_nodes.append(0.5 * (b - a) * xg + 0.5 * (a + b))
            t_wts.append(0.5 * (b - a) * wg)
        t_nodes = np.concatenate(t_nodes)
        t_wts = np.concatenate(t_wts)
        lp = np.array([[log_prior(m, z, lam, t, glo, ghi) for t in t_nodes] for z in states])
        logj = ll[:, None] + lp + np.log(t_wts)[None, :]
        mx = logj.max()
        J = np.exp(logj - mx)
        Z = J.sum()
        wt = J.sum(axis=1) / Z
        Et0 = float((J.sum(axis=0) * t_nodes).sum() / Z)
    Ns = np.array([len(z) for z in states])
    pN = np.array([wt[Ns == k].sum() for k in range(kmax + 1)])
    occ = np.zeros(ghi - glo + 1)
    for z, p in zip(states, wt):
        for gg in z:
            occ[gg - glo] += p
    return {"states": states, "weights": wt, "pN": pN, "EN": float((Ns * wt).sum()),
            "EQ": float((Qz * wt).sum()), "Et0": Et0, "occupancy": occ}


def shift_pmf(m: Model, s):
    """P(rint(xi / dt) = s) for xi ~ N(0, shift_sd^2): normal mass of the cell around s dt."""
    dt = 1.0 / m.sub
    return stats.norm.cdf((s + 0.5) * dt / m.shift_sd) - stats.norm.cdf((s - 0.5) * dt / m.shift_sd)


# ---------------------------------------------------------------- MCP-PMT mixture charge law
# Sec. 2.1 (eq. mcp-multi-norm), Sec. 2.4 (eq. mcp), App. A for MCP-PMTs: every PE carries a
# component e with charge law N(mu_e, sigma_e^2) and prior weight G(e).

def dense_logp_mix(m: Model, w, z, e, mix):
    """log N(w; A mu_e, A diag(sigma_e^2) A^T + sigma_eps^2 I), the definition."""
    G, mu, sg = (np.asarray(v, np.float64) for v in mix)
    w = np.asarray(w, dtype=np.float64)
    Lw = len(w)
    A = m.A(z, Lw)
    e = np.asarray(e, dtype=np.int64)
    U = A @ mu[e] if len(z) else np.zeros(Lw)
    Sig = (A * sg[e] ** 2) @ A.T + m.sigma_eps ** 2 * np.eye(Lw)
    return stats.multivariate_normal(mean=U, cov=Sig).logpdf(w)


def charge_mean_mix(m: Model, w, z, e, mix):
    """E[q | z, e, w] by lstsq on [A/sigma_eps; diag(1/sigma_e)] q = [w/sigma_eps; mu_e/sigma_e]."""
    G, mu, sg = (np.asarray(v, np.float64) for v in mix)
    w = np.asarray(w, dtype=np.float64)
    K = len(z)
    if K == 0:
        return np.zeros(0)
    e = np.asarray(e, dtype=np.int64)
    A = m.A(z, len(w))
    M = np.vstack([A / m.sigma_eps, np.diag(1.0 / sg[e])])
    r = np.concatenate([w / m.sigma_eps, mu[e] / sg[e]])
    return np.linalg.lstsq(M, r, rcond=None)[0]


def posterior_exact_mix(m: Model, w, lam, glo, ghi, kmax, t0, mix):
    """Enumeration of the posterior of z = {(t_k, e_k)} at fixed t0: every multiset of
    (grid point, component) pairs with N <= kmax, weight p(w|z) times the Poisson process
    on T x E binned into cells (g, e) of mean lam dt phi(g dt - t0) G(e) (eq. mcp-pzmu),
    so the prior carries 1 / prod over cells of n!.  Returns P(N = k), E[N], E[Q] and the
    expected number of PEs in each component."""
    G = np.asarray(mix[0], np.float64)
    E = len(G)
    dt = 1.0 / m.sub
    cells = [(g, e) for g in range(glo, ghi + 1) for e in range(E)]
    LamT = m.Lambda_T(lam, t0, glo, ghi)
    states, lw, Qs = [], [], []
    for k in range(kmax + 1):
        for c in itertools.combinations_with_replacement(cells, k):
            z = [g for g, _ in c]
            e = [x for _, x in c]
            lp = -LamT
            ok = True
            for g, x in c:
                f = float(m.phi(g * dt - t0))
                if f <= 0:
                    ok = False
                    break
                lp += math.log(lam * dt * f * G[x])
            if not ok:
                continue
            _, counts = np.unique(np.asarray(c).reshape(-1, 2), axis=0, return_counts=True) if k else (None, [])
            lp -= sum(gammaln(n + 1) for n in counts)
            states.append(c)
            lw.append(dense_logp_mix(m, w, z, e, mix) + lp)
            Qs.append(charge_mean_mix(m, w, z, e, mix).sum())
    lw = np.array(lw)
    wt = np.exp(lw - lw.max())
    wt /= wt.sum()
    Ns = np.array([len(c) for c in states])
    pN = np.array([wt[Ns == k].sum() for k in range(kmax + 1)])
    ne = np.array([[sum(1 for _, x in c if x == q) for q in range(E)] for c in states], np.float64)
    return {"pN": pN, "EN": float((Ns * wt).sum()), "EQ": float((np.array(Qs) * wt).sum()),
            "En_e": (ne * wt[:, None]).sum(0)}
