"""Seeded synthetic PMT waveforms in the shapes of the FSMP workloads.

This module only *generates inputs*; it holds none of the sampler's arithmetic
and is shared by the tests (feeding both the HIP path and the CPU oracle) and
the benchmark.  The simulation follows the paper's forward model
(Sec. 1, eq. waveform; Sec. 3 for the simulation protocol):

    N ~ Poisson(lambda);  t_i = t0 + X_i with X_i ~ phi;  q_i ~ charge law;
    w[n] = sum_i q_i V(n - t_i) + sigma_eps * eps_n,   eps_n ~ N(0, 1),

with continuous PE times (not snapped to the sampler's grid), a peak-normalised
ex-Gaussian SER evaluated with scipy's ``exponnorm`` and t0 ~ U[t0_min, t0_max].
The paper's own simulated sets are not available; these stand in for them.

Presets (workloads quoted with the method):
  * ``plain``      1,000 x 256 samples, lambda ~ U[0.5, 5], EXP tau = 20 ns.
  * ``batched``    100,000 x 1,024 samples, lambda ~ logU[0.1, 30], rise 2 / decay 25 ns.
  * ``uneven``     250,000 windows in {128..2048}, lambda ~ logU[0.05, 100].
  * ``pileup``     50,000 x 1,024, lambda ~ U[20, 100], charges N(1, 0.35).
  * ``serving``    channels of 1,024 samples, MCP-like SER (6, 1, 3), Gamma(2, 0.5) charges,
                   lambda from 0.7 U[0,1) + 0.3 U[1,20].
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy import optimize, stats

PHI_EXP = 0
PHI_BIEXP = 1
KCAPS = (16, 32, 48, 64, 96, 128, 160, 192)


@dataclass
class Workload:
    name: str
    n_wave: int
    lengths: tuple = (256,)            # window lengths (samples); one is drawn uniformly per waveform
    lam_dist: str = "uniform"          # uniform | loguniform | mixture
    lam_lo: float = 0.5
    lam_hi: float = 5.0
    ser: tuple = (8.0, 1.5, 6.0)       # ex-Gaussian (mu, sigma, tau) in ns
    phi_kind: int = PHI_EXP
    tau_rise: float = 0.0
    tau_decay: float = 20.0
    t0_min: float = 50.0
    t0_max: float = 100.0
    charge: str = "normal"             # normal (truncated > 0) | gamma
    mu_q: float = 1.0
    sigma_q: float = 0.3
    sigma_eps: float = 0.1
    n_chains: int = 1
    n_steps: int = 2000
    seed: int = 0
    extra: dict = field(default_factory=dict)


PRESETS = {
    "plain": Workload("plain", 1000, (256,), "uniform", 0.5, 5.0, n_chains=1, n_steps=2000),
    "batched": Workload("batched", 100_000, (1024,), "loguniform", 0.1, 30.0, phi_kind=PHI_BIEXP, tau_rise=2.0,
                        tau_decay=25.0, n_chains=4, n_steps=1000),
    "uneven": Workload("uneven", 250_000, (128, 256, 512, 1024, 2048), "loguniform", 0.05, 100.0,
                       phi_kind=PHI_BIEXP, tau_rise=2.0, tau_decay=25.0, n_chains=1, n_steps=1000),
    "pileup": Workload("pileup", 50_000, (1024,), "uniform", 20.0, 100.0, phi_kind=PHI_BIEXP, tau_rise=2.0,
                       tau_decay=25.0, sigma_q=0.35, n_chains=1, n_steps=2000),
    "serving": Workload("serving", 1000, (1024,), "mixture", 0.0, 20.0, ser=(6.0, 1.0, 3.0), phi_kind=PHI_BIEXP,
                        tau_rise=2.0, tau_decay=25.0, charge="gamma", mu_q=1.0, sigma_q=float(np.sqrt(0.5)),
                        n_chains=1, n_steps=1000),
}


def ser_peak(mu, sigma, tau):
    d = stats.exponnorm(K=tau / sigma, loc=mu, scale=sigma)
    r = optimize.minimize_scalar(lambda t: -d.pdf(t), bounds=(0.0, mu + 5 * tau), method="bounded",
                                 options={"xatol": 1e-12})
    return d, float(d.pdf(r.x))


def kmax_for(lam: np.ndarray, tail: float = 1e-7, caps=KCAPS) -> np.ndarray:
    """PE cap per waveform: the smallest cap >= the (1 - tail) Poisson quantile of lambda, plus one."""
    q = stats.poisson.ppf(1.0 - tail, np.asarray(lam, dtype=np.float64)) + 1
    caps = np.asarray(caps)
    idx = np.searchsorted(caps, q, side="left")
    idx = np.minimum(idx, len(caps) - 1)
    return caps[idx].astype(np.int32)


def _draw_lambda(rng, wl: Workload, n):
    if wl.lam_dist == "uniform":
        return rng.uniform(wl.lam_lo, wl.lam_hi, n)
    if wl.lam_dist == "loguniform":
        return np.exp(rng.uniform(np.log(wl.lam_lo), np.log(wl.lam_hi), n))
    if wl.lam_dist == "mixture":
        lo = rng.uniform(0.0, 1.0, n)
        hi = rng.uniform(1.0, wl.lam_hi, n)
        pick = rng.uniform(0.0, 1.0, n) < 0.7
        return np.where(pick, lo, hi)
    raise ValueError(wl.lam_dist)


def _draw_offsets(rng, wl: Workload, n):
    if wl.phi_kind == PHI_EXP:
        return rng.exponential(wl.tau_decay, n)
    t1, t2 = wl.tau_rise, wl.tau_decay
    # phi_BIEXP is the law of Exp(mean tau2) + Exp(mean tau1*tau2/(tau1+tau2))
    return rng.exponential(t2, n) + rng.exponential(t1 * t2 / (t1 + t2), n)


def _draw_charges(rng, wl: Workload, n):
    if wl.charge == "gamma":
        k = (wl.mu_q / wl.sigma_q) ** 2
        return rng.gamma(k, wl.sigma_q ** 2 / wl.mu_q, n)
    q = rng.normal(wl.mu_q, wl.sigma_q, n)
    bad = q <= 0
    while bad.any():
        q[bad] = rng.normal(wl.mu_q, wl.sigma_q, int(bad.sum()))
        bad = q <= 0
    return q


def generate(wl: Workload, n_wave: Optional[int] = None, seed: Optional[int] = None, lam: Optional[np.ndarray] = None,
             lengths: Optional[np.ndarray] = None):
    """Return a dict with the concatenated float32 samples, int64 offsets, lambda and the truth."""
    n = wl.n_wave if n_wave is None else n_wave
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    if lam is None:
        lam = _draw_lambda(rng, wl, n)
    lam = np.asarray(lam, dtype=np.float64)
    if lengths is None:
        lengths = np.asarray(wl.lengths)[rng.integers(0, len(wl.lengths), n)]
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    dist, peak = ser_peak(*wl.ser)
    t0 = rng.uniform(wl.t0_min, wl.t0_max, n)
    Ns = rng.poisson(lam)
    tot = int(Ns.sum())
    owner = np.repeat(np.arange(n), Ns)
    times = t0[owner] + _draw_offsets(rng, wl, tot)
    charges = _draw_charges(rng, wl, tot)
    noise = rng.standard_normal(int(offsets[-1]))
    acc = np.zeros(int(offsets[-1]), dtype=np.float64)
    span = int(np.ceil(wl.ser[0] + 20 * wl.ser[1] + 30 * wl.ser[2]))  # V / peak < 1e-12 beyond
    rel = np.arange(span + 1)
    chunk = max(1, 4_000_000 // (span + 1))
    for a in range(0, tot, chunk):
        b = min(tot, a + chunk)
        o, t, q = owner[a:b], times[a:b], charges[a:b]
        n0 = np.floor(t).astype(np.int64)[:, None] + rel[None, :]
        L = lengths[o][:, None]
        ok = (n0 >= 0) & (n0 < L)
        vals = q[:, None] * dist.pdf(n0 - t[:, None]) / peak
        base = int(offsets[o[0]])
        top = int(offsets[o[-1] + 1])
        flat = (offsets[o][:, None] + n0)[ok] - base
        acc[base:top] += np.bincount(flat, weights=vals[ok], minlength=top - base)
    wave = (acc + wl.sigma_eps * noise).astype(np.float32)
    splits = np.cumsum(Ns)[:-1]
    truth_t = np.split(times, splits)
    truth_q = np.split(charges, splits)
    return {"wave": wave, "offsets": offsets, "lam": lam, "t0": t0, "N": Ns, "times": truth_t, "charges": truth_q,
            "lengths": lengths}
