"""The oracle's chain driver against exact posteriors and prior-only invariants.

* tiny grids: MCMC estimates of P(N = k), E[N], E[Q], E[t0] against enumeration of
  every multiset (Sec. 2.2 target on the grid, App. A likelihood), with t0 fixed
  and with t0 integrated out;
* data term off (SER amplitude 0): N ~ Poisson(Lambda_T) truncated at K_max, PE
  positions ~ h, and t0 ~ U[t0_min, t0_max] when it is sampled;
* counter-based streams: a chain depends only on (seed, wave id, chain), not on
  the batch it runs in; the replay of a chain's own log agrees with it.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import brute


def _tiny(kind=0, t0_range=(1.0, 1.0)):
    ser = (1.0, 0.5, 1.0)
    kw = dict(ser=ser, sigma_eps=0.3, sigma_q=0.4, mu_q=1.0, phi_kind=kind, tau_rise=0.7 if kind else 0.0,
              tau_decay=2.0, t0_min=t0_range[0], t0_max=t0_range[1], J=0.25)
    p = oracle.make_params(ser_support=16, shift_sd=0.5, t0_sd=0.3, **kw)
    m = brute.Model(LV=16, shift_sd=0.5, **kw)
    return p, m


def _wave(m, Lw, gs, qs, seed):
    rng = np.random.default_rng(seed)
    w = np.zeros(Lw)
    for g, q in zip(gs, qs):
        w += q * m.column(g, Lw)
    return (w + m.sigma_eps * rng.standard_normal(Lw)).astype(np.float32)


def _mcmc(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn, seed=7, t0_init=None):
    offsets = np.array([0, len(w)], np.int64)
    r = oracle.run(p, w, offsets, np.array([lam]), n_chains, n_steps, burn, seed, kz=kmax,
                   kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32),
                   t0_init=None if t0_init is None else np.array([t0_init]))
    return r


@pytest.mark.parametrize("kind", [0, 1])
def test_mcmc_matches_enumeration_t0_fixed(kind):
    p, m = _tiny(kind)
    Lw, glo, ghi, kmax, lam = 12, 6, 17, 3, 1.6
    w = _wave(m, Lw, [8, 13], [1.0, 0.8], seed=21 + kind)
    exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=1.0)
    n_chains, n_steps, burn = 48, 40000, 2000
    r = _mcmc(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn)
    s = oracle.summarize(r.acc, n_steps, burn, n_chains)
    for name, want in (("N", exact["EN"]), ("Q", exact["EQ"])):
        mean, _, mcse = (v[0] for v in s[name])
        assert abs(mean - want) < 4 * mcse + 1e-12, (name, mean, want, mcse)
    pN = r.nhist.sum(0)[: kmax + 1] / r.nhist.sum()
    np.testing.assert_allclose(pN, exact["pN"], atol=0.01)
    assert (r.status & 1).any() or exact["pN"][kmax] < 1e-3


def test_mcmc_matches_enumeration_t0_sampled():
    p, m = _tiny(0, t0_range=(0.5, 2.0))
    Lw, glo, ghi, kmax, lam = 12, 6, 15, 3, 1.8
    w = _wave(m, Lw, [9, 12], [1.0, 1.1], seed=5)
    exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=None)
    n_chains, n_steps, burn = 48, 40000, 2000
    r = _mcmc(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn, t0_init=1.0)
    s = oracle.summarize(r.acc, n_steps, burn, n_chains)
    for name, want in (("N", exact["EN"]), ("Q", exact["EQ"]), ("t0", exact["Et0"])):
        mean, _, mcse = (v[0] for v in s[name])
        assert abs(mean - want) < 4 * mcse + 1e-12, (name, mean, want, mcse)
    pN = r.nhist.sum(0)[: kmax + 1] / r.nhist.sum()
    np.testing.assert_allclose(pN, exact["pN"], atol=0.012)


def test_enumeration_catches_planted_mistake():
    # the chain targets the posterior; the prior alone (a plausible slip: data term dropped)
    # must be distinguishable from it on this waveform
    p, m = _tiny(0)
    Lw, glo, ghi, kmax, lam = 12, 6, 17, 3, 1.6
    w = _wave(m, Lw, [8, 13], [1.0, 0.8], seed=21)
    exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=1.0)
    p0 = oracle.make_params(ser=(1.0, 0.5, 1.0), ser_amp=0.0, ser_support=16, sigma_eps=0.3, sigma_q=0.4,
                            phi_kind=0, tau_decay=2.0, t0_min=1.0, t0_max=1.0, shift_sd=0.5)
    r = _mcmc(p0, w, lam, glo, ghi, kmax, 16, 20000, 1000)
    s = oracle.summarize(r.acc, 20000, 1000, 16)
    assert abs(s["N"][0][0] - exact["EN"]) > 10 * s["N"][2][0]


@pytest.mark.parametrize("kind", [0, 1])
def test_prior_only_fixed_t0(kind):
    p, m = _tiny(kind)
    p.ser_amp = 0.0
    Lw, glo, ghi, kmax, lam = 24, 0, 95, 12, 3.0
    w = np.zeros(Lw, np.float32)
    n_chains, n_steps, burn = 32, 30000, 1000
    r = _mcmc(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn)
    Lam = m.Lambda_T(lam, 1.0, glo, ghi)
    k = np.arange(kmax + 1)
    want = stats.poisson.pmf(k, Lam)
    want /= want.sum()
    got = r.nhist.sum(0)[: kmax + 1] / r.nhist.sum()
    np.testing.assert_allclose(got, want, atol=0.01)
    s = oracle.summarize(r.acc, n_steps, burn, n_chains)
    assert abs(s["N"][0][0] - (k * want).sum()) < 4 * s["N"][2][0]
    # PE positions of the final states are draws from h (pooled chi-square on coarse bins)
    pos = r.z[r.z >= 0]
    h = m.h(1.0, glo, ghi)
    edges = [0, 8, 16, 32, 96]
    obs = np.array([((pos >= glo + a) & (pos < glo + b)).sum() for a, b in zip(edges[:-1], edges[1:])])
    exp_ = np.array([h[a:b].sum() for a, b in zip(edges[:-1], edges[1:])]) * len(pos)
    keep = exp_ > 5
    if keep.sum() >= 2:
        chi2 = (((obs - exp_) ** 2) / np.maximum(exp_, 1e-12))[keep].sum()
        assert chi2 < stats.chi2.ppf(0.999, keep.sum() - 1)


def test_prior_only_t0_uniform():
    p, m = _tiny(0, t0_range=(0.0, 4.0))
    p.ser_amp = 0.0
    p.t0_sd = 1.0
    Lw, glo, ghi, kmax, lam = 32, 0, 127, 16, 2.0
    w = np.zeros(Lw, np.float32)
    n_chains, n_steps, burn = 32, 40000, 1000
    r = _mcmc(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn, t0_init=2.0)
    s = oracle.summarize(r.acc, n_steps, burn, n_chains)
    mean, var, mcse = (v[0] for v in s["t0"])
    assert abs(mean - 2.0) < 4 * mcse
    assert abs(var - 16.0 / 12.0) < 0.1


def test_chain_is_independent_of_batch_and_deterministic():
    p = oracle.make_params()
    from paper_2403_03156_amd import synth
    b = synth.generate(synth.PRESETS["plain"], n_wave=12, seed=3)
    kz = 16
    r1 = oracle.run(p, b["wave"], b["offsets"], b["lam"], 2, 300, 100, 9, kz)
    r2 = oracle.run(p, b["wave"], b["offsets"], b["lam"], 2, 300, 100, 9, kz)
    np.testing.assert_array_equal(r1.z, r2.z)
    np.testing.assert_array_equal(r1.acc, r2.acc)
    # waveform 5 alone, with its identity passed in, reproduces its two chains exactly
    o = b["offsets"]
    w5 = b["wave"][o[5]:o[6]]
    r3 = oracle.run(p, w5, np.array([0, len(w5)]), b["lam"][5:6], 2, 300, 100, 9, kz,
                    wave_id=np.array([5], np.uint64))
    np.testing.assert_array_equal(r3.z, r1.z[10:12])
    np.testing.assert_array_equal(r3.acc, r1.acc[10:12])
    # a different seed changes the chains
    r4 = oracle.run(p, b["wave"], b["offsets"], b["lam"], 2, 300, 100, 10, kz)
    assert not np.array_equal(r4.acc, r1.acc)


def test_replay_of_own_log():
    p = oracle.make_params()
    from paper_2403_03156_amd import synth
    b = synth.generate(synth.PRESETS["plain"], n_wave=4, seed=4)
    kz = 16
    r = oracle.run(p, b["wave"], b["offsets"], b["lam"], 1, 400, 200, 11, kz, log=True)
    o = b["offsets"]
    for i in range(4):
        w = b["wave"][o[i]:o[i + 1]]
        dnu, la, bad = oracle.replay(p, w, b["lam"][i], kz, 0, 4 * len(w) - 1, i, 11, r.log[i])
        assert bad == 0
        valid = (r.log[i]["flags"] & 1) != 0
        np.testing.assert_array_equal(dnu[valid], r.log[i]["dnu"][valid])
        assert valid.sum() > 100


def test_per_waveform_sweeps_equal_separate_runs():
    """wsteps: every waveform runs its own sweep count with burn-in wsteps * burn_in // n_steps,
    the same chains as separate runs of each count"""
    p = oracle.make_params()
    rng = np.random.default_rng(8)
    L, n = 96, 5
    wave = (0.1 * rng.standard_normal(n * L)).astype(np.float32)
    off = np.arange(n + 1, dtype=np.int64) * L
    lam = np.full(n, 2.0)
    steps = np.array([40, 100, 73, 100, 1], np.int32)
    r = oracle.run(p, wave, off, lam, 2, 100, 50, 9, 8, wsteps=steps)
    for i, s in enumerate(steps):
        one = oracle.run(p, wave[off[i]:off[i + 1]], np.array([0, L], np.int64), lam[i:i + 1], 2, int(s),
                         int(s) * 50 // 100, 9, 8, wave_id=np.array([i], np.uint64))
        np.testing.assert_array_equal(r.z[2 * i:2 * i + 2], one.z)
        np.testing.assert_array_equal(r.nhist[2 * i:2 * i + 2], one.nhist)
        np.testing.assert_array_equal(r.acc[2 * i:2 * i + 2], one.acc)
