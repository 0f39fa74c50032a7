"""The oracle's Lucy-Richardson initialisation (Sec. 2.3) against what fixes it:

* the two sums as printed (with the convolution's limits) on a small case, term by term;
* flux: after every iteration the total of qhat times sum(V) equals the total of the
  clipped data over the samples where w^r > 0 (sum_tau qhat^{r+1}(tau) = sum_t ratio(t)
  w^r(t)), which holds only if the two sums are exact adjoints;
* fixed point: data that are exactly u * K for a non-negative u whose kernel support lies
  inside the window are reproduced by one iteration from u;
* recovery: a noise-free waveform of PEs on whole samples converges to those PEs with
  their charges, and the initial state (list, T, cut, t0) follows from it;
* degenerate data (no positive sample) give no PE and an empty T.
"""
import numpy as np
import pytest

import oracle
from oracle import lucy


def _V(LV=24):
    s = np.arange(LV, dtype=np.float64)
    v = (s / 3.0) ** 2 * np.exp(-s / 3.0)
    return v / v.max()


def _literal(w, V, n_iter):
    Lw, LV = len(w), len(V)
    A = V.sum()
    K = V / A
    d = np.maximum(w, 0.0)
    u = {tau: d.sum() / (Lw + LV - 1) for tau in range(-LV + 1, Lw)}
    for _ in range(n_iter):
        wr = {t: sum(u[tau] * K[t - tau] for tau in range(max(t - LV + 1, -LV + 1), min(t, Lw - 1) + 1))
              for t in range(Lw)}
        u = {tau: u[tau] * sum((d[t] / wr[t] if wr[t] > 0 else 0.0) * K[t - tau]
                               for t in range(max(tau, 0), min(Lw - 1, tau + LV - 1) + 1)) for tau in u}
    return np.array([u[tau] for tau in range(-LV + 1, Lw)]) / A


def test_vectorised_equals_the_two_sums():
    rng = np.random.default_rng(0)
    V = _V(7)
    w = rng.normal(0.3, 0.5, 20)
    np.testing.assert_allclose(lucy.lucy(w, V, 5), _literal(w, V, 5), rtol=1e-13, atol=1e-15)


def test_flux_identity():
    rng = np.random.default_rng(1)
    V = _V()
    w = rng.normal(0.2, 0.4, 80)
    d = np.maximum(w, 0.0)
    for r in (1, 2, 7, 30):
        q = lucy.lucy(w, V, r)
        q_prev = lucy.lucy(w, V, r - 1) * V.sum()
        # samples where the previous model is positive
        wr = np.convolve(q_prev, V / V.sum())[len(V) - 1:len(V) - 1 + len(w)]
        assert q.sum() * V.sum() == pytest.approx(d[wr > 0].sum(), rel=1e-12)


def test_fixed_point():
    rng = np.random.default_rng(2)
    V = _V()
    Lw, LV = 60, len(V)
    u = np.zeros(Lw + LV - 1)
    inside = np.arange(LV - 1, LV - 1 + Lw - LV + 1)    # tau in [0, Lw - LV]
    u[inside] = rng.uniform(0.1, 2.0, len(inside))
    K = V / V.sum()
    w = np.convolve(u, K)[LV - 1:LV - 1 + Lw]
    # one iteration from u: the data's total is u's total, so start from u via a rescaled run
    ratio = (w > 0).astype(np.float64)
    rp = np.concatenate([np.zeros(LV - 1), ratio, np.zeros(LV - 1)])
    u1 = u * np.correlate(rp, K, "valid")
    np.testing.assert_allclose(u1[inside], u[inside], rtol=1e-13)
    # and the oracle's iteration from its own start converges towards data reproduction
    q = lucy.lucy(w, V, 400) * V.sum()
    wr = np.convolve(q, K)[LV - 1:LV - 1 + Lw]
    assert np.abs(wr - w).max() < 0.05 * w.max()


def test_recovers_separated_pes_and_initial_state():
    V = _V()
    Lw, LV, sub = 120, len(V), 4
    times, charges = [20, 45, 80], [1.0, 1.3, 0.8]
    w = np.zeros(Lw)
    for t, q in zip(times, charges):
        w[t:t + LV] += q * V[:Lw - t]
    qh = lucy.lucy(w, V, 2000)
    taus = np.arange(len(qh)) - (LV - 1)
    for t, q in zip(times, charges):
        assert qh[taus == t][0] == pytest.approx(q, rel=0.05)
    assert qh[~np.isin(taus, times)].max() < 0.05
    st = lucy.initial_state(qh, LV, sub, 0.1, 4, 16, 0.0, 100.0, Lw)
    assert st["z"] == [sub * t for t in times]
    assert st["g_range"] == (sub * (20 - 4), sub * (80 + 4))
    assert st["cut"] == (16, min(Lw - 1, 80 + 4 + LV))
    assert st["t0"] == pytest.approx(20 - 0.5 / sub)
    assert st["lam"] == pytest.approx(sum(charges), rel=0.02)
    # kmax keeps the largest qhat, in time order; the t0 prior clamps t0 and drops earlier PEs
    st2 = lucy.initial_state(qh, LV, sub, 0.1, 4, 2, 0.0, 100.0, Lw)
    assert st2["z"] == [sub * 20, sub * 45]
    st3 = lucy.initial_state(qh, LV, sub, 0.1, 4, 16, 30.0, 100.0, Lw)
    assert st3["t0"] == 30.0 and st3["z"] == [sub * 45, sub * 80]


def test_no_positive_sample_gives_no_pe():
    V = _V()
    qh = lucy.lucy(-np.abs(np.random.default_rng(3).normal(size=50)), V, 10)
    assert (qh == 0).all()
    st = lucy.initial_state(qh, len(V), 4, 0.1, 4, 16, 0.0, 100.0, 50)
    assert st["z"] == [] and st["g_range"][0] > st["g_range"][1]


def test_ser_samples_follow_the_table():
    p = oracle.make_params()
    V = lucy.ser_samples(p, 96)
    tab, LV = oracle.ser_table(p)
    assert V[0] == tab[0] and V[10] == tab[10 * p.sub]
    assert V.max() <= 1.0 + 1e-12 and V.argmax() == 10   # peak near 10.03 ns for (8, 1.5, 6)
