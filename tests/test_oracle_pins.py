"""Pins for the oracle: every check compares it with something other than itself.

* Philox4x32-10 against published known-answer vectors, and an independent Python
  Philox whose 4x64 instance is checked against numpy's bit generator.
* SER against scipy's ``exponnorm`` and the paper's erf form (Sec. 3).
* phi normalisation by quadrature; BIEXP as the convolution of two exponentials.
* the grid normaliser Lambda_T and the birth draw against direct grid sums.
* log p(w|z) against the dense normal law (App. A, eq. mgauss).
* delta-nu against the paper's Woodbury form (App. A, eqs. 11-18).
* charge means against least squares on the augmented system.
* acceptances (Sec. 2.4) through exact stationarity of the full transition matrix.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


def philox_py(ctr, key, W, rounds=10):
    """Philox-4xW (Salmon et al. 2011), written independently of the C oracle."""
    if W == 32:
        mask, M0, M1, W0, W1 = M32, 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    else:
        mask, M0, M1, W0, W1 = M64, 0xD2E7470EE14C6C93, 0xCA5A826395121157, 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
    c, k = list(ctr), list(key)
    for _ in range(rounds):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [(p1 >> W) ^ c[1] ^ k[0], p1 & mask, (p0 >> W) ^ c[3] ^ k[1], p0 & mask]
        k = [(k[0] + W0) & mask, (k[1] + W1) & mask]
    return c


def test_philox_py_matches_numpy_4x64():
    # numpy's Philox bit generator is Philox4x64-10; it bumps the counter before each block
    for key, ctr in [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 8, 9, 10)), ((M64, 1), (M64 - 1, 5, 0, M64))]:
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        got = [int(v) for v in bg.random_raw(4)]
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) & M64
        if nxt[0] == 0:
            nxt[1] = (nxt[1] + 1) & M64
        assert got == philox_py(nxt, key, 64)


def test_philox4x32_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert philox_py(ctr, key, 32) == want
        assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == want


def test_philox4x32_oracle_matches_py_random():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 1 << 32, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64)]
        assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == philox_py(ctr, key, 32)


# ---------------------------------------------------------------- SER
@pytest.mark.parametrize("ser", [(8.0, 1.5, 6.0), (6.0, 1.0, 3.0), (4 * 1.62, 1.62, 7.2)])
def test_ser_table_matches_exponnorm(ser):
    p = oracle.make_params(ser=ser)
    tab, LV = oracle.ser_table(p)
    d = stats.exponnorm(K=ser[2] / ser[1], loc=ser[0], scale=ser[1])
    tp = oracle.lib().ora_ser_peak_time(*ser)
    # the oracle's peak is a true maximum of the scipy density
    grid = np.linspace(tp - 0.05, tp + 0.05, 20001)
    assert d.pdf(tp) >= d.pdf(grid).max() * (1 - 1e-12)
    m = np.arange(len(tab))
    want = d.pdf(m / 4.0) / d.pdf(tp)
    np.testing.assert_allclose(tab, want, rtol=1e-10, atol=1e-15)
    assert 0.999 < tab.max() <= 1.0 + 1e-15  # the grid need not hit the peak time


def test_ser_paper_form_is_exponnorm_with_mean_4sigma():
    # Sec. 3: V(t) = 1/(2 tau) exp((sigma^2 - 2 (t - 4 sigma) tau) / (2 tau^2)) (1 + erf(-(sigma^2 - (t - 4 sigma) tau)/(sqrt2 sigma tau)))
    sigma, tau = 1.62, 7.2
    t = np.linspace(0, 80, 801)
    paper = 1 / (2 * tau) * np.exp((sigma ** 2 - 2 * (t - 4 * sigma) * tau) / (2 * tau ** 2)) * (
        1 + special.erf(-(sigma ** 2 - (t - 4 * sigma) * tau) / (math.sqrt(2) * sigma * tau)))
    d = stats.exponnorm(K=tau / sigma, loc=4 * sigma, scale=sigma)
    np.testing.assert_allclose(paper, d.pdf(t), rtol=1e-9, atol=1e-14)
    # and the oracle's un-normalised value matches it (amplitude = 1 / peak)
    p = oracle.make_params(ser=(4 * sigma, sigma, tau), ser_support=128)
    tp = oracle.lib().ora_ser_peak_time(4 * sigma, sigma, tau)
    vals = np.array([oracle.lib().ora_ser_value(p, x) for x in t[:-1]])
    np.testing.assert_allclose(vals * d.pdf(tp), paper[:-1], rtol=1e-9, atol=1e-14)


def test_ser_support_rule():
    assert oracle.lib().ora_ser_support_auto(8.0, 1.5, 6.0) == 96
    assert oracle.lib().ora_ser_support_auto(6.0, 1.0, 3.0) == 64
    for ser in [(8.0, 1.5, 6.0), (6.0, 1.0, 3.0)]:
        L = oracle.lib().ora_ser_support_auto(*ser)
        d = stats.exponnorm(K=ser[2] / ser[1], loc=ser[0], scale=ser[1])
        tp = oracle.lib().ora_ser_peak_time(*ser)
        assert d.pdf(L) / d.pdf(tp) < 1e-6 <= d.pdf(L - 16) / d.pdf(tp)


# ---------------------------------------------------------------- phi
@pytest.mark.parametrize("kind,t1,t2", [(0, 0.0, 20.0), (1, 2.0, 25.0), (1, 1.16, 26.76)])
def test_phi_normalised(kind, t1, t2):
    p = oracle.make_params(phi_kind=kind, tau_rise=t1, tau_decay=t2)
    f = lambda t: oracle.lib().ora_phi(p, t)
    val, err = integrate.quad(f, 0, np.inf, limit=200)
    assert abs(val - 1.0) < 1e-9
    assert f(-0.1) == 0.0


def test_biexp_is_convolution_of_exponentials():
    t1, t2 = 2.0, 25.0
    t12 = t1 * t2 / (t1 + t2)
    p = oracle.make_params(phi_kind=1, tau_rise=t1, tau_decay=t2)
    for t in [0.3, 1.0, 4.0, 17.0, 60.0]:
        conv, _ = integrate.quad(lambda s: np.exp(-s / t2) / t2 * np.exp(-(t - s) / t12) / t12, 0, t)
        assert abs(oracle.lib().ora_phi(p, t) - conv) < 1e-12


# ---------------------------------------------------------------- Lambda_T, h
@pytest.mark.parametrize("kind,t1,t2", [(0, 0.0, 20.0), (1, 2.0, 25.0)])
def test_lambda_T_matches_direct_grid_sum(kind, t1, t2):
    p = oracle.make_params(phi_kind=kind, tau_rise=t1, tau_decay=t2)
    m = brute.Model(phi_kind=kind, tau_rise=t1, tau_decay=t2)
    for t0 in [50.0, 73.3, 75.25, 99.999, 0.0, 300.0]:
        for glo, ghi in [(0, 1023), (0, 4095), (210, 260), (400, 400), (5000, 6000)]:
            want = m.Lambda_T(3.7, t0, glo, ghi)
            got = oracle.lib().ora_lambda_T(p, 3.7, t0, glo, ghi)
            assert abs(got - want) <= 1e-12 * max(1.0, want), (t0, glo, ghi, got, want)


@pytest.mark.parametrize("kind,t1,t2", [(0, 0.0, 20.0), (1, 2.0, 25.0)])
def test_birth_draw_is_inverse_cdf_of_h(kind, t1, t2):
    p = oracle.make_params(phi_kind=kind, tau_rise=t1, tau_decay=t2)
    m = brute.Model(phi_kind=kind, tau_rise=t1, tau_decay=t2)
    rng = np.random.default_rng(3)
    for t0 in [50.0, 61.7, 99.0]:
        glo, ghi = 0, 1023
        cdf = np.cumsum(m.h(t0, glo, ghi))
        for u in np.concatenate([rng.uniform(0, 1, 300), [1e-12, 0.5, 1 - 1e-12]]):
            g = oracle.lib().ora_birth_draw(p, t0, glo, ghi, u)
            want = glo + int(np.searchsorted(cdf, u, side="right"))
            if abs(cdf[want - glo] - u) > 1e-12 and (want == glo or abs(cdf[want - glo - 1] - u) > 1e-12):
                assert g == want, (t0, u, g, want)
            assert m.phi(g / 4 - t0) > 0


# ---------------------------------------------------------------- likelihood
def _small_case(seed, Lw=48, LV=16, K=3, ser=(3.0, 0.8, 2.0), sigma_eps=0.2, sigma_q=0.3, mu_q=1.0):
    rng = np.random.default_rng(seed)
    p = oracle.make_params(ser=ser, ser_support=LV, sigma_eps=sigma_eps, sigma_q=sigma_q, mu_q=mu_q)
    m = brute.Model(ser=ser, LV=LV, sigma_eps=sigma_eps, sigma_q=sigma_q, mu_q=mu_q)
    z = [int(g) for g in rng.integers(0, 4 * Lw, K)]
    w = np.zeros(Lw)
    for g in z:
        w += rng.normal(1.0, 0.3) * m.column(g, Lw)
    w += sigma_eps * rng.standard_normal(Lw)
    return p, m, np.asarray(w, np.float32), z


@pytest.mark.parametrize("seed", range(6))
def test_loglik_matches_dense_mvn(seed):
    p, m, w, z = _small_case(seed, K=1 + seed % 4)
    if seed == 5:
        z = z[:1] * 2 + z[1:]                         # repeated grid point
    if seed == 4:
        z = z + [4 * len(w) - 3]                      # column cut by the window end
    got, x = oracle.log_likelihood(p, w, z)
    want = brute.dense_logp(m, w.astype(np.float64), z)
    assert abs(got - want) < 1e-9 * max(1.0, abs(want))
    np.testing.assert_allclose(x, brute.charge_mean(m, w.astype(np.float64), z), rtol=1e-8, atol=1e-10)
    got0, _ = oracle.log_likelihood(p, w, [])
    assert abs(got0 - brute.dense_logp(m, w.astype(np.float64), [])) < 1e-9 * abs(got0)


@pytest.mark.parametrize("seed", range(5))
def test_delta_nu_matches_paper_woodbury(seed):
    p, m, w, z = _small_case(100 + seed, K=3)
    wd = w.astype(np.float64)
    lam, glo, ghi, t0 = 2.0, 0, 4 * len(w) - 1, 0.0
    rng = np.random.default_rng(seed)
    gnew = int(rng.integers(0, 4 * len(w)))
    # birth
    _, dnu = oracle.log_alpha(p, w, lam, glo, ghi, t0, z, oracle.MOVE_BIRTH, -1, gnew)
    want = brute.paper_dnu(m, wd, z, None, gnew)
    dense = brute.dense_logp(m, wd, z + [gnew]) - brute.dense_logp(m, wd, z)
    assert abs(dnu - want) < 1e-8 * max(1, abs(want)) and abs(dnu - dense) < 1e-8 * max(1, abs(dense))
    # death of j = 1 (the last PE moves into slot 1)
    _, dnu = oracle.log_alpha(p, w, lam, glo, ghi, t0, z, oracle.MOVE_DEATH, 1, -1)
    want = brute.paper_dnu(m, wd, z, z[1], None)
    assert abs(dnu - want) < 1e-8 * max(1, abs(want))
    # update of j = 2 to gnew
    _, dnu = oracle.log_alpha(p, w, lam, glo, ghi, t0, z, oracle.MOVE_UPDATE, 2, gnew)
    want = brute.paper_dnu(m, wd, z, z[2], gnew)
    assert abs(dnu - want) < 1e-8 * max(1, abs(want))


def test_overlap_against_columns():
    p = oracle.make_params(ser=(3.0, 0.8, 2.0), ser_support=16)
    m = brute.Model(ser=(3.0, 0.8, 2.0), LV=16)
    Lw = 40
    for g1, g2 in [(0, 0), (5, 9), (9, 5), (150, 158), (158, 159), (100, 180), (3, 70)]:
        want = float(m.column(g1, Lw) @ m.column(g2, Lw))
        assert abs(oracle.lib().ora_overlap(p, Lw, g1, g2) - want) < 1e-12


# ---------------------------------------------------------------- acceptance: exact stationarity
def _tiny_model(kind=0):
    ser = (1.0, 0.5, 1.0)
    kw = dict(ser=ser, sigma_eps=0.3, sigma_q=0.4, mu_q=1.0, phi_kind=kind, tau_rise=0.7 if kind else 0.0,
              tau_decay=2.0, t0_min=1.0, t0_max=1.0, J=0.25, shift_sd=0.5)
    p = oracle.make_params(ser_support=16, **kw)
    kw.pop("shift_sd")
    m = brute.Model(LV=16, shift_sd=0.5, **kw)
    return p, m


def _transition_matrix(p, m, w, lam, glo, ghi, t0, kmax, alpha_fn):
    states = list(brute.multisets(glo, ghi, kmax))
    index = {s: i for i, s in enumerate(states)}
    n = len(states)
    P = np.zeros((n, n))
    h = m.h(t0, glo, ghi)
    smax = 12
    shifts = np.arange(-smax, smax + 1)
    pm = brute.shift_pmf(m, shifts)
    for i, s in enumerate(states):
        z = list(s)
        N = len(z)
        pb = 1.0 if N == 0 else m.J
        if N < kmax:
            for k, g in enumerate(range(glo, ghi + 1)):
                if h[k] == 0:
                    continue
                la = alpha_fn(z, oracle.MOVE_BIRTH, -1, g)
                a = min(1.0, math.exp(la)) if la > -np.inf else 0.0
                P[i, index[tuple(sorted(z + [g]))]] += pb * h[k] * a
        if N > 0:
            for j in range(N):
                la = alpha_fn(z, oracle.MOVE_DEATH, j, -1)
                a = min(1.0, math.exp(la)) if la > -np.inf else 0.0
                zz = z[:j] + z[j + 1:]
                P[i, index[tuple(sorted(zz))]] += m.J / N * a
                for sh, ps in zip(shifts, pm):
                    gn = z[j] + int(sh)
                    la = alpha_fn(z, oracle.MOVE_UPDATE, j, gn)
                    a = min(1.0, math.exp(la)) if la > -np.inf else 0.0
                    if a > 0:
                        zu = z.copy()
                        zu[j] = gn
                        P[i, index[tuple(sorted(zu))]] += (1 - 2 * m.J) / N * ps * a
        P[i, i] += 1.0 - P[i].sum()
    return states, P


@pytest.mark.parametrize("kind", [0, 1])
def test_exact_stationarity(kind):
    p, m = _tiny_model(kind)
    rng = np.random.default_rng(11 + kind)
    Lw, glo, ghi, kmax, lam, t0 = 12, 8, 14, 3, 1.7, 1.0
    w = np.zeros(Lw)
    for g in (9, 12):
        w += m.column(g, Lw)
    w = (w + 0.3 * rng.standard_normal(Lw)).astype(np.float32)
    fn = lambda z, mv, j, g: oracle.log_alpha(p, w, lam, glo, ghi, t0, z, mv, j, g)[0]
    states, P = _transition_matrix(p, m, w, lam, glo, ghi, t0, kmax, fn)
    assert np.all(P >= -1e-15)
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-13)
    post = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=t0)
    pi = post["weights"]
    assert np.abs(pi @ P - pi).max() < 1e-12


def test_stationarity_catches_planted_mistake():
    # dropping the empty-sequence factor J from the birth acceptance must break pi P = pi
    p, m = _tiny_model(0)
    Lw, glo, ghi, kmax, lam, t0 = 12, 8, 12, 2, 1.7, 1.0
    w = (0.5 * m.column(9, Lw)).astype(np.float32)

    def wrong(z, mv, j, g):
        la = oracle.log_alpha(p, w, lam, glo, ghi, t0, z, mv, j, g)[0]
        if mv == oracle.MOVE_BIRTH and len(z) == 0:
            la -= math.log(m.J)
        return la

    states, P = _transition_matrix(p, m, w, lam, glo, ghi, t0, kmax, wrong)
    pi = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=t0)["weights"]
    assert np.abs(pi @ P - pi).max() > 1e-4


@pytest.mark.parametrize("kind", [0, 1])
def test_t0_acceptance_is_conditional_ratio(kind):
    p, m = _tiny_model(kind)
    p.t0_min, p.t0_max = 0.0, 3.0
    glo, ghi, lam = 4, 30, 2.5
    rng = np.random.default_rng(5)
    for _ in range(40):
        z = [int(g) for g in rng.integers(glo, ghi + 1, rng.integers(0, 4))]
        t0, t0p = rng.uniform(0, 3, 2)
        la = oracle.t0_log_alpha(p, lam, glo, ghi, z, t0, t0p)
        a = brute.log_prior(m, z, lam, t0p, glo, ghi)
        b = brute.log_prior(m, z, lam, t0, glo, ghi)
        if b == -np.inf:
            continue
        want = a - b
        if want == -np.inf:
            assert la == -np.inf
        else:
            assert abs(la - want) < 1e-10
    assert oracle.t0_log_alpha(p, lam, glo, ghi, [10], 1.0, 3.5) == -np.inf
