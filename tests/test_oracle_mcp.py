"""The oracle's MCP-PMT form (Sec. 2.1 Gaussian-mixture charge law, Sec. 2.4 eq. mcp, App. A
for MCP-PMTs) against the dense definitions:

* log p(w | z, e) against the dense normal law with per-PE means and variances, and the
  charges' conditional mean against least squares on the augmented system;
* tiny grids: the chain's P(N = k), E[N], E[Q] and the expected PEs per component against
  enumeration of every multiset of (grid point, component) pairs;
* with one component equal to the single normal law the chain is the dynode chain;
* data term off: components of the PEs follow G.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from tests.test_oracle_chain import _tiny, _wave

MIX = ([0.6, 0.4], [1.0, 2.2], [0.3, 0.6])


def _mcp(kind=0):
    p, m = _tiny(kind)
    p.n_mix = 2
    for i in range(2):
        p.mix_w[i], p.mix_mu[i], p.mix_sigma[i] = MIX[0][i], MIX[1][i], MIX[2][i]
    return p, m


def test_likelihood_and_charges_match_dense_definitions():
    p, m = _mcp()
    rng = np.random.default_rng(4)
    for trial in range(20):
        K = int(rng.integers(1, 5))
        z = rng.integers(0, 40, K).tolist()
        e = rng.integers(0, 2, K).tolist()
        w = rng.normal(0.5, 0.4, 14).astype(np.float32)
        ll, x = oracle.log_likelihood(p, w, z, e)
        assert ll == pytest.approx(brute.dense_logp_mix(m, w.astype(np.float64), z, e, MIX), rel=1e-10)
        np.testing.assert_allclose(x, brute.charge_mean_mix(m, w.astype(np.float64), z, e, MIX), rtol=1e-8, atol=1e-10)


def test_mcp_chain_matches_enumeration():
    p, m = _mcp()
    Lw, glo, ghi, kmax, lam = 12, 6, 13, 2, 1.4
    w = _wave(m, Lw, [8, 12], [1.0, 2.3], seed=31)
    exact = brute.posterior_exact_mix(m, w.astype(np.float64), lam, glo, ghi, kmax, 1.0, MIX)
    C, n_steps, burn = 48, 30000, 1500
    r = oracle.run(p, w, np.array([0, Lw], np.int64), np.array([lam]), C, n_steps, burn, 7, kz=kmax,
                   kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32))
    s = oracle.summarize(r.acc, n_steps, burn, C)
    _, mc = oracle.chain_diagnostics(r.acc, n_steps - burn, C)
    for a, (name, want) in enumerate((("N", exact["EN"]), ("Q", exact["EQ"]))):
        assert abs(s[name][0][0] - want) < 4 * mc[0, a] + 1e-12, (name, s[name][0][0], want, mc[0, a])
    pN = r.nhist.sum(0)[: kmax + 1] / r.nhist.sum()
    np.testing.assert_allclose(pN, exact["pN"], atol=0.012)
    # components of the final states of many short chains against the enumerated expectation
    C2 = 800
    r2 = oracle.run(p, w, np.array([0, Lw], np.int64), np.array([lam]), C2, 400, 200, 9, kz=kmax,
                    kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32))
    ne = np.array([[(r2.e[c] == q).sum() for q in range(2)] for c in range(C2)], np.float64)
    for q in range(2):
        se = ne[:, q].std() / np.sqrt(C2)
        assert abs(ne[:, q].mean() - exact["En_e"][q]) < 4 * se + 1e-3, (q, ne[:, q].mean(), exact["En_e"][q])


def test_single_component_is_the_dynode_chain():
    p, m = _tiny(1)
    q = oracle.make_params(ser=(1.0, 0.5, 1.0), ser_support=16, sigma_eps=0.3, sigma_q=0.4, mu_q=1.0, phi_kind=1,
                           tau_rise=0.7, tau_decay=2.0, t0_min=1.0, t0_max=1.0, shift_sd=0.5, t0_sd=0.3,
                           mix=([1.0], [1.0], [0.4]))
    Lw, glo, ghi, kmax, lam = 12, 6, 17, 3, 1.6
    w = _wave(m, Lw, [8, 13], [1.0, 0.8], seed=22)
    args = (w, np.array([0, Lw], np.int64), np.array([lam]), 4, 3000, 1000, 5)
    kw = dict(kz=kmax, kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32))
    a = oracle.run(p, *args, **kw)
    b = oracle.run(q, *args, **kw)
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.nhist, b.nhist)
    np.testing.assert_allclose(a.acc, b.acc, rtol=1e-10)
    assert (b.e[b.z >= 0] == 0).all()


def test_prior_only_components_follow_G():
    p, m = _mcp()
    p.ser_amp = 0.0
    Lw, glo, ghi, kmax, lam = 24, 0, 95, 12, 3.0
    r = oracle.run(p, np.zeros(Lw, np.float32), np.array([0, Lw], np.int64), np.array([lam]), 400, 600, 300, 3,
                   kz=kmax, kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32))
    e = r.e[r.e >= 0]
    frac = (e == 1).mean()
    assert abs(frac - MIX[0][1]) < 4 * np.sqrt(0.24 / len(e)), (frac, len(e))
