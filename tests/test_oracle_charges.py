"""Pins for the oracle's charge draws (Sec. 2.1 charge model; App. A, eq. mgauss read as
Bayesian linear regression): q | z, w ~ N(x, sigma_eps^2 G^-1), drawn as
q = x + sigma_eps L^-T xi with G = L L^T.

* xi = 0 gives the least-squares posterior mean of the augmented system;
* unit vectors xi = e_k give the columns of the upper-triangular factor R = L^-T of
  G^-1 = R R^T, with G and its Cholesky factor taken from numpy on the dense columns;
* the normals follow the documented Philox counter layout (block 2 + k/2, Box-Muller
  cosine for even k, sine for odd k), re-derived with an independent Philox;
* the chain driver records, at every thinned step, the PE list and the draw for that
  list with that step's normals.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from tests.test_oracle_pins import _small_case, philox_py


def _dense_gram(m, w, z):
    A = m.A(z, len(w))
    rho = m.sigma_eps ** 2 / m.sigma_q ** 2
    return A.T @ A + rho * np.eye(len(z))


@pytest.mark.parametrize("seed", range(4))
def test_zero_normals_give_posterior_mean(seed):
    p, m, w, z = _small_case(300 + seed, K=2 + seed)
    q = oracle.charge_draw(p, w, z, np.zeros(len(z)))
    np.testing.assert_allclose(q, brute.charge_mean(m, w.astype(np.float64), z), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_unit_normals_give_upper_factor_of_inverse_gram(seed):
    p, m, w, z = _small_case(400 + seed, K=2 + seed)
    if seed == 3:
        z = z[:1] * 2 + z[1:]  # repeated grid point: G stays positive definite through rho
    K = len(z)
    x = oracle.charge_draw(p, w, z, np.zeros(K))
    R = np.zeros((K, K))
    for k in range(K):
        e = np.zeros(K)
        e[k] = 1.0
        R[:, k] = (oracle.charge_draw(p, w, z, e) - x) / m.sigma_eps
    G = _dense_gram(m, w.astype(np.float64), z)
    Ln = np.linalg.cholesky(G)
    np.testing.assert_allclose(R, np.linalg.inv(Ln).T, rtol=1e-8, atol=1e-11)
    assert np.allclose(np.tril(R, -1), 0.0, atol=1e-14)          # upper triangular
    np.testing.assert_allclose(R @ R.T, np.linalg.inv(G), rtol=1e-8, atol=1e-11)


def test_charge_draw_moments():
    p, m, w, z = _small_case(500, K=4)
    K = len(z)
    rng = np.random.default_rng(1)
    xi = rng.standard_normal((20000, K))
    q = np.stack([oracle.charge_draw(p, w, z, v) for v in xi])
    G = _dense_gram(m, w.astype(np.float64), z)
    cov = m.sigma_eps ** 2 * np.linalg.inv(G)
    mean = brute.charge_mean(m, w.astype(np.float64), z)
    se = np.sqrt(np.diag(cov) / len(q))
    assert (np.abs(q.mean(0) - mean) < 5 * se).all()
    emp = np.cov(q.T)
    assert np.abs(emp - cov).max() < 0.1 * np.abs(cov).max()


def test_charge_normals_counter_layout():
    uid, seed, step, K = (7 << 16) | 3, 0x1234_5678_9ABC, 321, 7
    got = oracle.charge_normals(uid, seed, step, K)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    want = []
    for k in range(K):
        r = philox_py([step, 2 + k // 2, uid & 0xFFFFFFFF, uid >> 32], key, 32)
        R = math.sqrt(-2.0 * math.log((r[0] + 0.5) / 2 ** 32))
        th = 2.0 * math.pi * (r[1] + 0.5) / 2 ** 32
        want.append(R * (math.cos(th) if k % 2 == 0 else math.sin(th)))
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-15)


def test_run_records_charge_draws():
    p, m, w, z = _small_case(600, Lw=64, K=4)
    p.t0_min, p.t0_max = 0.0, 10.0  # PEs can sit anywhere in the 64-sample window
    lam = np.array([6.0])
    off = np.array([0, len(w)], np.int64)
    n_steps, burn, thin, seed, kz = 240, 100, 7, 5, 16
    r = oracle.run(p, w, off, lam, 1, n_steps, burn, seed, kz, thin=thin, charges=True)
    n_rec = (n_steps - burn + thin - 1) // thin
    assert r.qdraw.shape == (1, n_rec, kz) and r.zdraw.shape == (1, n_rec, kz)
    seen_nonempty = 0
    for i in range(n_rec):
        N = int(r.trace[0, i, 0])
        zl = r.zdraw[0, i]
        assert (zl[:N] >= 0).all() and (zl[N:] == -1).all()
        assert (r.qdraw[0, i, N:] == 0.0).all()
        if N == 0:
            continue
        seen_nonempty += 1
        step = burn + i * thin
        xi = oracle.charge_normals(0, seed, step, N)
        want = oracle.charge_draw(p, w, zl[:N], xi)
        np.testing.assert_allclose(r.qdraw[0, i, :N], want, rtol=1e-12, atol=1e-12)
        # the Rao-Blackwellised total charge of the trace is the draw's mean
        x = oracle.charge_draw(p, w, zl[:N], np.zeros(N))
        assert abs(x.sum() - r.trace[0, i, 2]) < 1e-9 * max(1.0, abs(x.sum()))
    assert seen_nonempty > n_rec // 2
