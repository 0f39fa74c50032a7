"""The oracle's convergence diagnostics and lambda estimate against hand-derived values,
closed forms and brute force.

* Gelman-Rubin R (Sec. 3.2 convergence check) on two chains worked by hand:
  (1, -1, 1, -1) and (3, 1, 3, 1) give W = 4/3, B = 8, V = 3, R = 1.5, and a
  between-chain MCSE of 1; constant chains give 1 (equal) or inf (different);
* R near 1 for long independent chains of one law, well above 1.1 for chains of two
  laws; the accumulator form against the recorded traces of real chains;
* lambda-hat (eq. reduce-mu0): a single sampled N = k gives k (f = -lambda + k log lambda);
  h_0 = h_1 gives 1 - lambda0 for lambda0 < 1 (f' = -1 + 1 / (lambda0 + lambda)) and the
  boundary 0 above; random histograms against a dense brute-force maximisation of f.
"""
import math

import numpy as np
import pytest

import oracle


def _acc_from_traces(tr):
    """[C][S] samples of one quantity -> accumulator rows with that quantity in slots 0, 1."""
    tr = np.asarray(tr, np.float64)
    acc = np.zeros((tr.shape[0], 12))
    acc[:, 0] = tr.sum(1)
    acc[:, 1] = (tr ** 2).sum(1)
    acc[:, 2:6] = np.tile(acc[:, 0:2], 2)
    return acc


def test_rhat_hand_worked_example():
    acc = _acc_from_traces([[1, -1, 1, -1], [3, 1, 3, 1]])
    r, mc = oracle.chain_diagnostics(acc, 4, 2)
    assert r[0, 0] == pytest.approx(1.5, rel=1e-15)
    assert mc[0, 0] == pytest.approx(1.0, rel=1e-15)


def test_rhat_edge_cases():
    r, _ = oracle.chain_diagnostics(_acc_from_traces([[2, 2, 2], [2, 2, 2]]), 3, 2)
    assert r[0, 0] == 1.0
    r, _ = oracle.chain_diagnostics(_acc_from_traces([[2, 2, 2], [5, 5, 5]]), 3, 2)
    assert np.isinf(r[0, 0])
    r, mc = oracle.chain_diagnostics(_acc_from_traces([[1, 2, 3]]), 3, 1)
    assert np.isnan(r[0, 0]) and np.isnan(mc[0, 0])


def test_rhat_detects_disagreeing_chains():
    rng = np.random.default_rng(1)
    same = rng.standard_normal((4, 20000))
    r, mc = oracle.chain_diagnostics(_acc_from_traces(same), 20000, 4)
    assert abs(r[0, 0] - 1.0) < 0.01
    # the MCSE of a mean of 80,000 iid unit normals is 1/sqrt(80000); 3 chain-spread dof
    assert 0.2 / math.sqrt(80000) < mc[0, 0] < 3.0 / math.sqrt(80000)
    split = same + np.array([0.0, 0.0, 1.0, 1.0])[:, None]
    r, _ = oracle.chain_diagnostics(_acc_from_traces(split), 20000, 4)
    assert r[0, 0] > 1.1


def test_rhat_from_accumulators_of_real_chains_matches_traces():
    p = oracle.make_params(t0_min=0.0, t0_max=10.0)
    rng = np.random.default_rng(2)
    L = 64
    w = (0.1 * rng.standard_normal(L)).astype(np.float32)
    n = np.arange(L)
    for t in (12.0, 30.0, 31.5):
        w += np.exp(-0.5 * ((n - t - 4) / 1.5) ** 2).astype(np.float32)
    C, n_steps, burn = 4, 600, 200
    r = oracle.run(p, w, np.array([0, L], np.int64), np.array([5.0]), C, n_steps, burn, 3, 16, thin=1)
    rh, mc = oracle.chain_diagnostics(r.acc, n_steps - burn, C)
    for a, col in enumerate((0, 2, 1)):   # trace columns: N, t0, Q
        x = r.trace[:, :, col]
        m = x.mean(1)
        W = x.var(1, ddof=1).mean()
        B = x.shape[1] * m.var(ddof=1)
        want = math.sqrt(((x.shape[1] - 1) / x.shape[1] * W + B / x.shape[1]) / W)
        assert rh[0, a] == pytest.approx(want, rel=1e-8)
        assert mc[0, a] == pytest.approx(m.std(ddof=1) / math.sqrt(C), rel=1e-8)


def test_lambda_hat_closed_forms():
    for k in (0, 1, 7, 40):
        h = np.zeros(64)
        h[k] = 123.0
        assert oracle.lambda_mle(h, 3.0) == k
    for lam0 in (0.1, 0.25, 0.6, 0.9):
        assert oracle.lambda_mle([5.0, 5.0], lam0) == pytest.approx(1.0 - lam0, abs=1e-12)
    for lam0 in (1.0, 2.0, 7.5):
        assert oracle.lambda_mle([5.0, 5.0], lam0) == 0.0


def test_lambda_hat_against_dense_maximisation():
    rng = np.random.default_rng(4)
    for trial in range(40):
        K = int(rng.integers(2, 40))
        lam0 = float(rng.uniform(0.2, 30.0))
        mu = float(rng.uniform(0.1, K))
        # a smooth sampled-N histogram (Poisson-shaped around mu), some with gaps
        h = np.array([math.exp(k * math.log(mu) - mu - math.lgamma(k + 1)) for k in range(K + 1)])
        h = np.floor(h / h.max() * 1000.0)
        if trial % 3 == 0:
            h[rng.integers(0, K + 1)] = 0.0
        if (h > 0).sum() == 0:
            continue
        est = oracle.lambda_mle(h, lam0)
        ks = np.arange(K + 1)
        lo, hi = ks[h > 0][0], ks[h > 0][-1]
        xs = np.linspace(lo, hi, 200001)
        lh = np.where(h > 0, np.log(np.where(h > 0, h, 1.0)), -np.inf)
        with np.errstate(divide="ignore", invalid="ignore"):
            a = lh[None, :] + ks[None, :] * np.log(xs[:, None] / lam0)
        a[xs == 0, :] = np.where(ks == 0, lh, -np.inf)
        mx = a.max(1)
        f = -(xs - lam0) + mx + np.log(np.exp(a - mx[:, None]).sum(1))
        best = xs[np.argmax(f)]
        assert abs(est - best) <= 2 * (hi - lo) / 200000 + 1e-9, (trial, est, best)
