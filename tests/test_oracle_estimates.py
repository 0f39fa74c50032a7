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


def _batch_means_mcse(x):
    """[C][S] recorded values -> batch-means MCSE of the pooled mean, written out from the
    definition: floor(sqrt(S)) batches of S // floor(sqrt(S)) consecutive values per chain (the
    values past the last whole batch are left out), the unbiased variance of all C x nb batch
    means, divided by their number"""
    C, S = x.shape
    nb = int(math.isqrt(S))
    lb = S // nb
    bm = x[:, :nb * lb].reshape(C, nb, lb).mean(2).reshape(-1)
    return math.sqrt(bm.var(ddof=1) / bm.size)


def test_summarize_matches_batch_means_of_recorded_traces():
    """the pooled mean, variance and batch-means MCSE that summarize() forms from the chain
    driver's accumulators (sums and batch sums) against numpy on the thin = 1 trace of the same
    chains (S = 440 and 899 recorded sweeps: 20 batches of 22, and 29 batches of 31, so that a
    batch count swapped with a batch length fails)"""
    p = oracle.make_params(t0_min=0.0, t0_max=10.0)
    rng = np.random.default_rng(4)
    L = 64
    n = np.arange(L)
    waves = []
    for k in range(3):
        w = (0.1 * rng.standard_normal(L)).astype(np.float32)
        for t in rng.uniform(5, 40, k + 1):
            w += np.exp(-0.5 * ((n - t - 4) / 1.5) ** 2).astype(np.float32)
        waves.append(w)
    wave = np.concatenate(waves)
    off = np.arange(4, dtype=np.int64) * L
    C = 3
    for n_steps, burn in ((640, 200), (1099, 200)):
        r = oracle.run(p, wave, off, np.array([2.0, 4.0, 6.0]), C, n_steps, burn, 7, 16, thin=1)
        s = oracle.summarize(r.acc, n_steps, burn, C)
        tr = r.trace.reshape(3, C, n_steps - burn, 3)
        for name, col in (("N", 0), ("t0", 1), ("Q", 2)):
            mean, var, mcse = s[name]
            for i in range(3):
                x = tr[i, :, :, col]
                assert mean[i] == pytest.approx(x.mean(), rel=1e-12, abs=1e-12)
                assert var[i] == pytest.approx(x.var(), rel=1e-9, abs=1e-12)
                assert mcse[i] == pytest.approx(_batch_means_mcse(x), rel=1e-8, abs=1e-12)


def test_summarize_mcse_of_ar1_chains_matches_closed_form():
    """chains of a stationary AR(1) process v_t = phi v_{t-1} + e_t, e_t ~ N(0, 1): the mean of
    S values has variance (1 / (1 - phi^2)) (1 + phi) / (1 - phi) / S for large S, so the batch-
    means MCSE of C chains of S values must approach sqrt(1 / ((1 - phi)^2 C S)); with
    floor(sqrt(S)) = 447 batches of 447 values per chain (far longer than the correlation
    time) and 4 chains, the estimate's own relative error is about 1/sqrt(2 x 1788) = 1.7%"""
    rng = np.random.default_rng(6)
    phi, C, S = 0.8, 4, 200000
    acc = np.zeros((C, 12))
    nb = int(math.isqrt(S))
    lb = S // nb
    for c in range(C):
        e = rng.standard_normal(S)
        v = np.empty(S)
        v[0] = e[0] / math.sqrt(1.0 - phi * phi)
        for t in range(1, S):
            v[t] = phi * v[t - 1] + e[t]
        bs = v[:nb * lb].reshape(nb, lb).sum(1)
        for a in range(3):
            acc[c, 2 * a] = v.sum()
            acc[c, 2 * a + 1] = (v * v).sum()
            acc[c, 6 + 2 * a] = bs.sum()
            acc[c, 7 + 2 * a] = (bs * bs).sum()
    s = oracle.summarize(acc[None].reshape(C, 12), S, 0, C)
    want = math.sqrt(1.0 / ((1.0 - phi) ** 2 * C * S))
    mean, var, mcse = s["N"]
    assert mcse[0] == pytest.approx(want, rel=0.07)
    assert var[0] == pytest.approx(1.0 / (1.0 - phi * phi), rel=0.05)
