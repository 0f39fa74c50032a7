"""Posterior extras of fsmp_posterior against the oracle (needs an MI355X): the Gelman-Rubin
R and the between-chain MCSE of N, Q and t0 (Sec. 3.2 convergence check), lambda-hat_FSMP
(eq. reduce-mu0) and lambda-hat_Q = E[Q] / mu_q.

On every waveform whose chains all match the oracle's, the kernel's values must equal the
oracle's computed from its own accumulators and N histograms: lambda-hat to 1e-9 relative
(a root of m(lambda) = lambda, found to rounding on both sides); R and the MCSE to 1e-7
relative, since the chain variances come from sums of v and v^2 whose difference cancels
by up to mean^2 / variance (about 1e4 for t0 here) the 1e-12 relative agreement of the
accumulators.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import check_partings, compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_diagnostics_and_lambda_hat_match_oracle():
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn = 80, 4, 400, 200
    b = synth.generate(wl, n_wave=n, seed=131)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] estimates batched n={n} chains={C}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 17)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz)
    post = smp.posterior(n, out, diagnostics=True, lam=b["lam"])
    torch.cuda.synchronize()
    g = to_host(out)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, burn, 17, kz, kmax=km)
    parted = compare_chains(g, o)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, C, n_steps, burn, 17, kz,
                   lambda flags: gpu_sampler(wl, n_steps, burn, C, 17, record_flags=flags))
    bad = set(int(c) // C for c in parted)
    keep = np.array([i for i in range(n) if i not in bad])
    rh, mc = oracle.chain_diagnostics(o.acc, n_steps - burn, C)
    grh = post["rhat"].cpu().numpy()
    gmc = post["mcse_chains"].cpu().numpy()
    np.testing.assert_allclose(grh[keep], rh[keep], rtol=1e-7, atol=0)
    np.testing.assert_allclose(gmc[keep], mc[keep], rtol=1e-7, atol=1e-12)
    lh = post["lambda_hat"].cpu().numpy()
    hist = o.nhist.reshape(n, C, -1).sum(1)
    want = np.array([oracle.lambda_mle(hist[i], b["lam"][i]) for i in range(n)])
    np.testing.assert_allclose(lh[keep, 0], want[keep], rtol=1e-9, atol=1e-12)
    mean_q = post["mean"][:, 1].cpu().numpy()
    np.testing.assert_array_equal(lh[:, 1], mean_q / wl.mu_q)
    print(f"[estimates] {len(keep)} waveforms compared; R max {np.nanmax(grh):.3f}; "
          f"lambda-hat / lambda0 median {np.median(lh[:, 0] / b['lam']):.3f}", flush=True)


def test_diagnostics_single_chain_and_lambda_zero():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=8, seed=132)
    km = synth.kmax_for(b["lam"])
    lam = b["lam"].copy()
    lam[:4] = 0.0   # no births: N stays 0, lambda-hat 0
    smp = gpu_sampler(wl, 100, 50, 1, 2)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], lam, kmax=km, kz=int(km.max()))
    post = smp.posterior(8, out, diagnostics=True, lam=lam)
    torch.cuda.synchronize()
    assert np.isnan(post["rhat"].cpu().numpy()).all() and np.isnan(post["mcse_chains"].cpu().numpy()).all()
    lh = post["lambda_hat"].cpu().numpy()
    assert (lh[:4, 0] == 0.0).all()
    with pytest.raises(RuntimeError):
        smp.posterior(8, out, lam=np.full(8, -1.0))
