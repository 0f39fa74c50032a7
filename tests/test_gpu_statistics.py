"""Statistical two-way parity (needs an MI355X): the GPU and the oracle run independent
chains (different seeds, so no shared random numbers) on the same 1,000 waveforms of the
batched workload (windows of 1,024 samples, lambda ~ logU[0.1, 30], 1,000 sweeps with half
burn-in), and their posterior means must agree within their Monte Carlo errors: per
waveform and for each of N, Q and t0,

    z = (m_gpu - m_oracle) / sqrt(MCSE_gpu^2 + MCSE_oracle^2),

with |z| <= 3 on all but 1 % of the waveforms and the mean of z within 3 / sqrt(B) of 0
(B the number of waveforms with a non-zero MCSE; swapping the two runs negates z, so its
mean is 0 for a correct sampler).  Waveforms with zero MCSE on both sides must have equal
means.  The MCSE is the spread of 16 chain means per waveform (fsmp_posterior's
mcse_chains): the within-chain batch-means MCSE of chains this short underestimates the
error by a factor of 2-4 (oracle against oracle at 4 x 1,000 sweeps: z standard
deviation 3.6), while the 16-chain spread gives z with standard deviation 1.0.
Run for the FP64 form and for the FP32 storage form with its FP64 refresh, which must
sample the same posterior.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import gpu_sampler, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_WAVE, C, N_STEPS, BURN = 1000, 16, 1000, 500
_ORACLE = {}


def _batch():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=N_WAVE, seed=123)
    return wl, b, synth.kmax_for(b["lam"])


def _oracle_summary():
    if "s" not in _ORACLE:
        wl, b, km = _batch()
        o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, N_STEPS, BURN, 4004, int(km.max()),
                       kmax=km)
        summ = oracle.summarize(o.acc, N_STEPS, BURN, C)
        _, mc = oracle.chain_diagnostics(o.acc, N_STEPS - BURN, C)
        _ORACLE["s"] = (np.stack([summ[k][0] for k in ("N", "Q", "t0")], 1), mc)
    return _ORACLE["s"]


@pytest.mark.parametrize("precision", [fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH])
def test_posterior_means_agree_within_mcse(precision):
    wl, b, km = _batch()
    print(f"[case] statistics n={N_WAVE} chains={C} precision={precision}", flush=True)
    if precision == fsmp.FSMP_FP64:
        smp = gpu_sampler(wl, N_STEPS, BURN, C, 3003)
    else:
        smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                           t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                           sigma_q=wl.sigma_q, grid_sub=4, t0_step_sd=1.0, shift_sd=1.0, n_steps=N_STEPS,
                           n_chains=C, burn_in=BURN, seed=3003, precision=precision, refresh_M=64)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=int(km.max()))
    post = smp.posterior(N_WAVE, out, diagnostics=True)
    torch.cuda.synchronize()
    mg = post["mean"].cpu().numpy()
    sg = post["mcse_chains"].cpu().numpy()
    mo, so = _oracle_summary()
    for a, name in enumerate(("N", "Q", "t0")):
        den = np.sqrt(sg[:, a] ** 2 + so[:, a] ** 2)
        ok = den > 0
        z = (mg[ok, a] - mo[ok, a]) / den[ok]
        exceed = float((np.abs(z) > 3).mean())
        dmax = np.abs(mg[~ok, a] - mo[~ok, a]).max(initial=0.0)
        print(f"[statistics] {name}: {ok.sum()} waveforms, |z| > 3 on {exceed * 100:.2f}%, mean z {z.mean():+.3f} "
              f"(bound {3 / np.sqrt(ok.sum()):.3f}), z sd {z.std():.3f}; {(~ok).sum()} with zero MCSE on both "
              f"sides, largest |difference| {dmax:.2e}", flush=True)
        assert exceed <= 0.01, name
        assert abs(z.mean()) <= 3 / np.sqrt(ok.sum()), name
        assert dmax == 0.0, name
