"""Per-waveform chain lengths and the chain-length autotuner (needs an MI355X).

* fsmp_batch.n_steps: every waveform runs its own number of sweeps (burn-in in the
  configured proportion); each chain must equal the oracle run with that waveform's sweep
  count and identity, the recorded-sweep counts must be right, and fsmp_posterior must
  divide by each chain's own count;
* fsmp_autotune_steps: counts within the bounds, more sweeps where the pilot's MCSE is
  larger, and a run with the tuned counts meets the MCSE target on most waveforms.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tuned", [False, True])
def test_per_waveform_steps_match_oracle(tuned):
    # tuned: the kernel designs from fsmp_autotune with the same sweep counts (its trial keeps
    # their proportions), which may pick any design per capacity, the wide groups included
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn = 60, 2, 600, 300
    b = synth.generate(wl, n_wave=n, seed=91)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    steps = np.random.default_rng(3).choice([200, 351, 600, 457], size=n).astype(np.int32)
    print(f"[case] per-waveform steps n={n} chains={C} steps={sorted(set(steps.tolist()))} tuned={tuned}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 12)
    if tuned:
        designs = smp.autotune(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, trial_steps=20,
                               n_steps=steps)
        print(f"[autotune] {designs}", flush=True)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz, n_steps=steps)
    post = smp.posterior(n, out)
    torch.cuda.synchronize()
    g = to_host(out)
    burn_w = steps.astype(np.int64) * burn // n_steps
    np.testing.assert_array_equal(g["rec_steps"], np.repeat(steps - burn_w, C))
    lengths = np.diff(b["offsets"])
    for s in sorted(set(steps.tolist())):
        idx = np.where(steps == s)[0]
        off = np.concatenate([[0], np.cumsum(lengths[idx])])
        wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in idx])
        bw = s * burn // n_steps
        o = oracle.run(oracle_params(wl), wave, off, b["lam"][idx], C, s, bw, 12, kz, kmax=km[idx],
                       wave_id=idx.astype(np.uint64))
        rows = (idx[:, None] * C + np.arange(C)[None, :]).reshape(-1)
        sub = {k: (v[rows] if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == n * C else v)
               for k, v in g.items()}
        parted = compare_chains(sub, o)
        assert len(parted) == 0, (s, parted)
        summ = oracle.summarize(o.acc, s, bw, C)
        for a_, name in enumerate(("N", "Q", "t0")):
            np.testing.assert_allclose(post["mean"][idx, a_].cpu().numpy(), summ[name][0], rtol=1e-9, atol=1e-9)
            np.testing.assert_allclose(post["mcse"][idx, a_].cpu().numpy(), summ[name][2], rtol=1e-7, atol=1e-9)


def test_per_waveform_steps_rejected_out_of_range():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=4, seed=1)
    km = synth.kmax_for(b["lam"])
    smp = gpu_sampler(wl, 100, 50, 1, 1)
    with pytest.raises(RuntimeError):
        smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km,
                   n_steps=np.array([10, 101, 50, 50], np.int32))


def test_autotune_steps():
    wl = synth.PRESETS["batched"]
    n, n_steps, burn = 400, 4000, 2000
    b = synth.generate(wl, n_wave=n, seed=92)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    smp = gpu_sampler(wl, n_steps, burn, 1, 21)
    wave = torch.from_numpy(b["wave"]).cuda()
    target = 0.02
    steps = smp.autotune_steps(wave, b["offsets"], b["lam"], kmax=km, pilot_steps=400, target_rel_mcse=target,
                               min_steps=500, max_steps=4000)
    print(f"[steps] tuned sweeps: min {steps.min()} median {int(np.median(steps))} max {steps.max()}", flush=True)
    assert steps.min() >= 500 and steps.max() <= 4000
    assert len(set(steps.tolist())) > 3   # the counts adapt to the waveforms
    out = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, n_steps=steps)
    post = smp.posterior(n, out)
    torch.cuda.synchronize()
    mean = post["mean"][:, 0].cpu().numpy()
    mcse = post["mcse"][:, 0].cpu().numpy()
    free = (steps > 500) & (steps < 4000)  # not clamped
    ok = mcse[free] <= 2.0 * target * np.maximum(1.0, mean[free])
    print(f"[steps] {free.sum()} unclamped waveforms, {ok.mean() * 100:.1f}% within 2x the MCSE target", flush=True)
    assert free.sum() > 20 and ok.mean() >= 0.8
