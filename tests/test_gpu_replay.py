"""fsmp_replay: the sampler's delta-nu along a given path (needs an MI355X).

The strongest form of the two-way check: the oracle runs its own chains (its own Philox
draws, every log p(w|z) from a fresh Cholesky factorisation) and records every proposal;
the GPU kernels then follow those recorded proposals and accept decisions, and the
delta-nu and log-acceptance they compute with their incremental G^-1 algebra must equal
the oracle's from-scratch values step by step, at every PE capacity, to 1e-9 relative:
|d - d_ref| <= 1e-9 max(1, |d_ref|).  The final PE lists must be identical, since both
followed the same path.

On pile-up waveforms nu(z) reaches ~1e6 while delta-nu is 10-40, so the reference there is
the oracle's extended-precision replay (both nu's from scratch in long double), not the
FP64 difference recorded in its log (itself up to ~3e-9 off on these windows).  The long
replay (4,000 sweeps at K around 100) holds the FP64 form to the bound over its whole
length: there the charge means' residual against the exact G corrects what the explicitly
inverted G^-1 leaves (about 1e-8 of delta-nu without it, with or without rebuilds).
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import ext_reference, gpu_sampler, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _replay_oracle_log(wl, b, km, n_steps, n_chains, seed, extended=False, wide=False):
    """wide: the wide lane groups (one chain per wavefront) from capacity 64 up, else the
    narrow ones"""
    kz = int(km.max())
    print(f"[case] replay {wl.name} n={len(km)} caps={sorted(set(km.tolist()))} steps={n_steps} wide={wide}",
          flush=True)
    p = oracle_params(wl)
    o = oracle.run(p, b["wave"], b["offsets"], b["lam"], n_chains, n_steps, n_steps // 2, seed, kz, kmax=km,
                   log=True)
    smp = gpu_sampler(wl, n_steps, n_steps // 2, n_chains, seed)
    if wide:
        for cap in (64, 96, 128, 160, 192):
            smp.set_design(cap, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
    dnu, la, out = smp.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], o.log, kmax=km, kz=kz)
    torch.cuda.synchronize()
    dnu, la = dnu.cpu().numpy(), la.cpu().numpy()
    valid = (o.log["flags"] & 1) != 0
    if extended:
        ref_d, ref_a = ext_reference(p, b, km, o.log, n_chains, seed)
        e64 = np.abs(o.log["dnu"][valid] - ref_d[valid]) / np.maximum(np.abs(ref_d[valid]), 1.0)
        print(f"[replay] the oracle's own FP64 delta-nu against the extended one: max rel err {e64.max():.2e}",
              flush=True)
    else:
        ref_d, ref_a = o.log["dnu"], o.log["log_alpha"]
    # only the evaluated proposals (the others hold -inf log-alphas on both sides)
    err_d = np.abs(dnu[valid] - ref_d[valid]) / np.maximum(np.abs(ref_d[valid]), 1.0)
    err_a = np.abs(la[valid] - ref_a[valid]) / np.maximum(np.abs(ref_a[valid]), 1.0)
    print(f"[replay] {valid.sum()} proposals: max rel err delta-nu {err_d.max():.2e}, log-alpha {err_a.max():.2e}",
          flush=True)
    assert valid.sum() > 0
    assert np.isfinite(dnu[valid]).all()
    assert err_d.max() < TOL and err_a.max() < TOL
    assert (dnu[~valid] == 0).all() and np.isneginf(la[~valid]).all()
    np.testing.assert_array_equal(out["n_pe"].cpu().numpy(), o.N)
    np.testing.assert_array_equal(out["z"].cpu().numpy(), o.z)
    return o, err_d


def test_replay_oracle_log_batched():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=60, seed=71)
    km = synth.kmax_for(b["lam"])
    _replay_oracle_log(wl, b, km, 300, 2, 21)


@pytest.mark.parametrize("wide", [False, True])
def test_replay_oracle_log_high_capacity(wide):
    wl = synth.PRESETS["pileup"]
    lam = np.array([20.0, 45.0, 60.0, 80.0, 100.0])
    b = synth.generate(wl, n_wave=len(lam), seed=9, lam=lam)
    km = synth.kmax_for(b["lam"])
    assert km.max() >= 128
    _replay_oracle_log(wl, b, km, 250, 1, 4, extended=True, wide=wide)


@pytest.mark.parametrize("wide", [False, True])
def test_replay_long_chains_high_capacity(wide):
    # 4,000 sweeps at K ~ 90-110: the FP64 form edits G^-1 by rank-one / rank-two updates the
    # whole way; its delta-nu must stay within the bound to the last sweep
    wl = synth.PRESETS["pileup"]
    lam = np.array([95.0, 100.0])
    b = synth.generate(wl, n_wave=len(lam), seed=13, lam=lam)
    km = synth.kmax_for(b["lam"])
    assert km.min() >= 128
    o, err = _replay_oracle_log(wl, b, km, 4000, 1, 8, extended=True, wide=wide)
    assert o.N.min() >= 80
    valid = (o.log["flags"] & 1) != 0
    late = np.zeros_like(valid)
    late[:, 3000:] = True
    tail = err[late[valid]]
    print(f"[replay] sweeps 3000-4000: max rel err {tail.max():.2e}", flush=True)


def test_replay_own_log_matches_recorded():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=50, seed=72)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    smp = gpu_sampler(wl, 200, 100, 2, 5, record_flags=fsmp.FSMP_REC_LOG)
    wave = torch.from_numpy(b["wave"]).cuda()
    out = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz)
    dnu, la, out2 = smp.replay(wave, b["offsets"], b["lam"], out["log"], kmax=km, kz=kz)
    torch.cuda.synchronize()
    logs = fsmp.log_records(out["log"])
    valid = (logs["flags"] & 1) != 0
    d = dnu.cpu().numpy()
    e = np.abs(d - logs["dnu"])[valid] / np.maximum(np.abs(logs["dnu"][valid]), 1.0)
    assert e.max() < TOL
    np.testing.assert_array_equal(out2["z"].cpu().numpy(), out["z"].cpu().numpy())


def test_replay_rejects_fp32_and_bad_log():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=4, seed=1)
    km = synth.kmax_for(b["lam"])
    smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                       t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                       n_steps=20, n_chains=1, burn_in=10, seed=1, precision=fsmp.FSMP_FP32_REFRESH)
    log = np.zeros((4, 20), dtype=oracle.LOGREC_DTYPE)
    with pytest.raises(RuntimeError):
        smp.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], log, kmax=km)
    smp64 = gpu_sampler(wl, 20, 10, 1, 1)
    with pytest.raises(ValueError):
        smp64.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], log[:, :10], kmax=km)
