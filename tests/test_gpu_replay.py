"""fsmp_replay: the sampler's delta-nu along a given path (needs an MI355X).

The strongest form of the two-way check: the oracle runs its own chains (its own Philox
draws, every log p(w|z) from a fresh Cholesky factorisation) and records every proposal;
the GPU kernels then follow those recorded proposals and accept decisions, and the
delta-nu and log-acceptance they compute with their incremental G^-1 algebra must equal
the oracle's from-scratch values to FP64 rounding, step by step, at every PE capacity.
The final PE lists must be identical, since both followed the same path.

Tolerance: 1e-9 relative, |d - d_ref| <= 1e-9 max(1, |d_ref|).  On pile-up waveforms the
oracle's delta-nu is the difference nu(z') - nu(z) of two log-likelihood terms of up to
~1e6 (delta-nu itself is typically 10-40), each through a Cholesky factorisation whose
rounding grows like K eps; there the bound adds that rounding of the reference,
K eps (|nu(z)| + |nu(z')|), with nu taken from the oracle on the replayed states.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import gpu_sampler, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _ref_rounding(p, b, rec, n_chains):
    """K eps (|nu(z)| + |nu(z')|) of every step, K the larger PE count of the two states, from
    the oracle on the states the log passes through"""
    out = np.zeros(rec.shape)
    for c in range(rec.shape[0]):
        i = c // n_chains
        w = b["wave"][b["offsets"][i]:b["offsets"][i + 1]]
        l0, _ = oracle.log_likelihood(p, w, [])
        z = []
        nu = 0.0
        for s in range(rec.shape[1]):
            r = rec[c, s]
            if not (r["flags"] & 1):
                continue
            zp = list(z)
            if r["move"] == oracle.MOVE_BIRTH:
                zp.append(int(r["g"]))
            elif r["move"] == oracle.MOVE_DEATH:
                zp[r["j"]] = zp[-1]
                zp.pop()
            else:
                zp[r["j"]] = int(r["g"])
            nu_p = oracle.log_likelihood(p, w, zp)[0] - l0
            out[c, s] = max(len(z), len(zp)) * np.finfo(float).eps * (abs(nu) + abs(nu_p))
            if r["flags"] & 2:
                z, nu = zp, nu_p
    return out


def _replay_oracle_log(wl, b, km, n_steps, n_chains, seed, ref_rounding=False):
    kz = int(km.max())
    print(f"[case] replay {wl.name} n={len(km)} caps={sorted(set(km.tolist()))} steps={n_steps}", flush=True)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], n_chains, n_steps, n_steps // 2, seed, kz,
                   kmax=km, log=True)
    smp = gpu_sampler(wl, n_steps, n_steps // 2, n_chains, seed)
    dnu, la, out = smp.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], o.log, kmax=km, kz=kz)
    torch.cuda.synchronize()
    dnu, la = dnu.cpu().numpy(), la.cpu().numpy()
    valid = (o.log["flags"] & 1) != 0
    ref_d, ref_a = o.log["dnu"], o.log["log_alpha"]
    err_d = np.abs(dnu - ref_d)[valid] / np.maximum(np.abs(ref_d[valid]), 1.0)
    err_a = np.abs(la - ref_a)[valid] / np.maximum(np.abs(ref_a[valid]), 1.0)
    print(f"[replay] {valid.sum()} proposals: max rel err delta-nu {err_d.max():.2e}, log-alpha {err_a.max():.2e}",
          flush=True)
    assert valid.sum() > 0
    assert np.isfinite(dnu[valid]).all()
    if ref_rounding:
        bound = TOL * np.maximum(np.abs(ref_d), 1.0) + _ref_rounding(oracle_params(wl), b, o.log, n_chains)
        ratio = (np.abs(dnu - ref_d) / bound)[valid]
        print(f"[replay] largest |d - d_ref| / bound = {ratio.max():.3f}", flush=True)
        assert ratio.max() <= 1.0
        assert (np.abs(la - ref_a)[valid] <= (bound + TOL * np.maximum(np.abs(ref_a), 1.0))[valid]).all()
    else:
        assert err_d.max() < TOL and err_a.max() < TOL
    assert (dnu[~valid] == 0).all() and np.isneginf(la[~valid]).all()
    np.testing.assert_array_equal(out["n_pe"].cpu().numpy(), o.N)
    np.testing.assert_array_equal(out["z"].cpu().numpy(), o.z)
    return o


def test_replay_oracle_log_batched():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=60, seed=71)
    km = synth.kmax_for(b["lam"])
    _replay_oracle_log(wl, b, km, 300, 2, 21)


def test_replay_oracle_log_high_capacity():
    wl = synth.PRESETS["pileup"]
    lam = np.array([20.0, 45.0, 60.0, 80.0, 100.0])
    b = synth.generate(wl, n_wave=len(lam), seed=9, lam=lam)
    km = synth.kmax_for(b["lam"])
    assert km.max() >= 128
    _replay_oracle_log(wl, b, km, 250, 1, 4, ref_rounding=True)


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
