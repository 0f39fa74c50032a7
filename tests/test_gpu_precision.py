"""Precision form on the GPU (needs an MI355X): G^{-1} stored in FP32; every proposal
evaluated from it with a two-term residual correction against the exact FP64 Gram matrix
(whose entries come from the overlap tables), with an error bound from the size of the
last correction; the proposal is re-evaluated from an FP64 rebuild of G^{-1} when that bound
exceeds 1e-5 of max(1, |delta-nu|) or could turn the accept decision; an FP64 refresh every
refresh_M sweeps.

* every proposal an FP32-form chain made on the high pile-up workload (lambda ~ U[20, 100],
  charges N(1, 0.35), K up to 160) is replayed by the FP64 oracle: the relative error of
  delta-nu, |dnu - dnu_ref| / max(|dnu_ref|, 1), is at most 1e-4 at sigma_eps = 0.05, 0.1
  and 0.2 (refresh every 64 sweeps; at sigma_eps = 0.05 also 16 and 256), and no accept
  decision differs from the one the oracle takes;
* the same bound and no differing decision on the batched workload (capacities 16-64) with
  the FP32 form's wide groups (16 lanes per chain) at capacities 16 and 32;
* the FP32 form's chains on the batched workload are the oracle's chains, in its narrow and
  its wide groups: same PE lists, histograms, counts, and accumulators and charges to 1e-7
  (partings only at near-ties).
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


def _sampler(wl, n_steps, burn, n_chains, seed, precision, refresh_M=64, flags=0, wide=False):
    smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                       t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                       sigma_q=wl.sigma_q, n_steps=n_steps, n_chains=n_chains, burn_in=burn, seed=seed,
                       precision=precision, refresh_M=refresh_M, record_flags=flags)
    if wide:
        for cap in (16, 32):
            smp.set_design(cap, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
    return smp


def _pileup(sigma_eps, n=12):
    base = synth.PRESETS["pileup"]
    return synth.Workload("pileup", n, base.lengths, "uniform", 20.0, 100.0, phi_kind=base.phi_kind,
                          tau_rise=base.tau_rise, tau_decay=base.tau_decay, sigma_q=0.35, sigma_eps=sigma_eps)


def _replay_fp32(wl, b, km, n_steps, refresh_M, wide=False):
    smp = _sampler(wl, n_steps, n_steps // 2, 1, 5, fsmp.FSMP_FP32_REFRESH, refresh_M=refresh_M,
                   flags=fsmp.FSMP_REC_LOG, wide=wide)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=int(km.max()),
                     work=True)
    torch.cuda.synchronize()
    logs = fsmp.log_records(out["log"])
    work = out["work"].cpu().numpy()
    p = oracle_params(wl)
    off = b["offsets"]
    errs = []
    flips = 0
    for c in range(len(km)):
        w = b["wave"][off[c]:off[c + 1]]
        dnu, la, bad = oracle.replay(p, w, b["lam"][c], int(km[c]), 0, 4 * len(w) - 1, c, 5, logs[c], tie_eps=1e-9)
        v = (logs[c]["flags"] & 1) != 0
        errs.append(np.abs(logs[c]["dnu"][v] - dnu[v]) / np.maximum(np.abs(dnu[v]), 1.0))
        flips += bad
    e = np.concatenate(errs)
    n_prop = int(sum(((lg["flags"] & 1) != 0).sum() for lg in logs))
    refit = work[:, 4].sum()
    print(f"[precision] sigma_eps={wl.sigma_eps} M={refresh_M} wide={wide}: {e.size} proposals, delta-nu rel err "
          f"max {e.max():.2e}, p99 {np.quantile(e, 0.99):.2e}, median {np.median(e):.2e}; decision flips {flips}; "
          f"FP64 re-evaluations {refit:.0f} ({refit / max(n_prop, 1):.2%})", flush=True)
    assert np.isfinite(e).all()
    assert e.max() <= TOL
    assert flips == 0


@pytest.mark.parametrize("sigma_eps,refresh_M", [(0.05, 64), (0.1, 64), (0.2, 64), (0.05, 16), (0.05, 256)])
def test_fp32_refresh_delta_nu_replay(sigma_eps, refresh_M):
    wl = _pileup(sigma_eps)
    b = synth.generate(wl, n_wave=12, seed=17)
    km = synth.kmax_for(b["lam"])
    print(f"[case] fp32 pileup sigma_eps={sigma_eps} M={refresh_M} kmax={sorted(set(km.tolist()))}", flush=True)
    _replay_fp32(wl, b, km, 300, refresh_M)


def test_fp32_refresh_delta_nu_replay_wide_groups():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=40, seed=29)
    km = synth.kmax_for(b["lam"])
    assert {16, 32} <= set(km.tolist())
    print(f"[case] fp32 batched wide groups kmax={sorted(set(km.tolist()))}", flush=True)
    _replay_fp32(wl, b, km, 300, 64, wide=True)


@pytest.mark.parametrize("wide", [False, True])
def test_fp32_refresh_chains_are_the_oracles(wide):
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn, seed = 120, 2, 400, 200, 31
    b = synth.generate(wl, n_wave=n, seed=23)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] fp32 batched n={n} caps={sorted(set(km.tolist()))} wide={wide}", flush=True)
    smp = _sampler(wl, n_steps, burn, C, seed, fsmp.FSMP_FP32_REFRESH, wide=wide)
    if wide:
        assert smp.get_design(16) == smp.get_design(32) == fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz))
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, burn, seed, kz, kmax=km)
    parted = compare_chains(g, o, tol=1e-7)
    print(f"[precision] {len(parted)} of {n * C} FP32-form chains parted from the oracle", flush=True)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, C, n_steps, burn, seed, kz,
                   lambda flags: _sampler(wl, n_steps, burn, C, seed, fsmp.FSMP_FP32_REFRESH, flags=flags, wide=wide))
