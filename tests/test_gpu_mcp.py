"""The MCP-PMT Gaussian-mixture charge law (Sec. 2.1 eq. mcp-multi-norm, Sec. 2.4 eq. mcp,
App. A for MCP-PMTs) against the oracle (needs an MI355X).

The components are the paper's five-Gaussian table for MCP-PMTs (weights 4.1 / 51.6 /
18.7 / 19.5 / 6.1 %, means 0.92-6.79, sigmas 0.22-2.04, in units of the SER amplitude
here).  Both sides draw a born or updated PE's component from Philox word 7 by the
inverse CDF of the weights; the kernels update G^-1 with the per-PE ridge incrementally,
the oracle factors from scratch.  Checked: chains element by element (PE lists,
components, histograms, counts, accumulators, charges) at capacities 16-64 and at
160-192; a one-component mixture equal to the single normal law gives the dynode
kernels' chains exactly; the host rejects the forms the mixture does not run in.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = ([0.041, 0.516, 0.187, 0.195, 0.061], [0.92, 1.98, 3.01, 4.70, 6.79], [0.22, 0.48, 0.80, 1.30, 2.04])


def _sampler(wl, n_steps, burn, C, seed, mix=MIX, **kw):
    return fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                        t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                        grid_sub=4, t0_step_sd=1.0, shift_sd=1.0, k_max=64, n_steps=n_steps, n_chains=C, burn_in=burn,
                        seed=seed, mix=mix, **kw)


def _oracle_params(wl, mix=MIX):
    p = oracle_params(wl)
    p.n_mix = len(mix[0])
    for i in range(p.n_mix):
        p.mix_w[i], p.mix_mu[i], p.mix_sigma[i] = mix[0][i], mix[1][i], mix[2][i]
    return p


def _run(wl, b, km, n_steps, burn, C, seed):
    kz = int(km.max())
    smp = _sampler(wl, n_steps, burn, C, seed)
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz))
    o = oracle.run(_oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, burn, seed, kz, kmax=km)
    parted = compare_chains(g, o)
    check_partings(parted, _oracle_params(wl), b, b["lam"], km, C, n_steps, burn, seed, kz,
                   lambda flags: _sampler(wl, n_steps, burn, C, seed, record_flags=flags))
    keep = np.setdiff1d(np.arange(len(g["n_pe"])), parted)
    np.testing.assert_array_equal(g["comp"][keep], o.e[keep])
    return g, o, parted


def test_mcp_chains_match_oracle():
    wl = synth.PRESETS["batched"]
    n, C = 60, 2
    b = synth.generate(wl, n_wave=n, seed=161)
    km = synth.kmax_for(b["lam"])
    print(f"[case] mcp batched n={n} caps={sorted(set(km.tolist()))}", flush=True)
    g, o, parted = _run(wl, b, km, 300, 150, C, 41)
    used = np.bincount(g["comp"][g["comp"] >= 0], minlength=5)
    print(f"[mcp] {len(parted)} of {n * C} chains parted; final PEs per component {used.tolist()}", flush=True)
    assert (used > 0).sum() >= 4


def test_mcp_high_capacity():
    wl = synth.PRESETS["pileup"]
    lam = np.array([50.0, 80.0, 100.0])
    b = synth.generate(wl, n_wave=len(lam), seed=162, lam=lam)
    km = synth.kmax_for(b["lam"])
    assert km.max() >= 160
    print(f"[case] mcp pileup caps={km.tolist()}", flush=True)
    g, o, parted = _run(wl, b, km, 150, 75, 1, 42)
    print(f"[mcp] high capacity: {len(parted)} of {len(km)} chains parted", flush=True)


def test_one_component_equals_single_normal():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=40, seed=163)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    wave = torch.from_numpy(b["wave"]).cuda()
    one = ([1.0], [wl.mu_q], [wl.sigma_q])
    a = to_host(_sampler(wl, 200, 100, 2, 7, mix=one).sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz))
    s = _sampler(wl, 200, 100, 2, 7, mix=None)
    s.set_design(0, fsmp.FSMP_DESIGN_GROUP_DEVMEM)
    d = to_host(s.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz))
    for k in ("n_pe", "t0", "z", "charge", "acc", "nhist", "counts", "status"):
        np.testing.assert_array_equal(a[k], d[k], err_msg=k)
    assert (a["comp"][a["z"] >= 0] == 0).all()


def test_mcp_rejections():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=4, seed=1)
    km = synth.kmax_for(b["lam"])
    wave = torch.from_numpy(b["wave"]).cuda()
    with pytest.raises(RuntimeError):
        _sampler(wl, 20, 10, 1, 1, precision=fsmp.FSMP_FP32_REFRESH)
    with pytest.raises(RuntimeError):
        _sampler(wl, 20, 10, 1, 1, mix=([0.5, 0.4], [1.0, 2.0], [0.3, 0.5]))
    smp = _sampler(wl, 20, 10, 1, 1)
    with pytest.raises(RuntimeError):
        smp.sample(wave, b["offsets"], b["lam"], kmax=km, z_init=[[400], [], [], []])
    log = np.zeros((4, 20), dtype=oracle.LOGREC_DTYPE)
    with pytest.raises(RuntimeError):
        smp.replay(wave, b["offsets"], b["lam"], log, kmax=km)
    # a request for another design falls back to the one the mixture runs in
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP)
    out = smp.sample(wave, b["offsets"], b["lam"], kmax=km)
    torch.cuda.synchronize()
    assert (out["comp"].cpu().numpy()[out["z"].cpu().numpy() < 0] == -1).all()
