"""Launch machinery around the chain kernels (needs an MI355X).

* fsmp_graph_*: a captured batch replays to bit-identical outputs, several times, with
  eager sampling on the same context, output clearing and synchronisations between the
  replays (FP64 with the default designs; the FP32-refresh form with its wide groups at
  capacities 16 and 32);
* fsmp_set_design / fsmp_autotune: the chosen design per PE capacity is one that exists,
  and a batch run with the tuned designs still agrees with the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("n_pe", "t0", "z", "charge", "acc", "nhist", "counts", "status")


def _batch(n, seed, preset="batched"):
    wl = synth.PRESETS[preset]
    b = synth.generate(wl, n_wave=n, seed=seed)
    return wl, b, synth.kmax_for(b["lam"])


@pytest.mark.parametrize("form", ["fp64", "fp32_wide"])
def test_graph_replays_equal_eager(form):
    wl, b, km = _batch(96, 41)
    _, b2, km2 = _batch(40, 42)
    kz = int(km.max())
    print(f"[case] graph replay {form} n=96 kz={kz} caps={sorted(set(km.tolist()))}", flush=True)
    if form == "fp64":
        smp = gpu_sampler(wl, 200, 100, 2, 9)
    else:
        smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                           t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                           sigma_q=wl.sigma_q, n_steps=200, n_chains=2, burn_in=100, seed=9,
                           precision=fsmp.FSMP_FP32_REFRESH, refresh_M=64)
        for cap in (16, 32):
            smp.set_design(cap, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
        assert {16, 32} <= set(km.tolist())
    wave = torch.from_numpy(b["wave"]).cuda()
    ref = to_host(smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz))
    g, out = smp.graph(wave, b["offsets"], b["lam"], kmax=km, kz=kz)
    wave2 = torch.from_numpy(b2["wave"]).cuda()
    for r in range(3):
        for k in KEYS:
            out[k].zero_()
        # eager work on the same context between replays: another batch, other sizes
        smp.sample(wave2, b2["offsets"], b2["lam"], kmax=km2, kz=int(km2.max()))
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        got = to_host(out)
        for k in KEYS:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"replay {r}: {k}")
    g.close()


def test_graph_rejects_bad_batch():
    wl, b, km = _batch(4, 3)
    smp = gpu_sampler(wl, 10, 5, 1, 1)
    km_bad = km.copy()
    km_bad[0] = 1000
    with pytest.raises(RuntimeError):
        smp.graph(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km_bad, kz=1000)


def test_set_design_validation():
    wl, _, _ = _batch(2, 1)
    smp = gpu_sampler(wl, 10, 5, 1, 1)
    smp.set_design(16, fsmp.FSMP_DESIGN_GROUP)
    assert smp.get_design(16) == fsmp.FSMP_DESIGN_GROUP
    smp.set_design(16, fsmp.FSMP_DESIGN_LANE)
    assert smp.get_design(16) == fsmp.FSMP_DESIGN_LANE
    smp.set_design(32, fsmp.FSMP_DESIGN_LANE)
    for cap in (48, 64, 96, 128, 160, 192):   # one lane per chain exists at capacities 16 and 32 only
        with pytest.raises(RuntimeError):
            smp.set_design(cap, fsmp.FSMP_DESIGN_LANE)
    with pytest.raises(RuntimeError):
        smp.set_design(96, fsmp.FSMP_DESIGN_GROUP)
    with pytest.raises(RuntimeError):
        smp.set_design(20, fsmp.FSMP_DESIGN_LANE)
    before = [smp.get_design(c) for c in synth.KCAPS]
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP)  # every capacity that has the design; the rest keep theirs
    assert [smp.get_design(c) for c in synth.KCAPS] == [0, 0, 0, 0] + before[4:]
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP_DEVMEM)
    assert [smp.get_design(c) for c in synth.KCAPS] == [2] * 8
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)  # the wide groups exist from capacity 32 up
    assert [smp.get_design(c) for c in synth.KCAPS] == [2] + [3] * 7
    with pytest.raises(RuntimeError):
        smp.set_design(16, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
    with pytest.raises(RuntimeError):
        smp.set_design(16, 4)


def test_set_design_validation_fp32():
    # the FP32-refresh form: device-memory groups only; its wide groups at capacities 16 and 32
    wl, _, _ = _batch(2, 1)
    smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                       t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                       sigma_q=wl.sigma_q, n_steps=10, n_chains=1, burn_in=5, seed=1,
                       precision=fsmp.FSMP_FP32_REFRESH)
    for cap in synth.KCAPS:
        for d in (fsmp.FSMP_DESIGN_GROUP, fsmp.FSMP_DESIGN_LANE):
            with pytest.raises(RuntimeError):
                smp.set_design(cap, d)
    for cap in (16, 32):
        smp.set_design(cap, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
        assert smp.get_design(cap) == fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE
    for cap in (48, 64, 96, 128, 160, 192):
        with pytest.raises(RuntimeError):
            smp.set_design(cap, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP_DEVMEM)
    smp.set_design(0, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)  # every capacity that has it; the rest keep theirs
    assert [smp.get_design(c) for c in synth.KCAPS] == [3, 3] + [2] * 6


def test_autotune_keeps_results_correct():
    wl, b, km = _batch(400, 51)
    kz = int(km.max())
    smp = gpu_sampler(wl, 120, 60, 1, 13)
    wave = torch.from_numpy(b["wave"]).cuda()
    before = {c: smp.get_design(c) for c in synth.KCAPS}
    designs = smp.autotune(wave, b["offsets"], b["lam"], kmax=km, trial_steps=40)
    print(f"[autotune] {before} -> {designs}", flush=True)
    assert all(designs[c] in (fsmp.FSMP_DESIGN_GROUP, fsmp.FSMP_DESIGN_GROUP_DEVMEM, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE)
               for c in (48, 64))  # no lane

    assert all(designs[c] == before[c] for c in (96, 128, 160, 192))                # not in the batch: untouched
    # a sub-batch in the tuned designs against the oracle
    n = 60
    off = b["offsets"][:n + 1]
    out = smp.sample(torch.from_numpy(b["wave"][:off[-1]].copy()).cuda(), off, b["lam"][:n], kmax=km[:n],
                     kz=int(km[:n].max()))
    torch.cuda.synchronize()
    g = to_host(out)
    o = oracle.run(oracle_params(wl), b["wave"][:off[-1]], off, b["lam"][:n], 1, 120, 60, 13, int(km[:n].max()),
                   kmax=km[:n])
    parted = compare_chains(g, o)

    def tuned(flags):
        s = gpu_sampler(wl, 120, 60, 1, 13, record_flags=flags)
        for cap, d in designs.items():
            s.set_design(cap, d)
        return s
    check_partings(parted, oracle_params(wl), {"wave": b["wave"][:off[-1]], "offsets": off}, b["lam"][:n], km[:n], 1,
                   120, 60, 13, int(km[:n].max()), tuned)


def test_workspace_bytes_matches_device_allocation():
    wl, b, km = _batch(20000, 61)
    kz = int(km.max())
    smp = gpu_sampler(wl, 50, 25, 2, 3)
    wave = torch.from_numpy(b["wave"]).cuda()
    out = smp.alloc_samples(20000, kz)
    predicted = smp.workspace_bytes(b["offsets"], b["lam"], kmax=km)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=out)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    print(f"[workspace] predicted {predicted / 2**20:.1f} MiB, device memory taken {used / 2**20:.1f} MiB", flush=True)
    assert 0.9 * predicted <= used <= 1.1 * predicted + (64 << 20)
