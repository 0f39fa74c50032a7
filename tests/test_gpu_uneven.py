"""The uneven batch (windows of 128-2,048 samples, lambda ~ logU[0.05, 100], PE capacities
16-160 in one call) against the oracle (needs an MI355X).

* a small sample of the workload: every chain compared element by element;
* the full 250,000-waveform batch in one call, as a user would run it: chains sampled
  across window lengths and capacities are recomputed by the oracle one by one, with the
  same identities, and must match the GPU's (the rest are checked for validity).
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import check_partings, compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_uneven_sample_every_chain():
    wl = synth.PRESETS["uneven"]
    b = synth.generate(wl, n_wave=90, seed=81)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    lengths = np.diff(b["offsets"])
    print(f"[case] uneven sample n=90 caps={sorted(set(km.tolist()))} lengths={sorted(set(lengths.tolist()))}",
          flush=True)
    smp = gpu_sampler(wl, 300, 150, 1, 7)
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz))
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], 1, 300, 150, 7, kz, kmax=km)
    parted = compare_chains(g, o)
    print(f"[uneven] {len(parted)} of 90 chains parted", flush=True)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, 1, 300, 150, 7, kz,
                   lambda flags: gpu_sampler(wl, 300, 150, 1, 7, record_flags=flags))


def test_uneven_full_size_sampled_chains():
    wl = synth.PRESETS["uneven"]
    n_steps = wl.n_steps
    b = synth.generate(wl, seed=wl.seed)
    n = len(b["offsets"]) - 1
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] uneven full n={n} steps={n_steps} caps={sorted(set(km.tolist()))}", flush=True)
    smp = gpu_sampler(wl, n_steps, n_steps // 2, 1, 3)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz)
    torch.cuda.synchronize()
    g = to_host(out)
    # validity of every chain
    assert (g["n_pe"] >= 0).all() and (g["n_pe"] <= km).all()
    assert np.isfinite(g["t0"]).all() and ((g["t0"] >= wl.t0_min) & (g["t0"] <= wl.t0_max)).all()
    assert (g["nhist"].sum(1) == n_steps - n_steps // 2).all()
    # sampled chains: every window length, capacities up to 64 (the oracle's from-scratch
    # likelihood is O(K^3) per proposal), recomputed by the oracle with the same identities
    rng = np.random.default_rng(5)
    lengths = np.diff(b["offsets"])
    pick = []
    for L in wl.lengths:
        for cap in (16, 32, 64):
            idx = np.where((lengths == L) & (km == cap))[0]
            if len(idx):
                pick.extend(rng.choice(idx, size=min(3, len(idx)), replace=False).tolist())
    pick = np.array(sorted(pick))
    off = np.concatenate([[0], np.cumsum(lengths[pick])])
    wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in pick])
    o = oracle.run(oracle_params(wl), wave, off, b["lam"][pick], 1, n_steps, n_steps // 2, 3, kz, kmax=km[pick],
                   wave_id=pick.astype(np.uint64))
    sub = {k: (v[pick] if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    parted = compare_chains(sub, o)
    print(f"[uneven] full size: {len(pick)} sampled chains, {len(parted)} parted", flush=True)
    check_partings(parted, oracle_params(wl), {"wave": wave, "offsets": off}, b["lam"][pick], km[pick], 1, n_steps,
                   n_steps // 2, 3, kz, lambda flags: gpu_sampler(wl, n_steps, n_steps // 2, 1, 3, record_flags=flags),
                   wave_id=pick)
