"""The plain and the batched workloads at their full sizes, in one call each, against the
oracle (needs an MI355X).

* plain: 1,000 windows of 256 samples, lambda ~ U[0.5, 5], one chain of 2,000 steps each,
  seed 0, FP64: every chain is recomputed by the oracle and compared element by element;
* batched: 100,000 windows of 1,024 samples, lambda ~ logU[0.1, 30], four chains of 1,000
  sweeps each, FP64: the call runs at full size with the library's default designs, the
  chains of waveforms sampled from every PE capacity are recomputed by the oracle with the
  same identities and must match the GPU's, and every chain is checked for validity.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_plain_full_size_every_chain():
    wl = synth.PRESETS["plain"]
    n_steps, burn, seed = 2000, 1000, 0
    b = synth.generate(wl, seed=wl.seed)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    n = len(km)
    print(f"[case] plain full n={n} steps={n_steps} caps={sorted(set(km.tolist()))}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, 1, seed)
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz))
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], 1, n_steps, burn, seed, kz, kmax=km)
    parted = compare_chains(g, o)
    print(f"[configs] plain full size: {len(parted)} of {n} chains parted", flush=True)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, 1, n_steps, burn, seed, kz,
                   lambda flags: gpu_sampler(wl, n_steps, burn, 1, seed, record_flags=flags))
    assert (g["counts"][:, 3] > 0).mean() > 0.5


def test_batched_full_size_sampled_chains():
    wl = synth.PRESETS["batched"]
    n_steps, burn, C, seed = 1000, 500, 4, 2
    b = synth.generate(wl, seed=wl.seed)
    n = len(b["offsets"]) - 1
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] batched full n={n} chains={C} steps={n_steps} caps={sorted(set(km.tolist()))}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, seed)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz)
    torch.cuda.synchronize()
    g = to_host(out)
    kc = np.repeat(km, C)
    assert (g["n_pe"] >= 0).all() and (g["n_pe"] <= kc).all()
    assert np.isfinite(g["t0"]).all() and ((g["t0"] >= wl.t0_min) & (g["t0"] <= wl.t0_max)).all()
    assert (g["nhist"].sum(1) == n_steps - burn).all()
    bad = fsmp.FSMP_ST_NONFINITE | fsmp.FSMP_ST_DRIFT | fsmp.FSMP_ST_EMPTY_T | fsmp.FSMP_ST_FACTOR
    assert (g["status"] & bad == 0).all()
    # sampled waveforms, every capacity, all their chains: the oracle with the same identities
    rng = np.random.default_rng(11)
    pick = []
    for cap in sorted(set(km.tolist())):
        idx = np.where(km == cap)[0]
        pick.extend(rng.choice(idx, size=min(10, len(idx)), replace=False).tolist())
    pick = np.array(sorted(pick))
    lengths = np.diff(b["offsets"])
    off = np.concatenate([[0], np.cumsum(lengths[pick])])
    wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in pick])
    o = oracle.run(oracle_params(wl), wave, off, b["lam"][pick], C, n_steps, burn, seed, kz, kmax=km[pick],
                   wave_id=pick.astype(np.uint64))
    rows = (pick[:, None] * C + np.arange(C)[None, :]).ravel()
    sub = {k: (v[rows] if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    parted = compare_chains(sub, o)
    print(f"[configs] batched full size: {len(rows)} sampled chains, {len(parted)} parted", flush=True)
    check_partings(parted, oracle_params(wl), {"wave": wave, "offsets": off}, b["lam"][pick], km[pick], C, n_steps,
                   burn, seed, kz, lambda flags: gpu_sampler(wl, n_steps, burn, C, seed, record_flags=flags),
                   wave_id=pick)
