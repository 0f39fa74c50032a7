"""Grid occupancy (fsmp_samples.occ, fsmp_posterior_out.occupancy) against the oracle
(needs an MI355X).

The kernels accumulate the occupancy by PE residence (an atomic add of the remaining
recorded sweeps when a PE arrives, a subtraction when it leaves); the oracle counts the PEs
of every recorded state one by one.  Counts are integers: bit-exact on every waveform whose
chains all match the oracle's, in every kernel design; along a replayed oracle path (every
chain follows the oracle's proposals and decisions) on every waveform, at PE capacities up
to 192; at the full batched size (100,000 windows of 1,024 samples, 4 chains x 1,000
sweeps) on sampled waveforms, with the row-sum identity (a row sums to the sum of N over
the recorded steps) and the bounds on all of them.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SUB = 4


def _rows(occ, offsets, i):
    return occ[SUB * offsets[i]:SUB * offsets[i + 1]]


def _check_rows(g, o, offsets, n_chains, parted):
    n = len(offsets) - 1
    bad_w = set(int(c) // n_chains for c in parted)
    same = [i for i in range(n) if i not in bad_w]
    for i in same:
        np.testing.assert_array_equal(_rows(g["occ"], offsets, i), _rows(o.occ, offsets, i), err_msg=f"waveform {i}")
    return same


def _row_sums_match_nhist(occ, nhist, offsets, n_chains):
    ks = np.arange(nhist.shape[1])
    per_chain = (nhist.astype(np.int64) * ks).sum(1).reshape(-1, n_chains).sum(1)
    rows = np.add.reduceat(occ.astype(np.int64), SUB * offsets[:-1]) if len(occ) else np.zeros(0)
    np.testing.assert_array_equal(rows, per_chain)


@pytest.mark.parametrize("design", [None, fsmp.FSMP_DESIGN_GROUP, fsmp.FSMP_DESIGN_LANE,
                                    fsmp.FSMP_DESIGN_GROUP_DEVMEM])
def test_occupancy_matches_oracle(design):
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn = 60, 2, 300, 150
    b = synth.generate(wl, n_wave=n, seed=95)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] occupancy batched n={n} design={design} caps={sorted(set(km.tolist()))}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 31)
    if design is not None:
        smp.set_design(0, design)  # capacities without an instance of the design keep theirs
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz, occupancy=True)
    post = smp.posterior(n, out, offsets=b["offsets"])
    torch.cuda.synchronize()
    g = to_host(out)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, burn, 31, kz, kmax=km,
                   occupancy=True)
    parted = compare_chains(g, o)
    same = _check_rows(g, o, b["offsets"], C, parted)
    print(f"[occupancy] {len(same)} of {n} waveforms with identical chains, rows equal", flush=True)
    assert len(same) >= 0.8 * n
    assert (g["occ"] >= 0).all()
    _row_sums_match_nhist(g["occ"], g["nhist"], b["offsets"], C)
    occ_p = post["occupancy"].cpu().numpy()
    np.testing.assert_allclose(occ_p, g["occ"] / float(C * (n_steps - burn)), rtol=1e-15, atol=0)


def test_occupancy_per_waveform_steps():
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn = 40, 2, 400, 200
    b = synth.generate(wl, n_wave=n, seed=96)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    steps = np.random.default_rng(4).choice([120, 400, 255], size=n).astype(np.int32)
    print(f"[case] occupancy per-waveform steps n={n}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 8)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz, n_steps=steps,
                     occupancy=True)
    post = smp.posterior(n, out, offsets=b["offsets"])
    torch.cuda.synchronize()
    g = to_host(out)
    occ_p = post["occupancy"].cpu().numpy()
    rec = steps - steps.astype(np.int64) * burn // n_steps
    for s in sorted(set(steps.tolist())):
        idx = np.where(steps == s)[0]
        lengths = np.diff(b["offsets"])[idx]
        off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in idx])
        o = oracle.run(oracle_params(wl), wave, off, b["lam"][idx], C, s, s * burn // n_steps, 8, kz, kmax=km[idx],
                       wave_id=idx.astype(np.uint64), occupancy=True)
        rows = (idx[:, None] * C + np.arange(C)[None, :]).reshape(-1)
        sub = {k: (v[rows] if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == n * C else v)
               for k, v in g.items()}
        parted = compare_chains(sub, o)
        bad = set(int(c) // C for c in parted)
        for j, i in enumerate(idx):
            np.testing.assert_allclose(_rows(occ_p, b["offsets"], i), _rows(g["occ"], b["offsets"], i) / (C * rec[i]),
                                       rtol=1e-15)
            if j not in bad:
                np.testing.assert_array_equal(_rows(g["occ"], b["offsets"], i), _rows(o.occ, off, j))


@pytest.mark.parametrize("preset", ["batched", "pileup"])
def test_occupancy_along_replayed_oracle_path(preset):
    wl = synth.PRESETS[preset]
    if preset == "pileup":
        lam = np.array([20.0, 45.0, 80.0, 100.0])
        b = synth.generate(wl, n_wave=len(lam), seed=12, lam=lam)
        n_steps, C = 200, 1
    else:
        b = synth.generate(wl, n_wave=40, seed=97)
        n_steps, C = 300, 2
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] occupancy replay {preset} caps={sorted(set(km.tolist()))}", flush=True)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, n_steps // 2, 5, kz, kmax=km,
                   log=True, occupancy=True)
    smp = gpu_sampler(wl, n_steps, n_steps // 2, C, 5)
    _, _, out = smp.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], o.log, kmax=km, kz=kz,
                           occupancy=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out["z"].cpu().numpy(), o.z)
    np.testing.assert_array_equal(out["occ"].cpu().numpy(), o.occ)
    assert o.occ.sum() > 0


def test_occupancy_full_batched_size_sampled_waveforms():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, seed=wl.seed)
    n = len(b["offsets"]) - 1
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    C, n_steps, burn = wl.n_chains, wl.n_steps, wl.n_steps // 2
    print(f"[case] occupancy full batched n={n} chains={C} steps={n_steps}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 2)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz, occupancy=True)
    torch.cuda.synchronize()
    occ = out["occ"].cpu().numpy()
    nhist = out["nhist"].cpu().numpy()
    assert len(occ) == SUB * b["offsets"][-1]
    assert (occ >= 0).all()
    _row_sums_match_nhist(occ, nhist, b["offsets"], C)
    pick = np.sort(np.random.default_rng(6).choice(n, size=24, replace=False))
    lengths = np.diff(b["offsets"])[pick]
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in pick])
    o = oracle.run(oracle_params(wl), wave, off, b["lam"][pick], C, n_steps, burn, 2, kz, kmax=km[pick],
                   wave_id=pick.astype(np.uint64), occupancy=True)
    rows = (pick[:, None] * C + np.arange(C)[None, :]).reshape(-1)
    g = to_host(out)
    sub = {k: (v[rows] if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == n * C else v)
           for k, v in g.items() if k != "occ"}
    parted = compare_chains(sub, o)
    bad = set(int(c) // C for c in parted)
    for j, i in enumerate(pick):
        if j not in bad:
            np.testing.assert_array_equal(_rows(occ, b["offsets"], i), _rows(o.occ, off, j))
    print(f"[occupancy] full size: {len(pick) - len(bad)} of {len(pick)} sampled waveforms equal", flush=True)
    assert len(bad) <= 3


def test_occupancy_in_graph_and_rejected_overflow():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=30, seed=98)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    smp = gpu_sampler(wl, 200, 100, 2, 4)
    wave = torch.from_numpy(b["wave"]).cuda()
    ref = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, occupancy=True)["occ"].cpu().numpy()
    out = smp.alloc_samples(30, kz, occ_len=SUB * int(b["offsets"][-1]))
    g, out = smp.graph(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=out)
    for r in range(3):
        out["occ"].fill_(7)  # the graph's prologue must clear the rows
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out["occ"].cpu().numpy(), ref, err_msg=f"replay {r}")
    g.close()
    big = gpu_sampler(wl, 1 << 24, 0, 1, 1)
    with pytest.raises(RuntimeError):
        big.sample(wave, b["offsets"], b["lam"], kmax=np.full(30, 192, np.int32), kz=192, occupancy=True)
