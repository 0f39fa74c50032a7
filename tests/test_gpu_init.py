"""Chains started from given PE sequences (fsmp_batch.z_init) against the oracle (needs an
MI355X).

The kernels build G^-1 and the charges of a start list by bordering, one forced birth per
PE before the first sweep; the oracle factors the list from scratch.  Checked: every kernel
design at capacities 16-64 (chains must match the oracle's element by element), start
lists of up to 150 PEs at capacities 160 and 192, the replay of the oracle's own proposals
from the start lists (delta-nu to 1e-9 relative from the first step on, which holds only
if the initial G^-1 is right), and the host-side rejection of invalid lists.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, ext_reference, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SUB = 4


def _starts(wl, b, km, n_chains, seed, max_len=None):
    """Random start lists: per chain 0..min(kmax, max_len) PEs inside the window where phi
    is positive at the default t0_init (the middle of the t0 prior)."""
    rng = np.random.default_rng(seed)
    t0 = 0.5 * (wl.t0_min + wl.t0_max)
    out = []
    for i in range(len(km)):
        L = int(b["offsets"][i + 1] - b["offsets"][i])
        lo = int(np.floor(t0 * SUB)) + 1
        for _ in range(n_chains):
            cap = int(km[i]) if max_len is None else min(int(km[i]), max_len)
            n = int(rng.integers(0, cap + 1))
            out.append(rng.integers(lo, SUB * L, size=n).tolist())
    return out


@pytest.mark.parametrize("design", [None, fsmp.FSMP_DESIGN_GROUP, fsmp.FSMP_DESIGN_LANE,
                                    fsmp.FSMP_DESIGN_GROUP_DEVMEM, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE])
def test_started_chains_match_oracle(design):
    wl = synth.PRESETS["batched"]
    n, C, n_steps, burn = 60, 2, 300, 150
    b = synth.generate(wl, n_wave=n, seed=141)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    z0 = _starts(wl, b, km, C, 1, max_len=24)
    print(f"[case] start lists design={design} n={n} longest={max(len(z) for z in z0)}", flush=True)
    smp = gpu_sampler(wl, n_steps, burn, C, 23)
    if design is not None:
        smp.set_design(0, design)
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz, z_init=z0))
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, burn, 23, kz, kmax=km, z_init=z0)
    parted = compare_chains(g, o)
    print(f"[init] {len(parted)} of {n * C} chains parted", flush=True)

    def make(flags):
        m = gpu_sampler(wl, n_steps, burn, C, 23, record_flags=flags)
        if design is not None:
            m.set_design(0, design)
        return m
    check_partings(parted, oracle_params(wl), b, b["lam"], km, C, n_steps, burn, 23, kz, make, z_init=z0)


def test_long_start_lists_high_capacity():
    wl = synth.PRESETS["pileup"]
    lam = np.array([60.0, 90.0, 100.0, 100.0])
    b = synth.generate(wl, n_wave=len(lam), seed=15, lam=lam)
    km = synth.kmax_for(b["lam"])
    assert km.max() >= 160
    z0 = _starts(wl, b, km, 1, 2)
    z0 = [z if len(z) > 60 else z + z[: 60] for z in z0]   # long lists, some grid points twice
    z0 = [z[: int(k)] for z, k in zip(z0, km)]
    print(f"[case] long start lists caps={km.tolist()} lengths={[len(z) for z in z0]}", flush=True)
    smp = gpu_sampler(wl, 150, 75, 1, 8)
    g = to_host(smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=int(km.max()),
                           z_init=z0))
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], 1, 150, 75, 8, int(km.max()), kmax=km,
                   z_init=z0)
    parted = compare_chains(g, o, tol=1e-7)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, 1, 150, 75, 8, int(km.max()),
                   lambda flags: gpu_sampler(wl, 150, 75, 1, 8, record_flags=flags), z_init=z0)


@pytest.mark.parametrize("preset", ["batched", "pileup"])
def test_replay_from_start_lists(preset):
    wl = synth.PRESETS[preset]
    if preset == "pileup":
        b = synth.generate(wl, n_wave=3, seed=16, lam=np.array([40.0, 70.0, 100.0]))
        C, n_steps = 1, 120
    else:
        b = synth.generate(wl, n_wave=30, seed=142)
        C, n_steps = 2, 200
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    z0 = _starts(wl, b, km, C, 3)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], C, n_steps, n_steps // 2, 6, kz, kmax=km,
                   log=True, z_init=z0)
    smp = gpu_sampler(wl, n_steps, n_steps // 2, C, 6)
    dnu, la, out = smp.replay(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], o.log, kmax=km, kz=kz,
                              z_init=z0)
    torch.cuda.synchronize()
    dnu = dnu.cpu().numpy()
    valid = (o.log["flags"] & 1) != 0
    # pile-up: nu(z), nu(z') reach ~1e6, so the reference is the extended-precision replay from
    # the same start lists, not the FP64 difference in the oracle's log
    ref = o.log["dnu"] if preset == "batched" else ext_reference(oracle_params(wl), b, km, o.log, C, 6, z_init=z0)[0]
    err = np.abs(dnu - ref)[valid] / np.maximum(np.abs(ref[valid]), 1.0)
    print(f"[init] replay {preset}: {valid.sum()} proposals, max rel err {err.max():.2e}, first-step max "
          f"{(np.abs(dnu - ref)[:, 0][valid[:, 0]] / np.maximum(np.abs(ref[:, 0][valid[:, 0]]), 1)).max():.2e}",
          flush=True)
    assert err.max() < 1e-9
    np.testing.assert_array_equal(out["z"].cpu().numpy(), o.z)


def test_invalid_start_lists_rejected():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=2, seed=1)
    km = np.array([16, 16], np.int32)
    smp = gpu_sampler(wl, 20, 10, 1, 1)
    wave = torch.from_numpy(b["wave"]).cuda()
    good = [[400, 500], [1000]]
    smp.sample(wave, b["offsets"], b["lam"], kmax=km, z_init=good)
    for bad in ([[400] * 17, []],          # more than kmax
                [[SUB * 1024], []],        # outside T
                [[100], []],               # before t0 (phi = 0)
                [[400]]):                  # one list per chain
        with pytest.raises((RuntimeError, ValueError)):
            smp.sample(wave, b["offsets"], b["lam"], kmax=km, z_init=bad)
    with pytest.raises(RuntimeError):
        smp.sample(wave, b["offsets"], np.array([0.0, 1.0]), kmax=km, z_init=good)
