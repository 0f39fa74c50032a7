"""Parity of the HIP path with the oracle, through the C ABI (needs an MI355X).

Both sides draw every random number from the same Philox4x32-10 stream (each its
own implementation), so in FP64 a chain's whole trajectory must agree: final PE
lists and histograms exactly, t0 and the accumulators to 1e-9 relative, and
every replayed delta-nu to 1e-9 relative (|dnu_gpu - dnu_ref| / max(|dnu_ref|, 1)).
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DNU_TOL = 1e-9


def _run_both(wl, n_wave, n_steps, burn, n_chains, seed, data_seed, log=False, kmax=None):
    b = synth.generate(wl, n_wave=n_wave, seed=data_seed)
    km = synth.kmax_for(b["lam"]) if kmax is None else np.full(n_wave, kmax, np.int32)
    kz = int(km.max())
    print(f"[case] {wl.name} n_wave={n_wave} steps={n_steps} chains={n_chains} kz={kz}", flush=True)
    flags = 2 if log else 0
    smp = gpu_sampler(wl, n_steps, burn, n_chains, seed, record_flags=flags)
    wave = torch.from_numpy(b["wave"]).cuda()
    out = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz)
    torch.cuda.synchronize()
    g = to_host(out)
    p = oracle_params(wl)
    o = oracle.run(p, b["wave"], b["offsets"], b["lam"], n_chains, n_steps, burn, seed, kz, kmax=km, log=log)
    return b, km, smp, out, g, o


@pytest.mark.parametrize("data_seed", [0, 1])
def test_trajectory_parity_plain(data_seed):
    wl = synth.PRESETS["plain"]
    b, km, smp, out, g, o = _run_both(wl, 96, 600, 300, 1, 0, data_seed)
    parted = compare_chains(g, o)
    assert len(parted) == 0, f"chains parted from the oracle: {parted[:10]}"
    assert (g["counts"][:, 3] > 0).mean() > 0.7  # most chains accepted births


def test_trajectory_parity_biexp_multichain():
    wl = synth.PRESETS["batched"]
    b, km, smp, out, g, o = _run_both(wl, 24, 400, 200, 4, 5, 2)
    assert set(np.unique(synth.kmax_for(b["lam"]))) >= {16}
    parted = compare_chains(g, o)
    assert len(parted) == 0, f"chains parted from the oracle: {parted[:10]}"


def test_replay_delta_nu():
    wl = synth.PRESETS["batched"]
    b, km, smp, out, g, o = _run_both(wl, 12, 300, 150, 2, 9, 3, log=True)
    from paper_2403_03156_amd import fsmp
    logs = fsmp.log_records(out["log"])
    p = oracle_params(wl)
    off = b["offsets"]
    worst = 0.0
    nvalid = 0
    for c in range(logs.shape[0]):
        i = c // 2
        w = b["wave"][off[i]:off[i + 1]]
        dnu, la, bad = oracle.replay(p, w, b["lam"][i], int(km[i]), 0, 4 * len(w) - 1, c, 9, logs[c])
        assert bad == 0, f"chain {c}: decisions differ from the oracle's"
        v = (logs[c]["flags"] & 1) != 0
        nvalid += v.sum()
        err = np.abs(logs[c]["dnu"][v] - dnu[v]) / np.maximum(np.abs(dnu[v]), 1.0)
        worst = max(worst, float(err.max()) if err.size else 0.0)
    assert nvalid > 500
    assert worst < DNU_TOL, worst
    # the GPU's own log agrees with the oracle's log record for record
    np.testing.assert_array_equal(logs["move"], o.log["move"])
    np.testing.assert_array_equal(logs["flags"], o.log["flags"])
    np.testing.assert_array_equal(logs["g"], o.log["g"])


def test_posterior_kernel_matches_oracle_summary():
    wl = synth.PRESETS["plain"]
    n_steps, burn, C = 500, 200, 2
    b, km, smp, out, g, o = _run_both(wl, 40, n_steps, burn, C, 3, 4)
    post = smp.posterior(40, out)
    torch.cuda.synchronize()
    s = oracle.summarize(o.acc, n_steps, burn, C)
    for a, name in enumerate(("N", "Q", "t0")):
        np.testing.assert_allclose(post["mean"][:, a].cpu().numpy(), s[name][0], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(post["var"][:, a].cpu().numpy(), s[name][1], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(post["mcse"][:, a].cpu().numpy(), s[name][2], rtol=1e-6, atol=1e-9)
    pn = post["p_n"].cpu().numpy()
    np.testing.assert_allclose(pn.sum(1), 1.0, atol=1e-12)
