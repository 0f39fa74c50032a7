"""Side streams of the capacity buckets (needs an MI355X).

fsmp_sample deals the PE-capacity buckets of a call to at most GPU_MAX_HW_QUEUES lanes, the
caller's stream and side streams (the library reads the variable at every call; HIP's own
queue count is fixed at start-up and is not changed here). The stream a bucket runs on, and
which buckets share a stream, must not change a single output. A batch of the uneven workload
(seven buckets) is sampled with one, two, three and eight lanes and compared with the default
four, output by output and bit for bit; and after the design autotuner (whose trial times
then set the buckets' costs) with one lane and with the default.
"""
import numpy as np
import pytest

from paper_2403_03156_amd import synth
from tests.fsmp_cases import gpu_sampler, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_REF = {}


def _run(wl, b, km):
    smp = gpu_sampler(wl, 200, 100, 2, 13)
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=int(km.max()))
    torch.cuda.synchronize()
    return to_host(out)


def _batch():
    wl = synth.PRESETS["uneven"]
    lam = np.concatenate([np.full(6, 0.5), np.full(6, 6.0), np.full(6, 15.0), np.full(6, 25.0),
                          np.full(4, 40.0), np.full(4, 65.0), np.full(4, 90.0)])
    b = synth.generate(wl, n_wave=len(lam), seed=23, lam=lam)
    km = synth.kmax_for(b["lam"])
    return wl, b, km


@pytest.mark.parametrize("queues", ["1", "2", "3", "8"])
def test_outputs_do_not_depend_on_side_streams(queues, monkeypatch):
    wl, b, km = _batch()
    assert len(set(km.tolist())) >= 6
    if "ref" not in _REF:
        monkeypatch.delenv("GPU_MAX_HW_QUEUES", raising=False)
        print(f"[case] lanes default caps={sorted(set(km.tolist()))}", flush=True)
        _REF["ref"] = _run(wl, b, km)
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", queues)
    print(f"[case] lanes {queues}", flush=True)
    g = _run(wl, b, km)
    ref = _REF["ref"]
    for k, v in ref.items():
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(g[k], v, err_msg=f"{k} with {queues} lanes")


def test_tuned_costs_do_not_change_outputs(monkeypatch):
    wl, b, km = _batch()
    smp = gpu_sampler(wl, 200, 100, 2, 13)
    wave = torch.from_numpy(b["wave"]).cuda()
    print("[case] lanes after the design autotuner", flush=True)
    smp.autotune(wave, b["offsets"], b["lam"], kmax=km, trial_steps=20)
    res = {}
    for queues in ("1", None):
        if queues is None:
            monkeypatch.delenv("GPU_MAX_HW_QUEUES", raising=False)
        else:
            monkeypatch.setenv("GPU_MAX_HW_QUEUES", queues)
        out = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=int(km.max()))
        torch.cuda.synchronize()
        res[queues] = to_host(out)
    for k, v in res["1"].items():
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(res[None][k], v, err_msg=k)
