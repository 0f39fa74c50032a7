"""fsmp_sample_noalloc, the variant of fsmp_sample that allocates nothing (its workspace is a
static device array per GPU), against fsmp_sample through the C ABI (needs an MI355X).

Two calls in a row on one context, the second with a smaller batch (the scratch array keeps
the first call's contents), each compared with fsmp_sample on the same batch: every output
identical (the same kernels on the same inputs; only the launch order of the capacity
buckets differs).  Also: a batch beyond the array's size or the host arrays' limits is
rejected with a message, and the call leaves torch's device memory untouched."""
import numpy as np
import pytest

from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import gpu_sampler, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("n_pe", "t0", "z", "charge", "acc", "nhist", "counts", "status", "rec_steps", "work")


def _compare(smp, wl, n, seed, n_steps_w=None):
    b = synth.generate(wl, n_wave=n, seed=seed)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[case] noalloc {wl.name} n={n} seed={seed} caps={sorted(set(km.tolist()))}", flush=True)
    wave = torch.from_numpy(b["wave"]).cuda()
    steps = None if n_steps_w is None else n_steps_w[:n]
    ref = to_host(smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, n_steps=steps, work=True))
    out = smp.alloc_samples(n, kz, work=True)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, n_steps=steps, out=out, noalloc=True)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    got = to_host(out)
    for k in KEYS:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    return b, km


def test_noalloc_equals_sample_twice_second_smaller():
    wl = synth.PRESETS["uneven"]
    smp = gpu_sampler(wl, 300, 150, 2, 5, k_max=160)
    steps = np.random.default_rng(4).integers(100, 301, 400).astype(np.int32)
    _compare(smp, wl, 400, 21, steps)
    _compare(smp, wl, 60, 22, steps)


def test_noalloc_rejects_batches_beyond_its_limits():
    wl = synth.PRESETS["batched"]
    smp = gpu_sampler(wl, 10, 5, 8, 1)
    n = 65536 // 2 + 1   # 32,769 waveforms x 8 chains: more chains than the host arrays hold
    off = np.arange(n + 1, dtype=np.int64) * 16
    wave = torch.zeros(int(off[-1]), dtype=torch.float32, device="cuda")
    lam = np.full(n, 1.0)
    km = np.full(n, 16, np.int32)
    with pytest.raises(RuntimeError, match="at most"):
        smp.sample(wave, off, lam, kmax=km, kz=16, noalloc=True)
    # a workspace beyond the 256 MiB array: 60,000 windows of 2,048 samples (matched filter of
    # 8,192 grid points each, 3.9 GB)
    smp1 = gpu_sampler(wl, 10, 5, 1, 1)
    n = 60000
    off = np.arange(n + 1, dtype=np.int64) * 2048
    wave = torch.zeros(int(off[-1]), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="scratch"):
        smp1.sample(wave, off, np.full(n, 1.0), kmax=np.full(n, 16, np.int32), kz=16, noalloc=True)
