"""Serving loop (fsmp_server_*): continuous batching of trigger events (needs an MI355X).

* each event's results are identical alone and mixed with other events in micro-batches
  spread over several streams (FP64 and the FP32-refresh form: chains are keyed by the
  (event, channel) identity and never interact);
* a served event agrees with the oracle run on the same identities;
* a memory budget smaller than one micro-batch still drains the queue (one batch at a time).
"""
import time

import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_STEPS = 300


def _events(n_events, seed, lo=20, hi=120):
    wl = synth.PRESETS["serving"]
    rng = np.random.default_rng(seed)
    ev = []
    for e in range(n_events):
        n = int(rng.integers(lo, hi))
        b = synth.generate(wl, n_wave=n, seed=seed * 1000 + e)
        ev.append((1000 + e, b, synth.kmax_for(b["lam"])))
    return wl, ev


def _kwargs(wl, precision):
    return dict(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay, t0_min=wl.t0_min,
                t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q, n_steps=N_STEPS,
                n_chains=1, seed=3, precision=precision, refresh_M=64)


def _serve(srv, events, timeout=60.0):
    for eid, b, km in events:
        srv.submit(eid, b["wave"], b["offsets"], b["lam"], km)
    res = {}
    t_end = time.time() + timeout
    while len(res) < len(events):
        srv.progress(wait=True)
        for eid, _, _ in events:
            if eid not in res:
                r = srv.result(eid)
                if r is not None:
                    res[eid] = r
        assert time.time() < t_end, "server did not drain"
    return res


@pytest.mark.parametrize("precision", [fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH])
def test_alone_equals_mixed(precision):
    wl, events = _events(6, 1)
    kw = _kwargs(wl, precision)
    alone = {}
    for ev in events:
        srv = fsmp.Server(kw, n_streams=1, max_batch_wave=1 << 20)
        alone.update(_serve(srv, [ev]))
        srv.close()
    srv = fsmp.Server(kw, n_streams=3, max_batch_wave=150)  # micro-batches mix 1-3 events
    mixed = _serve(srv, events)
    srv.close()
    for eid, _, _ in events:
        np.testing.assert_array_equal(alone[eid]["mean"], mixed[eid]["mean"])
        np.testing.assert_array_equal(alone[eid]["mcse"], mixed[eid]["mcse"])
        np.testing.assert_array_equal(alone[eid]["status"], mixed[eid]["status"])
        assert mixed[eid]["latency"] > 0


def test_served_event_matches_oracle():
    wl, events = _events(2, 7)
    srv = fsmp.Server(_kwargs(wl, fsmp.FSMP_FP64), n_streams=2, max_batch_wave=1 << 20)
    res = _serve(srv, events)
    srv.close()
    p = oracle_params(wl)
    for eid, b, km in events:
        n = len(km)
        wid = (np.uint64(eid) << np.uint64(16)) + np.arange(n, dtype=np.uint64)
        o = oracle.run(p, b["wave"], b["offsets"], b["lam"], 1, N_STEPS, N_STEPS // 2, 3, int(km.max()), kmax=km,
                       wave_id=wid)
        s = oracle.summarize(o.acc, N_STEPS, N_STEPS // 2, 1)
        for a, name in enumerate(("N", "Q", "t0")):
            np.testing.assert_allclose(res[eid]["mean"][:, a], s[name][0], rtol=1e-9, atol=1e-9)


def test_tight_memory_budget_drains():
    wl, events = _events(5, 11)
    srv = fsmp.Server(_kwargs(wl, fsmp.FSMP_FP64), n_streams=4, max_batch_wave=1 << 20, memory_budget=1 << 16)
    res = _serve(srv, events)
    st = srv.stats()
    srv.close()
    assert len(res) == 5 and st["queued"] == 0 and st["in_flight"] == 0 and st["bytes_held"] == 0
