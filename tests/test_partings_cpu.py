"""The rule the GPU parity tests apply to chains that part from the oracle (a parting must sit
at a near-tie of a decision at the first step where the proposal logs differ), checked on
the CPU with the oracle's own logs: identical logs show no difference, and differences
planted into a copy of a log are found at their step, attributed to the right decision and,
being no ties, rejected."""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import TIE, assert_partings_explained, first_difference, oracle_params, tie_at


def _chains():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=6, seed=3)
    km = synth.kmax_for(b["lam"])
    p = oracle_params(wl)
    o = oracle.run(p, b["wave"], b["offsets"], b["lam"], 2, 200, 100, 5, int(km.max()), kmax=km, log=True)
    return wl, b, km, p, o


def test_identical_logs_show_no_difference():
    _, b, km, p, o = _chains()
    o2 = oracle.run(p, b["wave"], b["offsets"], b["lam"], 2, 200, 100, 5, int(km.max()), kmax=km, log=True)
    for c in range(o.log.shape[0]):
        assert first_difference(o2.log[c], o.log[c]) is None


def test_planted_differences_are_found_and_rejected():
    _, b, km, p, o = _chains()
    c = int(np.argmax(o.N))              # a chain with PEs
    i = c // 2
    L = int(b["offsets"][i + 1] - b["offsets"][i])
    uid = i * 2 + c % 2
    log = o.log[c]
    acc = np.where((log["flags"] & 3) == 3)[0]
    s = int(acc[len(acc) // 2])          # an accepted jump
    ga = log.copy()
    ga[s]["flags"] &= ~2
    assert first_difference(ga, log) == s
    kind, margin = tie_at(p, float(b["lam"][i]), 0, 4 * L - 1, uid, 5, ga, log, s, 75.0)
    lu = np.log((float(oracle.philox4x32_10([s, 1, uid, 0], [5, 0])[2]) + 0.5) * 2.0 ** -32)
    assert kind == "jump"
    assert margin == pytest.approx(abs(lu - log[s]["log_alpha"]) / max(1.0, abs(log[s]["log_alpha"])), rel=1e-12)
    assert margin > TIE
    with pytest.raises(AssertionError):
        assert_partings_explained([c], p, b, b["lam"], 2, 5, lambda cs: ga[None], lambda cs: log[None], km)
    # a t0 decision turned the other way
    t = np.where(log["flags"] & 4)[0]
    s = int(t[len(t) // 2])
    ga = log.copy()
    ga[s]["flags"] &= ~4
    ga[s]["t0"] = log[s - 1]["t0"]
    kind, margin = tie_at(p, float(b["lam"][i]), 0, 4 * L - 1, uid, 5, ga, log, s, 75.0)
    assert kind == "t0" and margin > TIE
    # a different birth position
    bth = np.where((log["move"] == oracle.MOVE_BIRTH) & (log["flags"] & 1))[0]
    s = int(bth[len(bth) // 2])
    ga = log.copy()
    ga[s]["g"] += 1
    kind, margin = tie_at(p, float(b["lam"][i]), 0, 4 * L - 1, uid, 5, ga, log, s, 75.0)
    assert kind == "birth" and margin > TIE
