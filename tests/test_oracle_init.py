"""The oracle started from given PE sequences (Sec. 2.3: an initial guess of z speeds up
convergence but does not change the target; Sec. 3.2: chains from different starts).

* tiny grids: chains started from random multisets (different per chain) reach the
  enumerated posterior P(N = k), E[N];
* explicit empty lists equal the default start bit for bit;
* the start is the state: the first proposal's delta-nu is measured from the start list
  (both likelihoods from scratch), and the charges are the conditional mean of the
  final list.
"""
import numpy as np

import oracle
from oracle import brute
from tests.test_oracle_chain import _tiny, _wave


def test_random_starts_reach_enumerated_posterior():
    p, m = _tiny(0)
    Lw, glo, ghi, kmax, lam = 12, 6, 17, 3, 1.6
    w = _wave(m, Lw, [8, 13], [1.0, 0.8], seed=21)
    exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=1.0)
    rng = np.random.default_rng(9)
    C = 48
    # t0 = 1 is fixed; EXP phi is positive from g = sub * t0 = 4 on, and T = [6, 17]
    starts = [sorted(rng.integers(glo, ghi + 1, size=int(rng.integers(0, kmax + 1))).tolist()) for _ in range(C)]
    r = oracle.run(p, w, np.array([0, Lw], np.int64), np.array([lam]), C, 30000, 2000, 7, kz=kmax,
                   kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32), z_init=starts)
    s = oracle.summarize(r.acc, 30000, 2000, C)
    mean, _, mcse = (v[0] for v in s["N"])
    assert abs(mean - exact["EN"]) < 4 * mcse + 1e-12
    pN = r.nhist.sum(0)[: kmax + 1] / r.nhist.sum()
    np.testing.assert_allclose(pN, exact["pN"], atol=0.012)


def test_empty_lists_equal_default_start():
    p = oracle.make_params(t0_min=0.0, t0_max=10.0)
    rng = np.random.default_rng(3)
    L = 48
    w = (0.1 * rng.standard_normal(2 * L)).astype(np.float32)
    off = np.array([0, L, 2 * L], np.int64)
    a = oracle.run(p, w, off, np.array([4.0, 6.0]), 2, 200, 100, 5, 12)
    b = oracle.run(p, w, off, np.array([4.0, 6.0]), 2, 200, 100, 5, 12, z_init=[[], [], [], []])
    for k in ("N", "t0", "z", "x", "acc", "nhist", "counts", "status"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))


def test_start_is_the_state():
    # the first proposal's delta-nu is measured from the start list: nu(z') - nu(z0) with
    # both terms from scratch, and the final charges are the conditional mean of the final z
    p = oracle.make_params(t0_min=0.0, t0_max=10.0)
    L = 40
    g0 = [40, 55, 90]
    rng = np.random.default_rng(1)
    wave = np.zeros(L, np.float64)
    tab, LV = oracle.ser_table(p)
    for g in g0:
        for n in range(L):
            k = p.sub * n - g
            if 0 <= k < len(tab):
                wave[n] += tab[k]
    wave = (wave + 0.05 * rng.standard_normal(L)).astype(np.float32)
    checked = 0
    for seed in range(1, 30):
        r = oracle.run(p, wave, np.array([0, L], np.int64), np.array([3.0]), 1, 3, 0, seed, 8, z_init=[g0], log=True)
        rec = r.log[0, 0]
        if not (rec["flags"] & 1):
            continue
        zp = list(g0)
        if rec["move"] == oracle.MOVE_BIRTH:
            zp.append(int(rec["g"]))
        elif rec["move"] == oracle.MOVE_DEATH:
            zp[rec["j"]] = zp[-1]
            zp.pop()
        else:
            zp[rec["j"]] = int(rec["g"])
        want = oracle.log_likelihood(p, wave, zp)[0] - oracle.log_likelihood(p, wave, g0)[0]
        assert abs(rec["dnu"] - want) <= 1e-9 * max(1.0, abs(want))
        z = r.z[0][r.z[0] >= 0].tolist()
        _, x = oracle.log_likelihood(p, wave, z)
        np.testing.assert_allclose(r.x[0][:len(z)], x, rtol=1e-9, atol=1e-12)
        checked += 1
    assert checked >= 10


def test_replay_from_start_list():
    # the replay started from a chain's start list follows that chain's own run: its FP64
    # delta-nu equals the logged one and every accept decision is re-derived; from the empty
    # list the same log is not the chain's (the deaths name PEs the empty start lacks)
    from paper_2403_03156_amd import synth
    p = oracle.make_params()
    b = synth.generate(synth.PRESETS["plain"], n_wave=3, seed=5)
    off = b["offsets"]
    kz, C, seed = 16, 2, 12
    rng = np.random.default_rng(4)
    starts = []
    for i in range(3):
        L = int(off[i + 1] - off[i])
        for _ in range(C):
            starts.append(sorted(rng.integers(40, p.sub * L - 1, size=int(rng.integers(2, 6))).tolist()))
    r = oracle.run(p, b["wave"], off, b["lam"], C, 300, 150, seed, kz, z_init=starts, log=True)
    differs = 0
    for i in range(3):
        w = b["wave"][off[i]:off[i + 1]]
        for ch in range(C):
            row = i * C + ch
            rec = r.log[row]
            valid = (rec["flags"] & 1) != 0
            assert valid.sum() > 100
            args = (p, w, b["lam"][i], kz, 0, 4 * len(w) - 1, row, seed, rec)
            dnu, la, bad = oracle.replay(*args, z_init=starts[row])
            assert bad == 0
            np.testing.assert_array_equal(dnu[valid], rec["dnu"][valid])
            dx, _, badx = oracle.replay(*args, z_init=starts[row], ext=True)
            assert badx == 0
            np.testing.assert_allclose(dx[valid], rec["dnu"][valid], rtol=1e-9, atol=1e-9)
            d0, _, bad0 = oracle.replay(*args)
            differs += bad0 > 0 or not np.array_equal(d0[valid], rec["dnu"][valid])
    assert differs == 3 * C
    # more PEs than kmax is refused
    w = b["wave"][off[0]:off[1]]
    assert oracle.replay(p, w, b["lam"][0], 3, 0, 4 * len(w) - 1, 0, seed, r.log[0], z_init=starts[0] + [50] * 4)[2] == -1
