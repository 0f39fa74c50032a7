"""The extended-precision reference of the oracle's replay (delta-nu as the difference of two
from-scratch nu's in long double, App. A eqs. mgauss and 11-18 in PE space) against the
definition evaluated with 40 significant digits (mpmath): the overlaps and matched-filter
terms summed exactly from the double SER table and the float samples, log det G and
b^T G^-1 b by an mpmath Cholesky factorisation.  On small PE counts it also equals the FP64
replay; on pile-up states (K ~ 100, nu ~ 1e6) the FP64 difference of two nu's carries their
rounding and the extended one does not."""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import synth
from tests.fsmp_cases import oracle_params

mpmath = pytest.importorskip("mpmath")


def _nu_mp(p, vtab, w, z):
    """nu(z) = -1/2 [-K log rho + log det G + (K rho mu^2 - b^T G^-1 b) / s] with 40 digits"""
    mp = mpmath.mp
    mp.dps = 40
    M = len(vtab)
    sub = p.sub
    K = len(z)
    s = mp.mpf(p.sigma_eps) ** 2
    rho = s / mp.mpf(p.sigma_q) ** 2
    m = mp.mpf(p.mu_q)
    cols = []
    for g in z:
        n0 = max(0, -(-g // sub))
        n1 = min(len(w) - 1, (g + M - 1) // sub)
        cols.append({n: mp.mpf(float(vtab[sub * n - g])) for n in range(n0, n1 + 1) if 0 <= sub * n - g < M})
    G = mp.matrix(K, K)
    b = mp.matrix(K, 1)
    for i in range(K):
        for k in range(i + 1):
            ci, ck = cols[i], cols[k]
            v = mp.fsum(ci[n] * ck[n] for n in ci if n in ck)
            G[i, k] = v
            G[k, i] = v
        G[i, i] += rho
        b[i] = mp.fsum(v * mp.mpf(float(w[n])) for n, v in cols[i].items()) + rho * m
    L = mp.cholesky(G)
    logdet = 2 * mp.fsum(mp.log(L[i, i]) for i in range(K))
    y = mp.lu_solve(L, b)  # L y = b (L lower triangular, its LU is itself)
    uu = mp.fsum(y[i] ** 2 for i in range(K))
    return -(-K * mp.log(rho) + logdet + (K * rho * m * m - uu) / s) / 2


def _states(log, s):
    """PE lists before and after the proposal of step s of a log"""
    z = []
    for k in range(s):
        r = log[k]
        if r["flags"] & 2:
            if r["move"] == oracle.MOVE_BIRTH:
                z.append(int(r["g"]))
            elif r["move"] == oracle.MOVE_DEATH:
                z[r["j"]] = z[-1]
                z.pop()
            else:
                z[r["j"]] = int(r["g"])
    r = log[s]
    zp = list(z)
    if r["move"] == oracle.MOVE_BIRTH:
        zp.append(int(r["g"]))
    elif r["move"] == oracle.MOVE_DEATH:
        zp[r["j"]] = zp[-1]
        zp.pop()
    else:
        zp[r["j"]] = int(r["g"])
    return z, zp


def test_extended_replay_equals_fp64_replay_at_small_k():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=4, seed=31)
    km = synth.kmax_for(b["lam"])
    p = oracle_params(wl)
    o = oracle.run(p, b["wave"], b["offsets"], b["lam"], 1, 200, 100, 3, int(km.max()), kmax=km, log=True)
    for i in range(4):
        w = b["wave"][b["offsets"][i]:b["offsets"][i + 1]]
        L = len(w)
        d64, _, bad64 = oracle.replay(p, w, b["lam"][i], int(km[i]), 0, 4 * L - 1, i, 3, o.log[i])
        dx, _, badx = oracle.replay(p, w, b["lam"][i], int(km[i]), 0, 4 * L - 1, i, 3, o.log[i], ext=True)
        assert bad64 == 0 and badx == 0
        np.testing.assert_allclose(dx, d64, rtol=1e-10, atol=1e-10)


def test_extended_replay_matches_40_digit_definition_on_pileup():
    wl = synth.PRESETS["pileup"]
    b = synth.generate(wl, n_wave=1, seed=9, lam=np.array([90.0]))
    km = synth.kmax_for(b["lam"])
    p = oracle_params(wl)
    n_steps = 400
    o = oracle.run(p, b["wave"], b["offsets"], b["lam"], 1, n_steps, 200, 4, int(km.max()), kmax=km, log=True)
    w = b["wave"]
    L = len(w)
    dx, _, _ = oracle.replay(p, w, b["lam"][0], int(km[0]), 0, 4 * L - 1, 0, 4, o.log[0], ext=True)
    vtab, _ = oracle.ser_table(p)
    valid = np.where(o.log[0]["flags"] & 1)[0]
    checked = 0
    for s in valid[::-1]:
        z, zp = _states(o.log[0], s)
        if len(z) < 60 or o.log[0][s]["move"] == oracle.MOVE_DEATH or checked >= 2:
            continue
        want = _nu_mp(p, vtab, w, zp) - _nu_mp(p, vtab, w, z)
        got = dx[s]
        print(f"step {s}: K {len(z)} -> {len(zp)}, delta-nu {float(want):.6f}, extended error "
              f"{abs(got - float(want)):.2e}, FP64 error {abs(o.log[0][s]['dnu'] - float(want)):.2e}")
        assert abs(got - float(want)) <= 1e-11 * max(1.0, abs(float(want)))
        checked += 1
    assert checked == 2
