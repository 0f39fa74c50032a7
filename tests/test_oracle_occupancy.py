"""The oracle's grid occupancy (expected number of PEs at each grid point, the PE sequence
of Sec. 2.2 seen as a point pattern on the grid of T) against what fixes it independently:

* tiny grids: the MCMC occupancy against enumeration of every multiset (App. A
  likelihood, Sec. 2.2 prior on the grid), t0 fixed and t0 integrated out; the same
  estimate shifted by one grid point must fail the comparison (the test has the power to
  see an index slip);
* data term off: given N the PE positions are i.i.d. with density h, so the occupancy is
  E[N] h on every grid point;
* every row sums to the sum of N over the recorded steps, and equals the histogram of the
  PE lists recorded at every step.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from tests.test_oracle_chain import _tiny, _wave


def _run(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn, seed=7, t0_init=None, **kw):
    offsets = np.array([0, len(w)], np.int64)
    return oracle.run(p, w, offsets, np.array([lam]), n_chains, n_steps, burn, seed, kz=kmax,
                      kmax=np.array([kmax], np.int32), g_range=np.array([glo, ghi], np.int32),
                      t0_init=None if t0_init is None else np.array([t0_init]), occupancy=True, **kw)


@pytest.mark.parametrize("t0_sampled", [False, True])
def test_occupancy_matches_enumeration(t0_sampled):
    if t0_sampled:
        p, m = _tiny(0, t0_range=(0.5, 2.0))
        Lw, glo, ghi, kmax, lam = 12, 6, 15, 3, 1.8
        w = _wave(m, Lw, [9, 12], [1.0, 1.1], seed=5)
        exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=None)
        t0i = 1.0
    else:
        p, m = _tiny(1)
        Lw, glo, ghi, kmax, lam = 12, 6, 17, 3, 1.6
        w = _wave(m, Lw, [8, 13], [1.0, 0.8], seed=22)
        exact = brute.posterior_exact(m, w.astype(np.float64), lam, glo, ghi, kmax, t0=1.0)
        t0i = None
    n_chains, n_steps, burn = 32, 30000, 1500
    r = _run(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn, t0_init=t0i)
    S = n_chains * (n_steps - burn)
    est = r.occ / S
    assert len(est) == p.sub * Lw
    assert (r.occ[:glo] == 0).all() and (r.occ[ghi + 1:] == 0).all()
    got = est[glo:ghi + 1]
    want = exact["occupancy"]
    np.testing.assert_allclose(got, want, atol=0.012)
    np.testing.assert_allclose(got.sum(), exact["EN"], atol=0.02)
    # an index slip of one grid point is visible at this precision
    assert np.abs(np.roll(got, 1) - want).max() > 0.05


def test_occupancy_prior_only_is_EN_times_h():
    p, m = _tiny(0)
    p.ser_amp = 0.0
    Lw, glo, ghi, kmax, lam = 24, 0, 95, 12, 3.0
    w = np.zeros(Lw, np.float32)
    n_chains, n_steps, burn = 32, 30000, 1000
    r = _run(p, w, lam, glo, ghi, kmax, n_chains, n_steps, burn)
    S = n_chains * (n_steps - burn)
    est = r.occ[glo:ghi + 1] / S
    EN = r.acc[:, 0].sum() / S
    h = m.h(1.0, glo, ghi)
    # coarse bins: relative error of a few percent at this chain length
    edges = [0, 4, 8, 16, 32, 96]
    for a, b in zip(edges[:-1], edges[1:]):
        want = EN * h[a:b].sum()
        if want > 0.05:
            assert abs(est[a:b].sum() - want) < 0.05 * want + 0.01, (a, b, est[a:b].sum(), want)
    # positions before t0 carry no intensity
    t0g = int(np.ceil(1.0 * p.sub))
    assert (r.occ[:t0g] == 0).all()


def test_occupancy_rows_sum_to_N_and_match_recorded_lists():
    p = oracle.make_params(t0_min=0.0, t0_max=10.0)
    rng = np.random.default_rng(3)
    lengths = np.array([40, 64, 33, 80])
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    wave = (0.1 * rng.standard_normal(offsets[-1])).astype(np.float32)
    for i, L in enumerate(lengths):
        for t in rng.uniform(5, L - 10, size=3):
            n = np.arange(L)
            wave[offsets[i]:offsets[i + 1]] += np.exp(-0.5 * ((n - t - 4) / 1.5) ** 2).astype(np.float32)
    lam = np.array([6.0, 8.0, 4.0, 10.0])
    C, n_steps, burn = 3, 400, 150
    r = oracle.run(p, wave, offsets, lam, C, n_steps, burn, 11, 24, thin=1, charges=True, occupancy=True)
    for i in range(len(lengths)):
        row = r.occ[p.sub * offsets[i]:p.sub * offsets[i + 1]]
        ks = np.arange(25)
        assert row.sum() == (r.nhist[i * C:(i + 1) * C] * ks).sum()
        assert int(row.sum()) == int(round(r.acc[i * C:(i + 1) * C, 0].sum()))
        zl = r.zdraw[i * C:(i + 1) * C]
        want = np.bincount(zl[zl >= 0], minlength=len(row))
        np.testing.assert_array_equal(row, want)
        assert row.sum() > 0
