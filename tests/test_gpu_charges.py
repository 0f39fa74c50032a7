"""Charge draws at recorded steps (FSMP_REC_CHARGE) against the oracle (needs an MI355X).

The kernels factor the maintained G^{-1} = R R^T backwards (R upper triangular) and draw
q = x + sigma_eps R xi; the oracle factors G = L L^T from scratch and back-solves
L^T y = xi.  Both take xi from the same Philox blocks, so on every chain whose trajectory
matches the oracle's the recorded PE lists are identical and the draws agree to rounding.
Covered: the three kernel designs, PE capacities 16..160, and the FP32-refresh form (which
draws from its FP64 rebuild of G^{-1} at the recorded steps).
"""
import numpy as np
import pytest

import oracle
from paper_2403_03156_amd import fsmp, synth
from tests.fsmp_cases import check_partings, compare_chains, gpu_sampler, oracle_params, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLAGS = fsmp.FSMP_REC_TRACE | fsmp.FSMP_REC_CHARGE


def _factory(wl, n_steps, burn, thin, seed, design, precision):
    def make(extra_flags=0):
        if precision == fsmp.FSMP_FP64:
            smp = gpu_sampler(wl, n_steps, burn, 1, seed, record_flags=FLAGS | extra_flags, thin=thin)
        else:
            smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                               t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                               sigma_q=wl.sigma_q, n_steps=n_steps, n_chains=1, burn_in=burn, seed=seed,
                               precision=precision, refresh_M=64, record_flags=FLAGS | extra_flags, thin=thin)
        if design is not None:
            smp.set_design(0, design)
        return smp
    return make


def _run(wl, b, km, n_steps, burn, thin, seed, design=None, precision=fsmp.FSMP_FP64):
    kz = int(km.max())
    print(f"[case] charges {wl.name} n={len(km)} caps={sorted(set(km.tolist()))} design={design} "
          f"precision={precision}", flush=True)
    make = _factory(wl, n_steps, burn, thin, seed, design, precision)
    smp = make()
    out = smp.sample(torch.from_numpy(b["wave"]).cuda(), b["offsets"], b["lam"], kmax=km, kz=kz)
    torch.cuda.synchronize()
    g = to_host(out)
    o = oracle.run(oracle_params(wl), b["wave"], b["offsets"], b["lam"], 1, n_steps, burn, seed, kz, kmax=km,
                   thin=thin, charges=True)
    parted = compare_chains(g, o, tol=1e-9 if precision == fsmp.FSMP_FP64 else 1e-7)
    check_partings(parted, oracle_params(wl), b, b["lam"], km, 1, n_steps, burn, seed, kz, make)
    return g, o, parted


def _check_identical_chains(g, o, parted, rtol, atol):
    keep = np.setdiff1d(np.arange(len(g["n_pe"])), parted)
    np.testing.assert_array_equal(g["zdraw"][keep], o.zdraw[keep])
    np.testing.assert_allclose(g["trace"][keep], o.trace[keep], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g["qdraw"][keep], o.qdraw[keep], rtol=rtol, atol=atol, equal_nan=True)
    n_drawn = int((o.zdraw[keep] >= 0).sum())
    print(f"[charges] {len(keep)}/{len(g['n_pe'])} chains identical, {n_drawn} PE charges drawn", flush=True)
    assert n_drawn > 0
    return keep


@pytest.mark.parametrize("design", [fsmp.FSMP_DESIGN_GROUP, fsmp.FSMP_DESIGN_LANE, fsmp.FSMP_DESIGN_GROUP_DEVMEM])
def test_charge_draws_match_oracle(design):
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=48, seed=61)
    km = synth.kmax_for(b["lam"])
    g, o, parted = _run(wl, b, km, 200, 100, 9, 17, design=design)
    _check_identical_chains(g, o, parted, rtol=1e-8, atol=1e-9)


def test_charge_draws_high_capacity():
    base = synth.PRESETS["pileup"]
    wl = synth.Workload("pileup", 6, base.lengths, "uniform", 20.0, 100.0, phi_kind=base.phi_kind,
                        tau_rise=base.tau_rise, tau_decay=base.tau_decay, sigma_q=0.35, sigma_eps=0.1)
    b = synth.generate(wl, n_wave=6, seed=5)
    km = synth.kmax_for(b["lam"])
    for design in (None, fsmp.FSMP_DESIGN_GROUP_DEVMEM, fsmp.FSMP_DESIGN_GROUP_DEVMEM_WIDE):
        g, o, parted = _run(wl, b, km, 160, 80, 20, 3, design=design)
        _check_identical_chains(g, o, parted, rtol=1e-7, atol=1e-8)


def test_charge_draws_fp32_refresh():
    wl = synth.PRESETS["batched"]
    b = synth.generate(wl, n_wave=48, seed=62)
    km = synth.kmax_for(b["lam"])
    g, o, parted = _run(wl, b, km, 200, 100, 9, 19, precision=fsmp.FSMP_FP32_REFRESH)
    # the FP32 form draws from its FP64 rebuild of G^-1 at recorded steps
    _check_identical_chains(g, o, parted, rtol=1e-7, atol=1e-8)
