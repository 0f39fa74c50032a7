"""Shared set-up for the parity tests: one workload description drives both the HIP
path (through the C ABI binding) and the oracle, with identical seeded inputs."""
import concurrent.futures

import numpy as np

import oracle
from paper_2403_03156_amd import synth


def oracle_params(wl: synth.Workload, ser_amp=1.0, t0_sd=1.0, shift_sd=1.0, J=0.25, sub=4, support=0):
    return oracle.make_params(ser=wl.ser, ser_amp=ser_amp, ser_support=support, sub=sub, sigma_eps=wl.sigma_eps,
                              mu_q=wl.mu_q, sigma_q=wl.sigma_q, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise,
                              tau_decay=wl.tau_decay, t0_min=wl.t0_min, t0_max=wl.t0_max, J=J, t0_sd=t0_sd,
                              shift_sd=shift_sd)


def gpu_sampler(wl: synth.Workload, n_steps, burn_in, n_chains, seed, k_max=64, record_flags=0, thin=1,
                ser_amp=1.0, t0_sd=1.0, shift_sd=1.0, J=0.25, sub=4, support=0, t0_range=None):
    from paper_2403_03156_amd import fsmp
    t0_min, t0_max = t0_range if t0_range else (wl.t0_min, wl.t0_max)
    return fsmp.Sampler(ser=wl.ser, ser_amp=ser_amp, ser_support=support, phi_kind=wl.phi_kind,
                        tau_rise=wl.tau_rise, tau_decay=wl.tau_decay, t0_min=t0_min, t0_max=t0_max,
                        sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q, grid_sub=sub, jump_J=J,
                        t0_step_sd=t0_sd, shift_sd=shift_sd, k_max=k_max, n_steps=n_steps, n_chains=n_chains,
                        burn_in=burn_in, thin=thin, record_flags=record_flags, seed=seed)


def to_host(out):
    res = {}
    for k, v in out.items():
        if k == "kz" or v is None:
            res[k] = v
        else:
            res[k] = v.cpu().numpy()
    return res


def compare_chains(g, o, tol=1e-9):
    """Element-by-element comparison of GPU and oracle per-chain outputs.

    Returns the indices of chains whose integer results differ (trajectories that
    parted), after asserting float agreement on every chain that did not part."""
    same = (g["n_pe"] == o.N) & (g["z"] == o.z).all(1) & (g["nhist"] == o.nhist).all(1) & \
        (g["counts"] == o.counts).all(1) & (g["status"].astype(np.uint32) == o.status)
    idx = np.where(same)[0]
    np.testing.assert_allclose(g["t0"][idx], o.t0[idx], rtol=tol, atol=tol)
    np.testing.assert_allclose(g["acc"][idx], o.acc[idx], rtol=tol, atol=tol)
    np.testing.assert_allclose(g["charge"][idx], o.x[idx], rtol=max(tol * 10, 1e-8), atol=max(tol / 10, 1e-10))
    return np.where(~same)[0]


# ------------------------------------------------------------------ partings
# With the same Philox stream on both sides, an FP64 chain of the HIP path can part from the
# oracle's only where a decision is a near-tie that rounding may settle either way: an accept
# test log U < log alpha, the t0 test, the birth's inverse-CDF search, or the rounding of an
# update shift to the grid.  Every parting must be explained by such a tie at the first step
# where the two proposal logs differ.
TIE = 1e-8


def _u01(r):
    return (float(r) + 0.5) * 2.0 ** -32


def _u53(lo, hi):
    return float(((int(hi) << 32) | int(lo)) >> 11) * 2.0 ** -53 + 2.0 ** -54


def _words(step, uid, seed):
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    ctr = [step, 0, uid & 0xFFFFFFFF, (uid >> 32) & 0xFFFFFFFF]
    r0 = oracle.philox4x32_10(ctr, key)
    ctr[1] = 1
    return np.concatenate([r0, oracle.philox4x32_10(ctr, key)])


def first_difference(ga, ob):
    """first step where two proposal logs of one chain differ, or None"""
    for s in range(len(ob)):
        a, b = ga[s], ob[s]
        if (int(a["move"]), int(a["flags"]), int(a["j"]), int(a["g"])) != \
                (int(b["move"]), int(b["flags"]), int(b["j"]), int(b["g"])) or \
                not np.isclose(a["t0"], b["t0"], rtol=1e-9, atol=1e-9):
            return s
    return None


def tie_at(p, lam, glo, ghi, uid, seed, ga, ob, s, t0_init, z_init=()):
    """(kind, margin) of the decision at step s, where the GPU's log ga and the oracle's log ob
    first differ: margin = how far the oracle's deciding value lies from its threshold,
    relative (|log U - log alpha| / max(1, |log alpha|) for the accept tests, the relative
    distance of the birth target from the partial sum between the two grid points, the
    distance of an update shift from a rounding boundary).  Infinite when the difference is not
    a decision at all (a state difference, which a tie earlier would have shown)."""
    r = _words(s, uid, seed)
    z = list(z_init)
    for k in range(s):
        rec = ob[k]
        if rec["flags"] & 2:
            if rec["move"] == oracle.MOVE_BIRTH:
                z.append(int(rec["g"]))
            elif rec["move"] == oracle.MOVE_DEATH:
                z[rec["j"]] = z[-1]
                z.pop()
            else:
                z[rec["j"]] = int(rec["g"])
    t0 = float(ob[s - 1]["t0"]) if s > 0 else float(t0_init)
    a, b = ga[s], ob[s]
    R = np.sqrt(-2.0 * np.log(_u01(r[0])))
    th = 2.0 * np.pi * _u01(r[1])
    if ((int(a["flags"]) ^ int(b["flags"])) & 4) or not np.isclose(a["t0"], b["t0"], rtol=1e-9, atol=1e-9):
        t0p = t0 + p.t0_sd * R * np.cos(th)
        la = oracle.t0_log_alpha(p, lam, glo, ghi, z, t0, t0p)
        lu = np.log(_u01(r[2]))
        return "t0", (abs(lu - la) / max(1.0, abs(la)) if np.isfinite(la) else np.inf)
    if a["move"] != b["move"] or a["j"] != b["j"]:
        return "state", np.inf
    if a["g"] != b["g"]:
        if b["move"] == oracle.MOVE_BIRTH:
            target = _u53(r[4], r[5]) * oracle.phi_sum(p, t0, glo, ghi)
            gsplit = int(min(a["g"], b["g"]))
            return "birth", abs(oracle.phi_sum(p, t0, glo, gsplit) - target) / target
        x = R * np.sin(th) * p.shift_sd * p.sub
        return "shift", abs(abs(x - np.floor(x)) - 0.5)
    if (int(a["flags"]) ^ int(b["flags"])) & 1:
        return "valid", np.inf
    lu = np.log(_u01(r[6]))
    la = float(b["log_alpha"])
    return "jump", abs(lu - la) / max(1.0, abs(la))


def assert_partings_explained(parted, p, b, lam, n_chains, seed, gpu_logs, ora_logs, kmax, g_range=None,
                              t0_init=None, wave_id=None, tie=TIE, z_init=None):
    """every chain in `parted` (chain index wave * n_chains + chain) must part at a near-tie;
    gpu_logs / ora_logs: a function of the list of parted chains giving their logs (rows in the
    order of the list); z_init: the chains' start lists, or None"""
    parted = [int(c) for c in parted]
    if not parted:
        return
    gl, ol = gpu_logs(parted), ora_logs(parted)
    sub = p.sub
    for row, c in enumerate(parted):
        i = c // n_chains
        L = int(b["offsets"][i + 1] - b["offsets"][i])
        glo, ghi = (int(g_range[i][0]), int(g_range[i][1])) if g_range is not None else (0, sub * L - 1)
        t0i = float(t0_init[i]) if t0_init is not None else 0.5 * (p.t0_min + p.t0_max)
        wid = int(wave_id[i]) if wave_id is not None else i
        uid = wid * n_chains + c % n_chains
        s = first_difference(gl[row], ol[row])
        assert s is not None, f"chain {c}: results differ but the proposal logs agree"
        kind, margin = tie_at(p, float(lam[i]), glo, ghi, uid, seed, gl[row], ol[row], s, t0i,
                              z_init=() if z_init is None else tuple(z_init[c]))
        print(f"[parting] chain {c} (waveform {i}) parts at step {s}: {kind}, margin {margin:.2e}", flush=True)
        assert margin < tie, f"chain {c}: parts at step {s} ({kind}) with margin {margin:.2e}, not a near-tie"


def gpu_log_runner(make_sampler, kz):
    """rerun function for rerun_logs: make_sampler(record_flags) builds the sampler of the test
    with the proposal log switched on"""
    def run(wave, off, lam, km, gr, ti, wid, z0=None):
        import torch
        from paper_2403_03156_amd import fsmp
        smp = make_sampler(fsmp.FSMP_REC_LOG)
        out = smp.sample(torch.from_numpy(np.ascontiguousarray(wave)).cuda(), off, lam, kmax=km, kz=kz, g_range=gr,
                         t0_init=ti, wave_id=wid, z_init=z0)
        torch.cuda.synchronize()
        return fsmp.log_records(out["log"])
    return run


def oracle_log_runner(p, n_chains, n_steps, burn, seed, kz):
    def run(wave, off, lam, km, gr, ti, wid, z0=None):
        return oracle.run(p, wave, off, lam, n_chains, n_steps, burn, seed, kz, kmax=km, g_range=gr, t0_init=ti,
                          wave_id=wid, log=True, z_init=z0).log
    return run


def check_partings(parted, p, b, lam, kmax, n_chains, n_steps, burn, seed, kz, make_sampler, g_range=None,
                   t0_init=None, wave_id=None, z_init=None):
    """every parted chain of a run must part at a near-tie (see tie_at); the parted chains'
    waveforms are rerun on both sides with proposal logs (z_init: the chains' start lists,
    one per chain, or None)"""
    if len(parted) == 0:
        return
    ids = np.arange(len(lam), dtype=np.uint64) if wave_id is None else np.asarray(wave_id, np.uint64)

    def sub_batch(chains):
        waves = sorted(set(int(c) // n_chains for c in chains))
        off = np.concatenate([[0], np.cumsum([b["offsets"][i + 1] - b["offsets"][i] for i in waves])]).astype(np.int64)
        wave = np.concatenate([b["wave"][b["offsets"][i]:b["offsets"][i + 1]] for i in waves])
        sel = np.array(waves)
        gr = None if g_range is None else np.asarray(g_range)[sel]
        ti = None if t0_init is None else np.asarray(t0_init)[sel]
        rows = [waves.index(int(c) // n_chains) * n_chains + int(c) % n_chains for c in chains]
        z0 = None if z_init is None else [list(z_init[i * n_chains + ch]) for i in waves for ch in range(n_chains)]
        return (wave, off, np.asarray(lam)[sel], np.asarray(kmax)[sel], gr, ti, ids[sel], z0), rows

    run_g = gpu_log_runner(make_sampler, kz)
    run_o = oracle_log_runner(p, n_chains, n_steps, burn, seed, kz)

    def gl(chains):
        args, rows = sub_batch(chains)
        return run_g(*args)[rows]

    def ol(chains):
        args, rows = sub_batch(chains)
        return run_o(*args)[rows]
    assert_partings_explained(parted, p, b, lam, n_chains, seed, gl, ol, kmax, g_range=g_range, t0_init=t0_init,
                              wave_id=ids, z_init=z_init)


def ext_reference(p, b, km, log, n_chains, seed, z_init=None):
    """delta-nu and log-alpha along the log from the oracle's extended-precision replay (the
    chains replayed side by side on the host cores; z_init: the chains' start lists or None)"""
    def one(c):
        i = c // n_chains
        w = b["wave"][b["offsets"][i]:b["offsets"][i + 1]]
        return oracle.replay(p, w, b["lam"][i], int(km[i]), 0, 4 * len(w) - 1, c, seed, log[c], ext=True,
                             z_init=None if z_init is None else z_init[c])
    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(one, range(log.shape[0])))
    assert all(r[2] == 0 for r in res)
    return np.stack([r[0] for r in res]), np.stack([r[1] for r in res])
