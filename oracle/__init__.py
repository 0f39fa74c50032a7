"""Oracle for the FSMP sampler: a plain, slow FP64 CPU implementation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It shares no code with the
HIP path (``paper_2403_03156_amd``) and never imports it.

* ``fsmp_oracle.c`` (loaded through ctypes): SER evaluation, light curve, the
  grid prior normaliser, the from-scratch likelihood of App. A (eq. mgauss), the
  acceptances of Sec. 2.4 and the chain driver with its own Philox4x32-10.
* ``brute.py``: dense-normal likelihood, the paper's Woodbury form of delta-nu
  (App. A, eqs. 11-18) and the exact posterior by enumeration on tiny grids.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PHI_EXP = 0
PHI_BIEXP = 1
MOVE_BIRTH, MOVE_DEATH, MOVE_UPDATE = 1, 2, 3


class Params(ctypes.Structure):
    _fields_ = [
        ("ser_mu", ctypes.c_double),
        ("ser_sigma", ctypes.c_double),
        ("ser_tau", ctypes.c_double),
        ("ser_amp", ctypes.c_double),
        ("ser_support", ctypes.c_int32),
        ("sub", ctypes.c_int32),
        ("sigma_eps", ctypes.c_double),
        ("mu_q", ctypes.c_double),
        ("sigma_q", ctypes.c_double),
        ("phi_kind", ctypes.c_int32),
        ("tau_rise", ctypes.c_double),
        ("tau_decay", ctypes.c_double),
        ("t0_min", ctypes.c_double),
        ("t0_max", ctypes.c_double),
        ("J", ctypes.c_double),
        ("t0_sd", ctypes.c_double),
        ("shift_sd", ctypes.c_double),
        ("n_mix", ctypes.c_int32),
        ("mix_w", ctypes.c_double * 8),
        ("mix_mu", ctypes.c_double * 8),
        ("mix_sigma", ctypes.c_double * 8),
    ]


LOGREC_DTYPE = np.dtype(
    [("move", "<i4"), ("flags", "<i4"), ("j", "<i4"), ("g", "<i4"),
     ("t0", "<f8"), ("dnu", "<f8"), ("log_alpha", "<f8")], align=True)
assert LOGREC_DTYPE.itemsize == 40


def make_params(ser=(8.0, 1.5, 6.0), ser_amp=1.0, ser_support=0, sub=4, sigma_eps=0.1, mu_q=1.0, sigma_q=0.3,
                phi_kind=PHI_EXP, tau_rise=0.0, tau_decay=20.0, t0_min=50.0, t0_max=100.0, J=0.25,
                t0_sd=1.0, shift_sd=1.0, mix=None) -> Params:
    """mix: None (one normal charge law N(mu_q, sigma_q^2)) or (G, mu, sigma) of the MCP-PMT
    Gaussian mixture (Sec. 2.1, eq. mcp-multi-norm), up to 8 components."""
    p = Params(ser[0], ser[1], ser[2], ser_amp, ser_support, sub, sigma_eps, mu_q, sigma_q, phi_kind,
               tau_rise, tau_decay, t0_min, t0_max, J, t0_sd, shift_sd)
    if mix is not None:
        g, mu, sg = (list(map(float, v)) for v in mix)
        p.n_mix = len(g)
        for i in range(len(g)):
            p.mix_w[i], p.mix_mu[i], p.mix_sigma[i] = g[i], mu[i], sg[i]
    return p


_lib = None

_P = ctypes.POINTER
_d, _i32, _i64, _u64, _u32 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.ora_philox4x32_10.argtypes = [_vp, _vp, _vp]
        L.ora_ser_peak_time.argtypes = [_d, _d, _d]
        L.ora_ser_peak_time.restype = _d
        L.ora_ser_support_auto.argtypes = [_d, _d, _d]
        L.ora_ser_support_auto.restype = ctypes.c_int
        L.ora_ser_value.argtypes = [_P(Params), _d]
        L.ora_ser_value.restype = _d
        L.ora_ser_table.argtypes = [_P(Params), _vp, _i32]
        L.ora_ser_table.restype = _i32
        L.ora_phi.argtypes = [_P(Params), _d]
        L.ora_phi.restype = _d
        L.ora_log_phi.argtypes = [_P(Params), _d]
        L.ora_log_phi.restype = _d
        L.ora_phi_sum.argtypes = [_P(Params), _d, _i32, _i32]
        L.ora_phi_sum.restype = _d
        L.ora_lambda_T.argtypes = [_P(Params), _d, _d, _i32, _i32]
        L.ora_lambda_T.restype = _d
        L.ora_birth_draw.argtypes = [_P(Params), _d, _i32, _i32, _d]
        L.ora_birth_draw.restype = _i32
        L.ora_log_likelihood.argtypes = [_P(Params), _vp, _i32, _vp, _vp, _i32, _vp]
        L.ora_log_likelihood.restype = _d
        L.ora_overlap.argtypes = [_P(Params), _i32, _i32, _i32]
        L.ora_overlap.restype = _d
        L.ora_log_alpha.argtypes = [_P(Params), _vp, _i32, _d, _i32, _i32, _d, _vp, _i32, _i32, _i32, _i32, _vp]
        L.ora_log_alpha.restype = _d
        L.ora_t0_log_alpha.argtypes = [_P(Params), _d, _i32, _i32, _vp, _i32, _d, _d]
        L.ora_t0_log_alpha.restype = _d
        L.ora_run.argtypes = [_P(Params), _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _u64, _i32,
                              _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32,
                              _vp]
        L.ora_charge_draw.argtypes = [_P(Params), _vp, _i32, _vp, _i32, _vp, _vp]
        L.ora_charge_draw.restype = ctypes.c_int
        L.ora_charge_normals.argtypes = [_u64, _u64, _i32, _i32, _vp]
        L.ora_charge_normals.restype = None
        L.ora_run.restype = ctypes.c_int
        L.ora_replay.argtypes = [_P(Params), _vp, _i32, _d, _i32, _i32, _i32, _u64, _u64, _i32, _vp, _vp, _vp, _d, _i32,
                                 _vp, _i32]
        L.ora_replay.restype = _i64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def ser_table(p: Params):
    cap = 1 << 16
    out = np.zeros(cap, dtype=np.float64)
    LV = lib().ora_ser_table(ctypes.byref(p), _ptr(out), cap)
    return out[: p.sub * LV].copy(), LV


def log_likelihood(p: Params, w, z, e=None):
    """log p(w | z) and the charges' conditional mean; e: the PEs' mixture components (MCP form)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.int32)
    e = None if e is None else np.ascontiguousarray(e, dtype=np.int32)
    x = np.zeros(max(len(z), 1), dtype=np.float64)
    v = lib().ora_log_likelihood(ctypes.byref(p), _ptr(w), len(w), _ptr(z), _ptr(e), len(z), _ptr(x))
    return v, x[: len(z)]


def log_alpha(p, w, lam, glo, ghi, t0, z, move, j, gnew):
    w = np.ascontiguousarray(w, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.int32)
    dnu = ctypes.c_double(0.0)
    zz = z if len(z) else np.zeros(1, np.int32)
    la = lib().ora_log_alpha(ctypes.byref(p), _ptr(w), len(w), lam, glo, ghi, t0, _ptr(zz), len(z), move, j, gnew,
                             ctypes.byref(dnu))
    return la, dnu.value


def phi_sum(p, t0, glo, ghi):
    """sum of phi(g dt - t0) over the grid points glo..ghi (closed-form geometric series)"""
    return lib().ora_phi_sum(ctypes.byref(p), t0, glo, ghi)


def t0_log_alpha(p, lam, glo, ghi, z, t0, t0p):
    z = np.ascontiguousarray(z, dtype=np.int32)
    zz = z if len(z) else np.zeros(1, np.int32)
    return lib().ora_t0_log_alpha(ctypes.byref(p), lam, glo, ghi, _ptr(zz), len(z), t0, t0p)


class RunResult:
    pass


def run(p: Params, wave, offsets, lam, n_chains, n_steps, burn_in, seed, kz, kmax=None, g_range=None, t0_init=None,
        wave_id=None, log=False, thin=0, n_threads=0, charges=False, occupancy=False, z_init=None, wsteps=None):
    """Run ``n_chains`` chains per waveform; outputs are per chain (index wave*n_chains + chain).

    ``thin`` > 0 records (N, t0, Q) every thin-th step after burn-in into ``trace``; with
    ``charges`` it also records the PE list (``zdraw``) and one charge draw (``qdraw``).
    ``occupancy`` gives ``occ``: per waveform the sub * L_i grid points (the waveform's row
    starts at sub * offsets[i]), the number of (chain, recorded sweep) pairs with a PE there,
    PEs counted with multiplicity (``occ_chain`` keeps the per-chain rows).  ``z_init``: None
    (empty start) or one initial PE list (grid indices) per chain.  ``wsteps``: None, or the
    sweeps of every waveform (at most n_steps), each with burn-in wsteps * burn_in // n_steps."""
    wave = np.ascontiguousarray(wave, dtype=np.float32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nw = len(offsets) - 1
    tot = nw * n_chains
    kmax = None if kmax is None else np.ascontiguousarray(kmax, dtype=np.int32)
    g_range = None if g_range is None else np.ascontiguousarray(g_range, dtype=np.int32).reshape(-1)
    t0_init = None if t0_init is None else np.ascontiguousarray(t0_init, dtype=np.float64)
    wave_id = None if wave_id is None else np.ascontiguousarray(wave_id, dtype=np.uint64)
    wsteps = None if wsteps is None else np.ascontiguousarray(wsteps, dtype=np.int32)
    if wsteps is not None and (len(wsteps) != nw or wsteps.min() < 1 or wsteps.max() > n_steps):
        raise ValueError("wsteps: one count in 1..n_steps per waveform")
    r = RunResult()
    r.N = np.zeros(tot, np.int32)
    r.t0 = np.zeros(tot, np.float64)
    r.z = np.zeros((tot, kz), np.int32)
    r.x = np.zeros((tot, kz), np.float64)
    r.acc = np.zeros((tot, 12), np.float64)
    r.nhist = np.zeros((tot, kz + 1), np.int32)
    r.counts = np.zeros((tot, 8), np.int32)
    r.status = np.zeros(tot, np.uint32)
    r.log = np.zeros((tot, n_steps), LOGREC_DTYPE) if log else None
    n_rec = (n_steps - burn_in + thin - 1) // thin if (thin > 0 and n_steps > burn_in) else 0
    r.trace = np.zeros((tot, n_rec, 3), np.float64) if n_rec else None
    r.qdraw = np.zeros((tot, n_rec, kz), np.float64) if (n_rec and charges) else None
    r.zdraw = np.zeros((tot, n_rec, kz), np.int32) if (n_rec and charges) else None
    r.occ_chain = np.zeros(n_chains * p.sub * int(offsets[-1]), np.int32) if occupancy else None
    zi, zo = flatten_lists(z_init, tot)
    r.e = np.zeros((tot, kz), np.int32) if p.n_mix > 0 else None
    lib().ora_run(ctypes.byref(p), nw, _ptr(wave), _ptr(offsets), _ptr(lam), _ptr(kmax), _ptr(g_range),
                  _ptr(t0_init), _ptr(wave_id), n_chains, n_steps, burn_in, seed, kz, _ptr(r.N), _ptr(r.t0),
                  _ptr(r.z), _ptr(r.x), _ptr(r.acc), _ptr(r.nhist), _ptr(r.counts), _ptr(r.status), _ptr(r.log),
                  _ptr(r.trace), thin, _ptr(r.qdraw), _ptr(r.zdraw), _ptr(r.occ_chain), _ptr(zi), _ptr(zo), _ptr(r.e), n_threads,
                  _ptr(wsteps))
    r.occ = None
    if occupancy:
        # sum the chains' rows of every waveform
        r.occ = np.zeros(p.sub * int(offsets[-1]), np.int64)
        for i in range(nw):
            n_g = p.sub * int(offsets[i + 1] - offsets[i])
            base = n_chains * p.sub * int(offsets[i])
            r.occ[p.sub * offsets[i]:p.sub * offsets[i + 1]] = \
                r.occ_chain[base:base + n_chains * n_g].reshape(n_chains, n_g).sum(0)
    return r


def flatten_lists(lists, n):
    """None, or n integer lists -> (concatenated int32 values, int64 offsets n + 1)."""
    if lists is None:
        return None, None
    if len(lists) != n:
        raise ValueError(f"need {n} lists, got {len(lists)}")
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(z) for z in lists])
    flat = np.ascontiguousarray(np.concatenate([np.asarray(z, np.int32).reshape(-1) for z in lists] +
                                               [np.zeros(1, np.int32)]))
    return flat, off


def charge_draw(p: Params, w, z, xi):
    """q = x + sigma_eps L^-T xi for the PE list z (G = L L^T); None if G is not positive definite."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.int32)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    q = np.zeros(max(len(z), 1), np.float64)
    rc = lib().ora_charge_draw(ctypes.byref(p), _ptr(w), len(w), _ptr(z), len(z), _ptr(xi), _ptr(q))
    return None if rc else q[: len(z)]


def charge_normals(uid, seed, step, K):
    """The K standard normals of the charge draw at ``step`` of chain ``uid``."""
    xi = np.zeros(max(K, 1), np.float64)
    lib().ora_charge_normals(uid, seed, step, K, _ptr(xi))
    return xi[:K]


def replay(p: Params, w, lam, kmax, glo, ghi, uid, seed, rec, tie_eps=1e-9, ext=False, z_init=None):
    """Recompute delta-nu / log-alpha along a recorded log of one chain.  ext: delta-nu as the
    difference of two from-scratch nu's in extended precision (long double), else in FP64.
    z_init: None (empty start) or the chain's initial PE list (grid indices), as `run` takes it.

    Returns (dnu_ref, la_ref, n_decision_mismatches)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    rec = np.ascontiguousarray(rec, dtype=LOGREC_DTYPE)
    n = len(rec)
    dnu = np.zeros(n, np.float64)
    la = np.zeros(n, np.float64)
    z0 = np.ascontiguousarray(z_init if z_init is not None else [], dtype=np.int32)
    bad = lib().ora_replay(ctypes.byref(p), _ptr(w), len(w), lam, kmax, glo, ghi, uid, seed, n, _ptr(rec),
                           _ptr(dnu), _ptr(la), tie_eps, 1 if ext else 0, _ptr(z0) if len(z0) else None, len(z0))
    return dnu, la, int(bad)


def summarize(acc, n_steps, burn_in, n_chains):
    """Posterior mean / variance / MCSE of (N, Q, t0) per waveform from the per-chain accumulators
    (batch means with floor(sqrt(S)) batches per chain, pooled over chains)."""
    acc = np.asarray(acc).reshape(-1, n_chains, 12)
    S = n_steps - burn_in
    nb = int(np.floor(np.sqrt(S)))
    lb = S // nb
    out = {}
    for a, name in enumerate(("N", "Q", "t0")):
        s1 = acc[:, :, 2 * a].sum(1)
        s2 = acc[:, :, 2 * a + 1].sum(1)
        n = S * n_chains
        mean = s1 / n
        var = np.maximum(s2 / n - mean ** 2, 0.0)
        bsum = acc[:, :, 6 + 2 * a].sum(1)
        bsq = acc[:, :, 7 + 2 * a].sum(1)
        B = nb * n_chains
        bm_mean = bsum / (B * lb)
        bm_var = np.maximum((bsq / lb ** 2 - B * bm_mean ** 2) / max(B - 1, 1), 0.0)
        out[name] = (mean, var, np.sqrt(bm_var / B))
    return out


def chain_diagnostics(acc, S, n_chains):
    """Per waveform and for each of (N, Q, t0), from the per-chain sums of v and v^2 over
    S recorded sweeps:

    * the Gelman-Rubin potential scale reduction (Sec. 3.2 convergence check; the form of
      Gelman and Rubin 1992 without the degrees-of-freedom factor or chain splitting):
      chain means m_i and unbiased chain variances s_i^2, W = mean of s_i^2,
      B = S / (C - 1) sum_i (m_i - m)^2, V = (S - 1) / S W + B / S, R = sqrt(V / W);
      R = 1 when V = W = 0 (every chain constant at one value), inf when only W = 0,
      NaN with fewer than 2 chains or 2 sweeps;
    * the Monte Carlo error of the pooled mean from the spread of the chain means,
      sqrt(sum_i (m_i - m)^2 / (C (C - 1))) (NaN with fewer than 2 chains).
    Returns (rhat [n_wave, 3], mcse_chains [n_wave, 3])."""
    acc = np.asarray(acc, np.float64).reshape(-1, n_chains, 12)
    nw = acc.shape[0]
    rhat = np.full((nw, 3), np.nan)
    mcb = np.full((nw, 3), np.nan)
    if n_chains < 2:
        return rhat, mcb
    for a in range(3):
        m = acc[:, :, 2 * a] / S
        dev2 = ((m - m.mean(1, keepdims=True)) ** 2).sum(1)
        mcb[:, a] = np.sqrt(dev2 / (n_chains * (n_chains - 1)))
        if S < 2:
            continue
        s2 = np.maximum((acc[:, :, 2 * a + 1] - S * m * m) / (S - 1), 0.0)
        W = s2.mean(1)
        B = S * dev2 / (n_chains - 1)
        V = (S - 1) / S * W + B / S
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.sqrt(V / W)
        r[(W == 0) & (V == 0)] = 1.0
        r[(W == 0) & (V > 0)] = np.inf
        rhat[:, a] = r
    return rhat, mcb


def lambda_mle(hist, lam0, n_grid=64):
    """lambda-hat of eq. reduce-mu0: the maximiser over lambda >= 0 of
        f(lambda) = -(lambda - lambda0) + log sum_k h_k (lambda / lambda0)^k,
    the importance-sampling estimate of log p(w | lambda, t0) from the sampled PE counts
    (h_k: the sweeps with N = k, any normalisation; the whole-line normaliser e^-lambda of
    eq. pzmu).  Stationary points solve d(lambda) = m(lambda) - lambda = 0, m the mean of k
    under the weights h_k (lambda / lambda0)^k; the maxima are where d goes from + to -, and
    all lie between the smallest and largest k with h_k > 0 (k_lo, k_hi).
    Steps: a single support point k gives k; otherwise d on n_grid evenly spaced points of
    [k_lo, k_hi]; every grid interval with d > 0 at its left end and d <= 0 at its right
    end holds a maximum, found by scipy's brentq to 1e-14; lambda = 0 is a candidate too
    when k_lo = 0 and d <= 0 at the second grid point; the candidate with the largest f
    wins (the smallest lambda of equals)."""
    from scipy.optimize import brentq
    h = np.asarray(hist, np.float64)
    ks = np.nonzero(h > 0)[0]
    if len(ks) == 0:
        return np.nan
    k_lo, k_hi = float(ks[0]), float(ks[-1])
    if k_lo == k_hi:
        return k_lo
    k = np.arange(len(h), dtype=np.float64)
    lh = np.full(len(h), -np.inf)
    lh[h > 0] = np.log(h[h > 0])

    def tilt(lam):
        # log-weights of the tilted law; lambda = 0 keeps k = 0 only
        a = np.where(k == 0, lh, -np.inf) if lam == 0.0 else lh + k * np.log(lam / lam0)
        mx = a.max()
        return mx, np.exp(a - mx)

    def f(lam):
        mx, e = tilt(lam)
        return -(lam - lam0) + mx + np.log(e.sum())

    def d(lam):
        _, e = tilt(lam)
        return (k * e).sum() / e.sum() - lam

    grid = k_lo + (k_hi - k_lo) * np.arange(n_grid) / (n_grid - 1)
    dv = np.array([d(x) for x in grid])
    cand = []
    if k_lo == 0.0 and dv[1] <= 0:
        cand.append(0.0)
    for i in range(n_grid - 1):
        if dv[i] > 0 and dv[i + 1] <= 0:
            cand.append(grid[i + 1] if dv[i + 1] == 0 else brentq(d, grid[i], grid[i + 1], xtol=1e-14, rtol=1e-14,
                                                                   maxiter=500))
    fv = [f(x) for x in cand]
    return cand[int(np.argmax(fv))]
