"""Thin Python binding of libfsmp.so (include/fsmp.h), same names as the C ABI.

Argument marshalling only: torch tensors supply device memory and the current HIP
stream; every step of the sampler runs in the library's HIP kernels.  There is no
fallback: if the library is missing or the device is not a gfx950, calls raise.
"""
import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsmp.so")

FSMP_OK, FSMP_EINVAL, FSMP_ENOMEM, FSMP_EDEVICE, FSMP_ENOTSUP, FSMP_EBUSY = 0, -1, -2, -3, -4, -5
FSMP_PHI_EXP, FSMP_PHI_BIEXP = 0, 1
FSMP_FP64, FSMP_FP32_REFRESH = 0, 1
FSMP_REC_TRACE, FSMP_REC_LOG, FSMP_REC_CHARGE = 1, 2, 4
FSMP_ST_KMAX, FSMP_ST_NONFINITE, FSMP_ST_DRIFT, FSMP_ST_EMPTY_T, FSMP_ST_FACTOR = 1, 2, 4, 8, 16

EXPORTS = ("fsmp_create", "fsmp_workspace_bytes", "fsmp_sample", "fsmp_posterior", "fsmp_last_timings",
           "fsmp_set_timing", "fsmp_last_error", "fsmp_destroy", "fsmp_version", "fsmp_server_create",
           "fsmp_server_submit", "fsmp_server_progress", "fsmp_server_result", "fsmp_server_stats",
           "fsmp_server_last_error", "fsmp_server_destroy", "fsmp_set_design", "fsmp_get_design", "fsmp_autotune",
           "fsmp_graph_create", "fsmp_graph_launch", "fsmp_graph_destroy", "fsmp_replay",
           "fsmp_autotune_steps", "fsmp_sample_noalloc")
FSMP_DESIGN_GROUP, FSMP_DESIGN_LANE, FSMP_DESIGN_GROUP_DEVMEM, FSMP_DESIGN_GROUP_DEVMEM_WIDE = 0, 1, 2, 3


class fsmp_ser(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("amplitude", ctypes.c_double), ("support", ctypes.c_int32)]


class fsmp_intensity(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tau_rise", ctypes.c_double), ("tau_decay", ctypes.c_double),
                ("t0_min", ctypes.c_double), ("t0_max", ctypes.c_double)]


class fsmp_config(ctypes.Structure):
    _fields_ = [("sigma_eps", ctypes.c_double), ("mu_q", ctypes.c_double), ("sigma_q", ctypes.c_double),
                ("grid_sub", ctypes.c_int32), ("jump_J", ctypes.c_double), ("t0_step_sd", ctypes.c_double),
                ("shift_sd", ctypes.c_double), ("k_max", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("burn_in", ctypes.c_int32), ("thin", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refresh_M", ctypes.c_int32), ("record_flags", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("n_mix", ctypes.c_int32), ("mix_weight", ctypes.c_double * 8),
                ("mix_mu", ctypes.c_double * 8), ("mix_sigma", ctypes.c_double * 8)]


class fsmp_batch(ctypes.Structure):
    _fields_ = [("n_wave", ctypes.c_int64), ("wave", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("lambda_", ctypes.c_void_p), ("kmax", ctypes.c_void_p), ("g_range", ctypes.c_void_p),
                ("t0_init", ctypes.c_void_p), ("wave_id", ctypes.c_void_p), ("n_steps", ctypes.c_void_p),
                ("z_init", ctypes.c_void_p), ("z_init_offsets", ctypes.c_void_p)]


class fsmp_samples(ctypes.Structure):
    _fields_ = [("n_pe", ctypes.c_void_p), ("t0", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("charge", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("nhist", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("status", ctypes.c_void_p), ("log", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("kz", ctypes.c_int32), ("work", ctypes.c_void_p),
                ("qdraw", ctypes.c_void_p), ("zdraw", ctypes.c_void_p), ("rec_steps", ctypes.c_void_p),
                ("occ", ctypes.c_void_p), ("comp", ctypes.c_void_p)]


class fsmp_posterior_out(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("var", ctypes.c_void_p), ("mcse", ctypes.c_void_p),
                ("p_n", ctypes.c_void_p), ("accept", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("occupancy", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("rhat", ctypes.c_void_p),
                ("mcse_chains", ctypes.c_void_p), ("lambda_hat", ctypes.c_void_p), ("lambda_", ctypes.c_void_p)]


class fsmp_lucy_out(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("n_pe", ctypes.c_void_p), ("g_range", ctypes.c_void_p),
                ("t0", ctypes.c_void_p), ("lambda_", ctypes.c_void_p), ("cut", ctypes.c_void_p),
                ("qhat", ctypes.c_void_p), ("kz", ctypes.c_int32)]


class fsmp_server_config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch_wave", ctypes.c_int64), ("memory_budget", ctypes.c_size_t)]


class fsmp_timing(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("kcap", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("chains", ctypes.c_int64), ("blocks", ctypes.c_int64), ("ms", ctypes.c_double)]


LOGREC_DTYPE = np.dtype([("move", "<i4"), ("flags", "<i4"), ("j", "<i4"), ("g", "<i4"),
                         ("t0", "<f8"), ("dnu", "<f8"), ("log_alpha", "<f8")], align=True)

_lib = None


class FsmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fsmp status {status}: {msg}")
        self.status = status


def load(path: Optional[str] = None):
    """Load libfsmp.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    # torch first: the library then binds to the HIP runtime torch has loaded, so device
    # pointers and streams from torch tensors are valid in it
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} is not built; run python -m paper_2403_03156_amd.build")
    L = ctypes.CDLL(p)
    P = ctypes.POINTER
    L.fsmp_create.argtypes = [P(ctypes.c_void_p), P(fsmp_ser), P(fsmp_intensity), P(fsmp_config), ctypes.c_int]
    L.fsmp_create.restype = ctypes.c_int
    L.fsmp_workspace_bytes.argtypes = [ctypes.c_void_p, P(fsmp_batch)]
    L.fsmp_workspace_bytes.restype = ctypes.c_size_t
    L.fsmp_sample.argtypes = [ctypes.c_void_p, P(fsmp_batch), P(fsmp_samples), ctypes.c_void_p]
    L.fsmp_sample.restype = ctypes.c_int
    L.fsmp_sample_noalloc.argtypes = [ctypes.c_void_p, P(fsmp_batch), P(fsmp_samples), ctypes.c_void_p]
    L.fsmp_sample_noalloc.restype = ctypes.c_int
    L.fsmp_posterior.argtypes = [ctypes.c_void_p, ctypes.c_int64, P(fsmp_samples), P(fsmp_posterior_out),
                                 ctypes.c_void_p]
    L.fsmp_posterior.restype = ctypes.c_int
    L.fsmp_last_timings.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    L.fsmp_last_timings.restype = ctypes.c_int32
    L.fsmp_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fsmp_set_timing.restype = ctypes.c_int
    L.fsmp_last_error.argtypes = [ctypes.c_void_p]
    L.fsmp_last_error.restype = ctypes.c_char_p
    L.fsmp_destroy.argtypes = [ctypes.c_void_p]
    L.fsmp_destroy.restype = None
    L.fsmp_version.argtypes = []
    L.fsmp_version.restype = ctypes.c_char_p
    L.fsmp_server_create.argtypes = [P(ctypes.c_void_p), P(fsmp_ser), P(fsmp_intensity), P(fsmp_config), ctypes.c_int,
                                     P(fsmp_server_config)]
    L.fsmp_server_create.restype = ctypes.c_int
    L.fsmp_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    L.fsmp_server_submit.restype = ctypes.c_int
    L.fsmp_server_progress.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fsmp_server_progress.restype = ctypes.c_int32
    L.fsmp_server_result.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     P(ctypes.c_double)]
    L.fsmp_server_result.restype = ctypes.c_int
    L.fsmp_server_stats.argtypes = [ctypes.c_void_p, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64),
                                    P(ctypes.c_size_t)]
    L.fsmp_server_stats.restype = ctypes.c_int
    L.fsmp_server_last_error.argtypes = [ctypes.c_void_p]
    L.fsmp_server_last_error.restype = ctypes.c_char_p
    L.fsmp_server_destroy.argtypes = [ctypes.c_void_p]
    L.fsmp_server_destroy.restype = None
    L.fsmp_set_design.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    L.fsmp_set_design.restype = ctypes.c_int
    L.fsmp_get_design.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fsmp_get_design.restype = ctypes.c_int32
    L.fsmp_autotune.argtypes = [ctypes.c_void_p, P(fsmp_batch), ctypes.c_int32, ctypes.c_void_p]
    L.fsmp_autotune.restype = ctypes.c_int
    L.fsmp_graph_create.argtypes = [ctypes.c_void_p, P(fsmp_batch), P(fsmp_samples), ctypes.c_void_p,
                                    P(ctypes.c_void_p)]
    L.fsmp_graph_create.restype = ctypes.c_int
    L.fsmp_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.fsmp_graph_launch.restype = ctypes.c_int
    L.fsmp_graph_destroy.argtypes = [ctypes.c_void_p]
    L.fsmp_graph_destroy.restype = None
    L.fsmp_replay.argtypes = [ctypes.c_void_p, P(fsmp_batch), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              P(fsmp_samples), ctypes.c_void_p]
    L.fsmp_replay.restype = ctypes.c_int
    L.fsmp_autotune_steps.argtypes = [ctypes.c_void_p, P(fsmp_batch), ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    L.fsmp_autotune_steps.restype = ctypes.c_int
    L.fsmp_lucy.argtypes = [ctypes.c_void_p, P(fsmp_batch), ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                            P(fsmp_lucy_out), ctypes.c_void_p]
    L.fsmp_lucy.restype = ctypes.c_int
    L.fsmp_ser_support.argtypes = [ctypes.c_void_p]
    L.fsmp_ser_support.restype = ctypes.c_int32
    _lib = L
    return L


def _hptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def fsmp_create(ser: fsmp_ser, phi: fsmp_intensity, cfg: fsmp_config, device: int = 0):
    L = load()
    h = ctypes.c_void_p()
    s = L.fsmp_create(ctypes.byref(h), ctypes.byref(ser), ctypes.byref(phi), ctypes.byref(cfg), device)
    if s != FSMP_OK:
        raise FsmpError(s, L.fsmp_last_error(None).decode())
    return h


class Sampler:
    """Owns one fsmp_ctx; ``sample`` takes a device waveform tensor and host metadata."""

    @staticmethod
    def default_refresh(precision):
        """FP64 rebuilds of G^-1 every this many sweeps by default: 128 in both forms."""
        return 128

    def __init__(self, ser=(8.0, 1.5, 6.0), ser_amp=1.0, ser_support=0, phi_kind=FSMP_PHI_EXP, tau_rise=0.0,
                 tau_decay=20.0, t0_min=50.0, t0_max=100.0, sigma_eps=0.1, mu_q=1.0, sigma_q=0.3, grid_sub=4,
                 jump_J=0.25, t0_step_sd=1.0, shift_sd=1.0, k_max=32, n_steps=2000, n_chains=1, burn_in=None,
                 thin=1, precision=FSMP_FP64, refresh_M=None, record_flags=0, seed=0, device=0, mix=None):
        """mix: None (charge law N(mu_q, sigma_q^2)) or (weights, means, sigmas) of the MCP-PMT
        Gaussian mixture, up to 8 components.  refresh_M: None for default_refresh(precision)."""
        if refresh_M is None:
            refresh_M = self.default_refresh(precision)
        self.lib = load()
        self.ser = fsmp_ser(ser[0], ser[1], ser[2], ser_amp, ser_support)
        self.phi = fsmp_intensity(phi_kind, tau_rise, tau_decay, t0_min, t0_max)
        if burn_in is None:
            burn_in = n_steps // 2
        self.cfg = fsmp_config(sigma_eps, mu_q, sigma_q, grid_sub, jump_J, t0_step_sd, shift_sd, k_max, n_steps,
                               n_chains, burn_in, thin, precision, refresh_M, record_flags, seed)
        if mix is not None:
            g, mu, sg = (list(map(float, v)) for v in mix)
            if not (len(g) == len(mu) == len(sg)) or len(g) > 8:
                raise ValueError("mix needs equal-length weights, means and sigmas (at most 8)")
            self.cfg.n_mix = len(g)
            for i in range(len(g)):
                self.cfg.mix_weight[i], self.cfg.mix_mu[i], self.cfg.mix_sigma[i] = g[i], mu[i], sg[i]
        self.device = device
        self.h = fsmp_create(self.ser, self.phi, self.cfg, device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.fsmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s != FSMP_OK:
            raise FsmpError(s, self.lib.fsmp_last_error(self.h).decode())

    def set_timing(self, on: bool):
        self._check(self.lib.fsmp_set_timing(self.h, 1 if on else 0))

    def last_timings(self):
        n = self.lib.fsmp_last_timings(self.h, None, 0)
        arr = (fsmp_timing * max(n, 1))()
        self.lib.fsmp_last_timings(self.h, arr, n)
        return [{"name": t.name.decode(), "kcap": t.kcap, "lanes": t.lanes, "chains": t.chains, "blocks": t.blocks,
                 "ms": t.ms} for t in arr[:n]]

    def alloc_samples(self, n_wave, kz, work=False, occ_len=0):
        """Device output buffers; occ_len > 0 adds the grid occupancy (grid_sub * offsets[-1])."""
        import torch
        dev = torch.device("cuda", self.device)
        C = n_wave * self.cfg.n_chains
        S = self.cfg.n_steps - self.cfg.burn_in
        out = {
            "n_pe": torch.zeros(C, dtype=torch.int32, device=dev),
            "t0": torch.zeros(C, dtype=torch.float64, device=dev),
            "z": torch.zeros((C, kz), dtype=torch.int32, device=dev),
            "charge": torch.zeros((C, kz), dtype=torch.float64, device=dev),
            "acc": torch.zeros((C, 12), dtype=torch.float64, device=dev),
            "nhist": torch.zeros((C, kz + 1), dtype=torch.int32, device=dev),
            "counts": torch.zeros((C, 8), dtype=torch.int32, device=dev),
            "status": torch.zeros(C, dtype=torch.int32, device=dev),
            "rec_steps": torch.zeros(C, dtype=torch.int32, device=dev),
            "log": None, "trace": None, "kz": kz,
            "work": torch.zeros((C, 5), dtype=torch.float64, device=dev) if work else None,
            "occ": torch.zeros(occ_len, dtype=torch.int32, device=dev) if occ_len > 0 else None,
            "comp": torch.zeros((C, kz), dtype=torch.int32, device=dev) if self.cfg.n_mix > 0 else None,
        }
        if self.cfg.record_flags & FSMP_REC_LOG:
            out["log"] = torch.zeros((C, self.cfg.n_steps * LOGREC_DTYPE.itemsize), dtype=torch.uint8, device=dev)
        n_rec = (S + self.cfg.thin - 1) // self.cfg.thin if (S > 0 and self.cfg.thin > 0) else 0
        if self.cfg.record_flags & FSMP_REC_TRACE:
            out["trace"] = torch.zeros((C, max(n_rec, 1), 3), dtype=torch.float64, device=dev)
        if self.cfg.record_flags & FSMP_REC_CHARGE:
            out["qdraw"] = torch.zeros((C, max(n_rec, 1), kz), dtype=torch.float64, device=dev)
            out["zdraw"] = torch.zeros((C, max(n_rec, 1), kz), dtype=torch.int32, device=dev)
        return out

    def _batch(self, wave, offsets, lam, kmax=None, g_range=None, t0_init=None, wave_id=None, n_steps=None,
               z_init=None):
        import torch
        if not wave.is_cuda or wave.dtype != torch.float32 or not wave.is_contiguous():
            raise ValueError("wave must be a contiguous float32 device tensor")
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        kmax = None if kmax is None else np.ascontiguousarray(kmax, dtype=np.int32)
        g_range = None if g_range is None else np.ascontiguousarray(g_range, dtype=np.int32).reshape(-1)
        t0_init = None if t0_init is None else np.ascontiguousarray(t0_init, dtype=np.float64)
        wave_id = None if wave_id is None else np.ascontiguousarray(wave_id, dtype=np.uint64)
        n_steps = None if n_steps is None else np.ascontiguousarray(n_steps, dtype=np.int32)
        zi, zo = (None, None)
        if z_init is not None:
            n_ch = (len(offsets) - 1) * self.cfg.n_chains
            if len(z_init) != n_ch:
                raise ValueError(f"z_init needs one list per chain ({n_ch})")
            zo = np.zeros(n_ch + 1, np.int64)
            zo[1:] = np.cumsum([len(z) for z in z_init])
            zi = np.ascontiguousarray(np.concatenate([np.asarray(z, np.int32).reshape(-1) for z in z_init] +
                                                     [np.zeros(1, np.int32)]))
        keep = (offsets, lam, kmax, g_range, t0_init, wave_id, n_steps, zi, zo)
        b = fsmp_batch(len(offsets) - 1, ctypes.c_void_p(wave.data_ptr()), _hptr(offsets), _hptr(lam), _hptr(kmax),
                       _hptr(g_range), _hptr(t0_init), _hptr(wave_id), _hptr(n_steps), _hptr(zi), _hptr(zo))
        return b, keep

    def workspace_bytes(self, offsets, lam, kmax=None, g_range=None):
        """Device workspace fsmp_sample would hold for this batch (fsmp_workspace_bytes)."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        kmax = None if kmax is None else np.ascontiguousarray(kmax, dtype=np.int32)
        g_range = None if g_range is None else np.ascontiguousarray(g_range, dtype=np.int32).reshape(-1)
        b = fsmp_batch(len(offsets) - 1, None, _hptr(offsets), _hptr(lam), _hptr(kmax), _hptr(g_range), None, None,
                       None)
        return int(self.lib.fsmp_workspace_bytes(self.h, ctypes.byref(b)))

    def autotune_steps(self, wave, offsets, lam, kmax=None, pilot_steps=200, target_rel_mcse=0.02, min_steps=500,
                       max_steps=4000, stream=None):
        """Per-waveform sweep counts from a pilot run's batch-means MCSE of N (fsmp_autotune_steps)."""
        import torch
        b, keep = self._batch(wave, offsets, lam, kmax)
        steps = np.zeros(len(offsets) - 1, dtype=np.int32)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.fsmp_autotune_steps(self.h, ctypes.byref(b), pilot_steps, target_rel_mcse, min_steps,
                                                 max_steps, _hptr(steps), ctypes.c_void_p(st.cuda_stream)))
        return steps

    @staticmethod
    def _samples(out):
        return fsmp_samples(_dptr(out["n_pe"]), _dptr(out["t0"]), _dptr(out["z"]), _dptr(out["charge"]),
                            _dptr(out["acc"]), _dptr(out["nhist"]), _dptr(out["counts"]), _dptr(out["status"]),
                            _dptr(out["log"]), _dptr(out["trace"]), out["kz"], _dptr(out.get("work")),
                            _dptr(out.get("qdraw")), _dptr(out.get("zdraw")), _dptr(out.get("rec_steps")),
                            _dptr(out.get("occ")), _dptr(out.get("comp")))

    def lucy(self, wave, offsets, kmax=None, kz=None, n_iter=2000, threshold=0.1, margin=4, qhat=False,
             stream=None):
        """Initial state by deconvolution (fsmp_lucy): device tensors z [n, kz], n_pe, g_range [n, 2],
        t0, lambda, cut [n, 2] and optionally qhat (row i at offsets[i] + i (L_V - 1))."""
        import torch
        dev = torch.device("cuda", self.device)
        b, keep = self._batch(wave, offsets, np.zeros(len(offsets) - 1), kmax)
        n = int(b.n_wave)
        km = keep[2]
        if kz is None:
            kz = int(km.max()) if km is not None and n > 0 else self.cfg.k_max
        lv = self.support_samples()
        res = {
            "z": torch.empty((n, kz), dtype=torch.int32, device=dev),
            "n_pe": torch.empty(n, dtype=torch.int32, device=dev),
            "g_range": torch.empty((n, 2), dtype=torch.int32, device=dev),
            "t0": torch.empty(n, dtype=torch.float64, device=dev),
            "lambda": torch.empty(n, dtype=torch.float64, device=dev),
            "cut": torch.empty((n, 2), dtype=torch.int32, device=dev),
            "qhat": (torch.empty(int(keep[0][-1]) + n * (lv - 1), dtype=torch.float64, device=dev)
                     if qhat else None),
            "kz": kz,
        }
        o = fsmp_lucy_out(_dptr(res["z"]), _dptr(res["n_pe"]), _dptr(res["g_range"]), _dptr(res["t0"]),
                          _dptr(res["lambda"]), _dptr(res["cut"]), _dptr(res["qhat"]), kz)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.fsmp_lucy(self.h, ctypes.byref(b), n_iter, ctypes.c_double(threshold), margin,
                                       ctypes.byref(o), ctypes.c_void_p(st.cuda_stream)))
        return res

    def support_samples(self):
        """L_V, the SER support in samples."""
        return int(self.lib.fsmp_ser_support(self.h))

    @staticmethod
    def start_from(lucy_res, n_chains):
        """Host inputs of sample() from a fsmp_lucy result: z_init (one list per chain, the
        waveform's list for each of its chains), g_range, t0_init."""
        z = lucy_res["z"].cpu().numpy()
        n = lucy_res["n_pe"].cpu().numpy()
        lists = []
        for i in range(len(n)):
            zi = z[i, :n[i]].tolist()
            lists.extend([zi] * n_chains)
        return lists, lucy_res["g_range"].cpu().numpy(), lucy_res["t0"].cpu().numpy()

    def set_design(self, capacity, design):
        self._check(self.lib.fsmp_set_design(self.h, capacity, design))

    def get_design(self, capacity):
        return self.lib.fsmp_get_design(self.h, capacity)

    def autotune(self, wave, offsets, lam, kmax=None, trial_steps=50, stream=None, n_steps=None):
        """fsmp_autotune; n_steps: the per-waveform sweep counts the run will use, if any."""
        import torch
        b, keep = self._batch(wave, offsets, lam, kmax, n_steps=n_steps)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.fsmp_autotune(self.h, ctypes.byref(b), trial_steps, ctypes.c_void_p(st.cuda_stream)))
        return {c: self.get_design(c) for c in (16, 32, 48, 64, 96, 128, 160, 192)}

    def graph(self, wave, offsets, lam, kmax=None, out=None, kz=None, stream=None):
        """Capture the kernels of one sample() call into a HIP graph; returns (Graph, out)."""
        import torch
        b, keep = self._batch(wave, offsets, lam, kmax)
        if kz is None:
            kz = int(np.max(kmax)) if kmax is not None else self.cfg.k_max
        if out is None:
            out = self.alloc_samples(len(offsets) - 1, kz)
        s = self._samples(out)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = ctypes.c_void_p()
        self._check(self.lib.fsmp_graph_create(self.h, ctypes.byref(b), ctypes.byref(s), ctypes.c_void_p(st.cuda_stream),
                                               ctypes.byref(g)))
        return Graph(self, g, keep), out

    def replay(self, wave, offsets, lam, log, kmax=None, kz=None, stream=None, occupancy=False, z_init=None):
        """Follow recorded proposals (``log``: device uint8 [chains, n_steps * 40] or a structured
        host array [chains, n_steps] of LOGREC_DTYPE); returns (dnu, log_alpha, out) on the device."""
        import torch
        dev = torch.device("cuda", self.device)
        b, keep = self._batch(wave, offsets, lam, kmax, z_init=z_init)
        n = len(offsets) - 1
        if kz is None:
            kz = int(np.max(kmax)) if kmax is not None else self.cfg.k_max
        C = n * self.cfg.n_chains
        if isinstance(log, np.ndarray):
            rec = np.ascontiguousarray(log, dtype=LOGREC_DTYPE)
            if rec.shape != (C, self.cfg.n_steps):
                raise ValueError(f"log must be [{C}, {self.cfg.n_steps}] records")
            log = torch.from_numpy(rec.view(np.uint8).reshape(C, -1).copy()).to(dev)
        if not log.is_cuda or log.numel() != C * self.cfg.n_steps * LOGREC_DTYPE.itemsize:
            raise ValueError("log must hold one record per chain and step")
        out = self.alloc_samples(n, kz, occ_len=self.cfg.grid_sub * int(keep[0][-1]) if occupancy else 0)
        dnu = torch.zeros((C, self.cfg.n_steps), dtype=torch.float64, device=dev)
        la = torch.zeros((C, self.cfg.n_steps), dtype=torch.float64, device=dev)
        s = self._samples(out)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.fsmp_replay(self.h, ctypes.byref(b), ctypes.c_void_p(log.data_ptr()),
                                         ctypes.c_void_p(dnu.data_ptr()), ctypes.c_void_p(la.data_ptr()),
                                         ctypes.byref(s), ctypes.c_void_p(st.cuda_stream)))
        return dnu, la, out

    def sample(self, wave, offsets, lam, kmax=None, g_range=None, t0_init=None, wave_id=None, out=None, kz=None,
               stream=None, work=False, n_steps=None, occupancy=False, z_init=None, noalloc=False):
        """wave: torch float32 device tensor; offsets/lam/kmax/g_range/t0_init/wave_id/n_steps: host numpy
        arrays (n_steps: sweeps per waveform, at most the configured n_steps).  occupancy: also count
        the PEs per grid point over the recorded sweeps (out["occ"]).  z_init: one initial PE list
        (grid indices) per chain, or None for the empty start.  noalloc: call fsmp_sample_noalloc
        (pass `out` to keep the call itself free of allocation)."""
        import torch
        b, keep = self._batch(wave, offsets, lam, kmax, g_range, t0_init, wave_id, n_steps, z_init)
        n = int(b.n_wave)
        kmax = keep[2]
        if kz is None:
            kz = int(kmax.max()) if kmax is not None and n > 0 else self.cfg.k_max
        if out is None:
            out = self.alloc_samples(n, kz, work=work,
                                     occ_len=self.cfg.grid_sub * int(keep[0][-1]) if occupancy and n > 0 else 0)
        s = self._samples(out)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = keep
        fn = self.lib.fsmp_sample_noalloc if noalloc else self.lib.fsmp_sample
        self._check(fn(self.h, ctypes.byref(b), ctypes.byref(s), ctypes.c_void_p(st.cuda_stream)))
        return out

    def posterior(self, n_wave, samples, with_pn=True, stream=None, offsets=None, diagnostics=False, lam=None):
        """Per-waveform summaries (fsmp_posterior); with the batch's offsets and sampled occupancy
        counts also the expected number of PEs per grid point ("occupancy"); with diagnostics the
        Gelman-Rubin R and the between-chain MCSE ("rhat", "mcse_chains"); with the batch's lambda0
        the estimates lambda-hat_FSMP and lambda-hat_Q ("lambda_hat")."""
        import torch
        dev = torch.device("cuda", self.device)
        kz = samples["kz"]
        res = {
            "mean": torch.zeros((n_wave, 3), dtype=torch.float64, device=dev),
            "var": torch.zeros((n_wave, 3), dtype=torch.float64, device=dev),
            "mcse": torch.zeros((n_wave, 3), dtype=torch.float64, device=dev),
            "p_n": torch.zeros((n_wave, kz + 1), dtype=torch.float64, device=dev) if with_pn else None,
            "accept": torch.zeros((n_wave, 4), dtype=torch.float64, device=dev),
            "status": torch.zeros(n_wave, dtype=torch.int32, device=dev),
            "occupancy": None,
            "rhat": torch.zeros((n_wave, 3), dtype=torch.float64, device=dev) if diagnostics else None,
            "mcse_chains": torch.zeros((n_wave, 3), dtype=torch.float64, device=dev) if diagnostics else None,
            "lambda_hat": torch.zeros((n_wave, 2), dtype=torch.float64, device=dev) if lam is not None else None,
        }
        hlam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        hoff = None
        if offsets is not None and samples.get("occ") is not None:
            hoff = np.ascontiguousarray(offsets, dtype=np.int64)
            res["occupancy"] = torch.zeros(self.cfg.grid_sub * int(hoff[-1]), dtype=torch.float64, device=dev)
        s = self._samples(samples)
        po = fsmp_posterior_out(_dptr(res["mean"]), _dptr(res["var"]), _dptr(res["mcse"]), _dptr(res["p_n"]),
                                _dptr(res["accept"]), _dptr(res["status"]), _dptr(res["occupancy"]), _hptr(hoff),
                                _dptr(res["rhat"]), _dptr(res["mcse_chains"]), _dptr(res["lambda_hat"]), _hptr(hlam))
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.fsmp_posterior(self.h, n_wave, ctypes.byref(s), ctypes.byref(po),
                                            ctypes.c_void_p(st.cuda_stream)))
        return res


def log_records(t):
    """View a device log tensor (uint8 [chains][n_steps*40]) as a numpy structured array."""
    a = t.cpu().numpy()
    return a.view(LOGREC_DTYPE).reshape(a.shape[0], -1)


class Server:
    """Continuous-batching request loop (fsmp_server_*): submit events from host memory,
    drive it with progress(), collect per-event posteriors and latencies."""

    def __init__(self, sampler_kwargs, n_streams=4, max_batch_wave=20000, memory_budget=8 << 30, device=0):
        self.lib = load()
        kw = dict(sampler_kwargs)
        ser = kw.get("ser", (8.0, 1.5, 6.0))
        self.ser = fsmp_ser(ser[0], ser[1], ser[2], kw.get("ser_amp", 1.0), kw.get("ser_support", 0))
        self.phi = fsmp_intensity(kw.get("phi_kind", FSMP_PHI_EXP), kw.get("tau_rise", 0.0), kw.get("tau_decay", 20.0),
                                  kw.get("t0_min", 50.0), kw.get("t0_max", 100.0))
        n_steps = kw.get("n_steps", 1000)
        burn = kw.get("burn_in", n_steps // 2)
        self.cfg = fsmp_config(kw.get("sigma_eps", 0.1), kw.get("mu_q", 1.0), kw.get("sigma_q", 0.3),
                               kw.get("grid_sub", 4), kw.get("jump_J", 0.25), kw.get("t0_step_sd", 1.0),
                               kw.get("shift_sd", 1.0), kw.get("k_max", 32), n_steps, kw.get("n_chains", 1), burn,
                               kw.get("thin", 1), kw.get("precision", FSMP_FP64), kw.get("refresh_M", 64), 0,
                               kw.get("seed", 0))
        self.scfg = fsmp_server_config(n_streams, max_batch_wave, memory_budget)
        h = ctypes.c_void_p()
        st = self.lib.fsmp_server_create(ctypes.byref(h), ctypes.byref(self.ser), ctypes.byref(self.phi),
                                         ctypes.byref(self.cfg), device, ctypes.byref(self.scfg))
        if st != FSMP_OK:
            raise FsmpError(st, self.lib.fsmp_server_last_error(None).decode())
        self.h = h
        self.sizes = {}

    def _check(self, st):
        if st < 0:
            raise FsmpError(st, self.lib.fsmp_server_last_error(self.h).decode())
        return st

    def submit(self, event_id, wave, offsets, lam, kmax=None):
        wave = np.ascontiguousarray(wave, dtype=np.float32)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        kmax = None if kmax is None else np.ascontiguousarray(kmax, dtype=np.int32)
        n = len(offsets) - 1
        self._check(self.lib.fsmp_server_submit(self.h, event_id, n, _hptr(wave), _hptr(offsets), _hptr(lam),
                                                _hptr(kmax)))
        self.sizes[event_id] = n

    def progress(self, wait=False):
        return self._check(self.lib.fsmp_server_progress(self.h, 1 if wait else 0))

    def result(self, event_id):
        n = self.sizes[event_id]
        mean = np.zeros((n, 3))
        mcse = np.zeros((n, 3))
        status = np.zeros(n, np.uint32)
        lat = ctypes.c_double(0.0)
        st = self.lib.fsmp_server_result(self.h, event_id, _hptr(mean), _hptr(mcse), _hptr(status), ctypes.byref(lat))
        if st == FSMP_EBUSY:
            return None
        self._check(st)
        del self.sizes[event_id]
        return {"mean": mean, "mcse": mcse, "status": status, "latency": lat.value}

    def stats(self):
        q, f, d, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        self._check(self.lib.fsmp_server_stats(self.h, ctypes.byref(q), ctypes.byref(f), ctypes.byref(d), ctypes.byref(b)))
        return {"queued": q.value, "in_flight": f.value, "done": d.value, "bytes_held": b.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.fsmp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured fsmp_sample launch sequence (fsmp_graph_*)."""

    def __init__(self, sampler, handle, keep):
        self.sampler, self.h, self._keep = sampler, handle, keep

    def launch(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.sampler.device)
        self.sampler._check(self.sampler.lib.fsmp_graph_launch(self.h, ctypes.c_void_p(st.cuda_stream)))

    def close(self):
        if getattr(self, "h", None):
            self.sampler.lib.fsmp_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
