"""The C ABI library loads and exports every symbol include/fsmp.h declares; argument
validation answers before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2403_03156_amd import fsmp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fsmp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(fsmp_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported():
    if not os.path.exists(fsmp.LIB_PATH):
        pytest.skip("libfsmp.so not built")
    lib = ctypes.CDLL(fsmp.LIB_PATH)
    names = _declared()
    assert {"fsmp_create", "fsmp_sample", "fsmp_posterior", "fsmp_destroy", "fsmp_last_error"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(fsmp.EXPORTS) <= set(names)


def test_version_and_validation_without_device():
    if not os.path.exists(fsmp.LIB_PATH):
        pytest.skip("libfsmp.so not built")
    L = fsmp.load()
    assert L.fsmp_version().decode().startswith("fsmp")
    ser = fsmp.fsmp_ser(8.0, 1.5, 6.0, 1.0, 0)
    phi = fsmp.fsmp_intensity(fsmp.FSMP_PHI_EXP, 0.0, 20.0, 50.0, 100.0)
    cfg = fsmp.fsmp_config(0.1, 1.0, 0.3, 4, 0.25, 1.0, 1.0, 32, 100, 1, 50, 1, 0, 64, 0, 0)
    bad = [
        ("sigma", fsmp.fsmp_ser(8.0, -1.0, 6.0, 1.0, 0), phi, cfg),
        ("phi kind", ser, fsmp.fsmp_intensity(7, 0.0, 20.0, 50.0, 100.0), cfg),
        ("t0 range", ser, fsmp.fsmp_intensity(0, 0.0, 20.0, 100.0, 50.0), cfg),
        ("rise", ser, fsmp.fsmp_intensity(fsmp.FSMP_PHI_BIEXP, 0.0, 20.0, 50.0, 100.0), cfg),
        ("burn-in", ser, phi, fsmp.fsmp_config(0.1, 1.0, 0.3, 4, 0.25, 1.0, 1.0, 32, 100, 1, 200, 1, 0, 64, 0, 0)),
        ("J", ser, phi, fsmp.fsmp_config(0.1, 1.0, 0.3, 4, 0.6, 1.0, 1.0, 32, 100, 1, 50, 1, 0, 64, 0, 0)),
        ("kmax", ser, phi, fsmp.fsmp_config(0.1, 1.0, 0.3, 4, 0.25, 1.0, 1.0, 500, 100, 1, 50, 1, 0, 64, 0, 0)),
        ("grid", ser, phi, fsmp.fsmp_config(0.1, 1.0, 0.3, 0, 0.25, 1.0, 1.0, 32, 100, 1, 50, 1, 0, 64, 0, 0)),
        ("noise", ser, phi, fsmp.fsmp_config(0.0, 1.0, 0.3, 4, 0.25, 1.0, 1.0, 32, 100, 1, 50, 1, 0, 64, 0, 0)),
    ]
    for name, s, p, c in bad:
        h = ctypes.c_void_p()
        st = L.fsmp_create(ctypes.byref(h), ctypes.byref(s), ctypes.byref(p), ctypes.byref(c), 0)
        assert st == fsmp.FSMP_EINVAL, name
        assert not h.value
        assert len(L.fsmp_last_error(None)) > 5
    # a null context is rejected without crashing
    assert L.fsmp_sample(None, None, None, None) == fsmp.FSMP_EINVAL
    assert L.fsmp_posterior(None, 0, None, None, None) == fsmp.FSMP_EINVAL
    L.fsmp_destroy(None)
