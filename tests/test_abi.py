"""The C-ABI library loads and exports every entry point include/digs.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(digs_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for must in ("digs_ffd_eval", "digs_deform_gaussians", "digs_project_fwd",
                 "digs_project_bwd", "digs_workspace_size"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2506_22280_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdigs.so is not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_validation_and_sizes():
    """Argument checks and workspace sizing run on the host: no GPU needed."""
    from paper_2506_22280_amd import _lib, synth
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdigs.so is not built")
    lib = _lib.load()
    p = synth.tiny()
    G, R = _lib.make_geom(p.geom), _lib.make_grid(p.grid)
    s1 = lib.digs_workspace_size(ctypes.byref(G), ctypes.byref(R), 4096, 16, None)
    s2 = lib.digs_workspace_size(ctypes.byref(G), ctypes.byref(R), 8192, 16, None)
    assert 0 < s1 < s2 and s1 % 256 == 0
    bad = _lib.make_grid(dict(p.grid, R=9))
    assert lib.digs_workspace_size(ctypes.byref(G), ctypes.byref(bad), 10, 1, None) == 0
    bad_geom = _lib.make_geom(dict(p.geom, sdd=500.0))          # detector inside the orbit
    assert lib.digs_workspace_size(ctypes.byref(bad_geom), ctypes.byref(R), 10, 1, None) == 0
    huge = _lib.make_geom(dict(p.geom, nu=2048, nv=2048))        # more than 4096 tiles
    assert lib.digs_workspace_size(ctypes.byref(huge), ctypes.byref(R), 10, 1, None) == 0
    ewa = _lib.make_geom(dict(p.geom, model="ewa"))               # the EWA model: same layout
    assert lib.digs_workspace_size(ctypes.byref(ewa), ctypes.byref(R), 4096, 16, None) == s1
    ewa.model = 7                                                 # no such model
    assert lib.digs_workspace_size(ctypes.byref(ewa), ctypes.byref(R), 10, 1, None) == 0
    # a list entry holds the Gaussian's index in 24 bits
    assert lib.digs_workspace_size(ctypes.byref(G), ctypes.byref(R), (1 << 24) - 1, 1, None) > 0
    assert lib.digs_workspace_size(ctypes.byref(G), ctypes.byref(R), 1 << 24, 1, None) == 0
    # null pointers are rejected before any device work
    rc = lib.digs_project_fwd(ctypes.byref(G), ctypes.byref(R), None, 10, None, None, None, None,
                              1, None, None, None, None, 0, None, None)
    assert rc == -1
    assert lib.digs_strerror(-2) == b"workspace missing, misaligned or too small"
    # a too-small workspace is rejected
    t = _lib.Tuning()
    t.capacity = 1000
    rc = lib.digs_project_fwd(ctypes.byref(G), ctypes.byref(R), ctypes.c_void_p(256), 10,
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              ctypes.c_void_p(256), 1, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              16, ctypes.byref(t), None)
    assert rc == -2
