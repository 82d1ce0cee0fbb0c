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
    # plan calls without a plan, or with a replay mode that does not exist
    assert lib.digs_plan_set_replay(None, 0) == -1
    assert lib.digs_plan_get_replay(None, None) == -1
    assert lib.digs_plan_fwd(None, None) == -1 and lib.digs_plan_bwd(None, None) == -1
    with pytest.raises(ValueError):
        _lib.Plan.set_replay(object(), "sometimes")
    # a too-small workspace is rejected
    t = _lib.Tuning()
    t.capacity = 1000
    rc = lib.digs_project_fwd(ctypes.byref(G), ctypes.byref(R), ctypes.c_void_p(256), 10,
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              ctypes.c_void_p(256), 1, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              16, ctypes.byref(t), None)
    assert rc == -2
    # so is a workspace that is not 256-byte aligned, however large
    rc = lib.digs_project_fwd(ctypes.byref(G), ctypes.byref(R), ctypes.c_void_p(256), 10,
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              ctypes.c_void_p(256), 1, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(128),
                              1 << 40, ctypes.byref(t), None)
    assert rc == -2



def test_tile_shape_validation():
    """Tile shapes of one, two or four 8x8 blocks with edges 8, 16 or 32 are accepted, others
    rejected (workspace size 0), and a shape whose tiles exceed DIGS_MAX_TILES too."""
    from paper_2506_22280_amd import _lib, synth
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdigs.so is not built")
    p = synth.tiny()
    sizes = {}
    for tw, th in ((16, 16), (32, 8), (8, 32), (16, 8), (8, 16), (8, 8)):
        sizes[tw, th] = _lib.workspace_size(p.geom, p.grid, p.n, 4, dict(tile_w=tw, tile_h=th))
        assert sizes[tw, th] > 0, (tw, th)
    assert sizes[16, 16] == _lib.workspace_size(p.geom, p.grid, p.n, 4, None)
    for tw, th in ((32, 16), (16, 32), (32, 32), (4, 8), (8, 0), (0, 8), (24, 8), (64, 4)):
        assert _lib.workspace_size(p.geom, p.grid, p.n, 4, dict(tile_w=tw, tile_h=th)) == 0, \
            (tw, th)
    # 8x8 tiles of a 1024x768 detector are more than DIGS_MAX_TILES; 16x16 and 32x8 fit
    big = dict(p.geom, nu=1024, nv=768)
    assert _lib.workspace_size(big, p.grid, p.n, 4, dict(tile_w=8, tile_h=8)) == 0
    assert _lib.workspace_size(big, p.grid, p.n, 4, dict(tile_w=32, tile_h=8)) > 0
    assert _lib.workspace_size(big, p.grid, p.n, 4, None) > 0


def test_binding_rejects_mismatched_shapes():
    """The library indexes each buffer by the sizes passed beside it; the binding checks every
    tensor's shape against them first (host side, before any device call)."""
    import torch
    from paper_2506_22280_amd import _lib, synth
    p = synth.tiny(n=16, nviews=2, det=16)
    n, T, R = p.n, 2, p.grid["R"]
    good = dict(coef=torch.zeros(p.coef.shape), mu=torch.zeros(3, n), scale=torch.ones(3, n),
                quat=torch.zeros(4, n), rho=torch.zeros(n), angles=torch.zeros(T),
                w=torch.zeros(T, R))
    ws = _lib.Workspace(device="cpu")
    cases = [("scale", torch.ones(3, n - 1)), ("quat", torch.zeros(3, n)),
             ("rho", torch.zeros(n + 1)), ("w", torch.zeros(T, R + 1)),
             ("angles", torch.zeros(T, 1)), ("coef", torch.zeros(R, 8, 8, 7, 3))]
    for name, bad in cases:
        a = dict(good, **{name: bad})
        with pytest.raises(ValueError, match=name):
            _lib.project_fwd(p.geom, p.grid, a["coef"], a["mu"], a["scale"], a["quat"], a["rho"],
                             a["angles"], a["w"], ws)
    with pytest.raises(ValueError, match="grad_proj"):
        _lib.project_bwd(p.geom, p.grid, *good.values(), torch.zeros(T, 16, 15), ws)
    with pytest.raises(ValueError, match="proj"):
        _lib.project_fwd(p.geom, p.grid, *good.values(), ws, proj=torch.zeros(T + 1, 16, 16))
    with pytest.raises(ValueError, match="g_rho"):
        out = dict(g_mu=torch.zeros(3, n), g_scale=torch.zeros(3, n), g_quat=torch.zeros(4, n),
                   g_rho=torch.zeros(n - 1), g_coef=torch.zeros(p.coef.shape),
                   g_w=torch.zeros(T, R))
        _lib.project_bwd(p.geom, p.grid, *good.values(), torch.zeros(T, 16, 16), ws, out=out)
    with pytest.raises(ValueError, match="g_w"):
        bufs = dict(good, proj=torch.zeros(T, 16, 16), g_w=torch.zeros(T + 1, R))
        _lib.Plan(p.geom, p.grid, n, T, bufs)
    with pytest.raises(ValueError, match="v"):
        _lib.adam(torch.zeros(10), torch.zeros(10), torch.zeros(10), torch.zeros(9), 1e-3, 1)
