"""Host-side checks of the C ABI that need no GPU: every function declared in
include/sbm.h is exported by libsbm.so and declared in the ctypes binding, and
the host-only entry points validate their arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2212_02362_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib


def test_header_functions_exported(L):
    names = _declared()
    assert len(names) >= 20
    so = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(so, n), f"{n} declared in sbm.h but not exported"
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_profile_classes_match_header(L):
    """The binding names one timing class per SBM_PROF_* constant, in the
    header's order (sbm_profile_read fills SBM_PROF_N entries)."""
    text = open(HEADER).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"\b(SBM_PROF_[A-Z0-9_]+)\s*=\s*(\d+)", text))
    n = consts.pop("SBM_PROF_N")
    assert len(L.PROF_CLASSES) == n
    assert sorted(consts.values()) == list(range(n))
    for k, v in consts.items():
        assert L.PROF_CLASSES[v] == k[len("SBM_PROF_"):].lower(), (k, L.PROF_CLASSES[v])


def test_options_defaults_and_levels(L):
    lib = L.lib()
    o = L.SbmOptions()
    lib.sbm_default_options(ctypes.byref(o))
    assert (o.smoother, o.nu_pre, o.nu_post, o.precision, o.max_cycles) == (0, 2, 2, 0, 200)
    assert o.rtol == 1e-10 and o.bottom_rtol == 1e-12
    g = L.SbmGrid()
    g.dim = 3
    for a, n in enumerate((192, 96, 96)):
        g.ncell[a] = n
        g.h[a] = 1 / 96
    assert lib.sbm_num_levels(ctypes.byref(g)) == 6  # (192,96,96) ... (6,3,3)
    g.ncell[0] = g.ncell[1] = g.ncell[2] = 256
    assert lib.sbm_num_levels(ctypes.byref(g)) == 8  # 256 ... 2
    assert lib.sbm_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) > 2 * 257 ** 3 * 3 * 8
    g.dim = 2
    g.ncell[0] = g.ncell[1] = 64
    assert lib.sbm_num_levels(ctypes.byref(g)) == 6
    g.ncell[0] = 63
    assert lib.sbm_num_levels(ctypes.byref(g)) == 1  # odd: the grid is its own bottom
    g.dim = 4
    assert lib.sbm_num_levels(ctypes.byref(g)) == 0
    assert lib.sbm_workspace_bytes(ctypes.byref(g), ctypes.byref(o)) == 0


def test_create_rejects_bad_arguments_without_device(L):
    lib = L.lib()
    o = L.SbmOptions()
    lib.sbm_default_options(ctypes.byref(o))
    g = L.SbmGrid()
    g.dim = 2
    g.ncell[0] = g.ncell[1] = 8
    g.h[0] = g.h[1] = 0.125
    ctx = ctypes.c_void_p()
    assert lib.sbm_create(ctypes.byref(g), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == -7
    assert b"workspace" in lib.sbm_last_error()
    assert lib.sbm_create(ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(256), 16, None,
                          ctypes.byref(ctx)) == -7
    g.h[0] = -1.0
    assert lib.sbm_create(ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(256), 1 << 40, None,
                          ctypes.byref(ctx)) == -2
    g.h[0] = 0.125
    o.smoother = 5
    assert lib.sbm_create(ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(256), 1 << 40, None,
                          ctypes.byref(ctx)) == -1
    assert lib.sbm_set_options(None, ctypes.byref(o)) == -1


def test_python_layer_holds_no_arithmetic():
    """The binding only marshals: no torch arithmetic on solver data."""
    pkg = os.path.join(ROOT, "paper_2212_02362_amd")
    for fn in ("solver.py", "autograd.py", "_lib.py"):
        src = open(os.path.join(pkg, fn)).read()
        for banned in ("torch.sum", "torch.where", ".sum(", "torch.matmul", "oracle"):
            assert banned not in src, (fn, banned)


def test_amr_layout_validation(L):
    """Adaptive layouts: block even and dividing twice the base cell count,
    1..4 levels; the workspace covers every dense level."""
    lib = L.lib()
    o = L.SbmOptions()
    lib.sbm_default_options(ctypes.byref(o))
    g = L.SbmGrid()
    g.dim = 3
    for a in range(3):
        g.ncell[a] = 64
        g.h[a] = 1 / 64
    ws = lib.sbm_amr_workspace_bytes(ctypes.byref(g), 3, 32, ctypes.byref(o))
    # level 2 alone: 257^3 nodes x 3 x (5 FP64 + 4 FP32 vectors)
    assert ws > 257 ** 3 * 3 * (5 * 8 + 4 * 4)
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 3, 31, ctypes.byref(o)) == 0
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 3, 48, ctypes.byref(o)) == 0
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 5, 32, ctypes.byref(o)) == 0
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 0, 32, ctypes.byref(o)) == 0
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 1, 32, ctypes.byref(o)) > 0
    g.dim = 2
    assert lib.sbm_amr_workspace_bytes(ctypes.byref(g), 3, 8, ctypes.byref(o)) > 0
