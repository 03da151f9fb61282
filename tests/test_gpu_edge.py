"""Degenerate problems through the C ABI against the FP64 oracle: a single
cell, a one-cell-thick 2D strip, two cells stacked in z, zero load (the
solve must return u = 0 at once), every face prescribed, and a box that is
all void (psi = floor everywhere).  Bars as for the solves: the same cycle
count and u to 1e-9 relative L2 (exactly 0 for the zero load)."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import rel_l2, say, to_np

pytestmark = pytest.mark.gpu

LAM, MU = si.lame(1.0, 0.3)


def _case(name):
    kind, val = si._bc_table()
    if name == "one_cell_3d":
        kind[4, :] = si.DISPLACEMENT
        val[5, 2] = 1e-3
        return (1, 1, 1), (0.5, 0.5, 0.5), np.ones((1, 1, 1)), 1e-6, kind, val
    if name == "strip_2d_7x1":
        kind[0, :] = si.DISPLACEMENT
        val[1, 0] = 2e-3
        return (7, 1), (0.1, 0.2), np.ones((1, 7)), 1e-6, kind, val
    if name == "two_cells_z":
        kind[4, :] = si.DISPLACEMENT
        val[5, 2] = 1e-3
        return (1, 1, 2), (0.5, 0.5, 0.5), np.ones((2, 1, 1)), 1e-6, kind, val
    if name == "zero_load_2d":
        kind[2, :] = si.DISPLACEMENT
        return (6, 5), (0.1, 0.1), np.ones((5, 6)), 1e-6, kind, val
    if name == "all_faces_prescribed_3d":
        kind[:, :] = si.DISPLACEMENT
        val[1, 0] = 1e-3
        val[3, 1] = -2e-3
        psi = np.random.default_rng(0).uniform(0.1, 1.0, (5, 3, 4))
        return (4, 3, 5), (0.2, 0.25, 0.2), psi, 1e-6, kind, val
    if name == "all_void_3d":
        kind[4, :] = si.DISPLACEMENT
        val[5, 2] = 1e-3
        return (8, 6, 10), (0.1, 0.1, 0.1), np.zeros((10, 6, 8)), 1e-4, kind, val
    raise KeyError(name)


NAMES = ["one_cell_3d", "strip_2d_7x1", "two_cells_z", "zero_load_2d", "all_faces_prescribed_3d",
         "all_void_3d"]


@pytest.mark.parametrize("name", NAMES)
def test_degenerate_problem(name):
    from paper_2212_02362_amd import Solver
    nc, h, psi, floor, kind, val = _case(name)
    u_o, h_o, st_o = oracle.solve(nc, h, LAM, MU, psi, floor, kind, val, None, rtol=1e-10)
    assert st_o == 0
    say("degenerate", name)
    S = Solver(nc, h)
    S.set_problem(psi, LAM, MU, floor, kind, val)
    u, hist, st = S.solve()
    assert st == 0 and len(hist) == len(h_o), (st, len(hist), len(h_o))
    if name == "zero_load_2d":
        assert not to_np(u).any()
    else:
        assert rel_l2(to_np(u), u_o) < 1e-9, rel_l2(to_np(u), u_o)


def test_aliased_buffers_rejected():
    """Every call that writes an output array rejects an output passed as
    one of its inputs (or as another output) with SBM_E_ARG before any
    launch; the context stays usable."""
    import ctypes

    from paper_2212_02362_amd import Solver
    from paper_2212_02362_amd._lib import SbmJ2, lib
    kind, val = si._bc_table()
    kind[4, :] = si.DISPLACEMENT
    val[5, 2] = 1e-3
    S = Solver((8, 8, 8), (0.1, 0.1, 0.1))  # two or more levels: restrict/prolong exist
    S.set_problem(np.ones((8, 8, 8)), LAM, MU, 1e-6, kind, val)
    assert S.nlevels >= 2
    say("aliased buffers")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    node = lambda: torch.zeros((3,) + S.node_shape, dtype=torch.float64, device="cuda")
    cell = lambda: torch.zeros(S.cell_shape, dtype=torch.float64, device="cuda")
    a, b = node(), node()
    ca = cell()
    ctx, L = S._ctx, lib()
    j2 = SbmJ2(1.0, 0.0, 1.0)
    eps = torch.zeros((6,) + S.cell_shape, dtype=torch.float64, device="cuda")
    calls = [
        lambda: L.sbm_apply(ctx, P(a), P(a)),
        lambda: L.sbm_residual(ctx, P(a), P(a), None),
        lambda: L.sbm_rhs(ctx, P(a), P(a)),
        lambda: L.sbm_sensitivity(ctx, P(a), P(b), 1.0, None, 0, P(a)),
        lambda: L.sbm_sensitivity(ctx, P(a), P(b), 1.0, None, 0, P(b)),
        lambda: L.sbm_plastic_source(ctx, P(eps), P(eps)),
        lambda: L.sbm_return_map(ctx, P(a), ctypes.byref(j2), P(eps), P(ca), P(ca), None),
        lambda: L.sbm_level_apply(ctx, 0, P(a), P(a)),
        lambda: L.sbm_level_smooth(ctx, 0, 0, 1.0, P(a), P(b), P(a)),
        lambda: L.sbm_level_smooth(ctx, 0, 0, 1.0, P(a), P(b), P(b)),
        lambda: L.sbm_level_residual(ctx, 0, P(a), P(b), P(a)),
        lambda: L.sbm_level_residual(ctx, 0, P(a), P(b), P(b)),
        lambda: L.sbm_level_restrict(ctx, 0, P(a), P(a)),
        lambda: L.sbm_level_prolong_add(ctx, 0, P(a), P(a)),
        lambda: L.sbm_bottom_solve(ctx, P(a), P(a), None),
    ]
    for k, call in enumerate(calls):
        assert call() == -1, k
        assert b"alias" in L.sbm_last_error(), (k, L.sbm_last_error())
    # distinct buffers still work on the same context
    assert L.sbm_apply(ctx, P(a), P(b)) == 0
    beta = torch.zeros_like(eps)  # 6 components per cell, as eps_p
    assert L.sbm_return_map(ctx, P(a), ctypes.byref(j2), P(eps), P(ca), P(beta), None) == 0
    torch.cuda.synchronize()
