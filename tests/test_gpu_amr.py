"""Parity of the GPU block-structured adaptive composite solve with the FP64
oracle (oracle.AmrProblem), through the C ABI.

Bars: block flags and node classes bit-exact (integer work; the tags are
taken in FP64 without contraction on both sides); floored and averaged-down
psi and ghost fill bit-exact (same operations in the same order, exact dyadic
weights); composite residual <= 1e-12 relative (different summation order of
the stencil); FP64 composite solves: the GPU runs exactly the oracle's cycle
count m* (the first cycle at a 1e-10 relative composite residual), every
residual of the history agrees to 1e-6 relative plus 1e-13 absolute (the
rounding floor of the residual evaluation) and the displacement to 1e-9
relative L2 on every level; the mixed solve reaches the same residual and
agrees to 1e-8.  The "wide3d" cases have a finest level 225 nodes wide and 33
deep, so its finest-level kernels run the LDS-tiled path over the list of
tiles that hold unknowns (with the ghost nodes outside them listed node by
node for the residual), the path of the 64^3 x 3 workload; in
"wide3d_sparse" some ghost faces lie in tiles without unknowns, which the
tiled passes never sweep."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import rel_l2, rel_max, say, to_np

pytestmark = pytest.mark.gpu

_CACHE = {}


def _case(name):
    """(base Problem, psi per level, block, explicit block flags or None)."""
    if name == "voids3d":
        p, psis = si.ellipsoidal_voids_amr(base=8, levels=3, block=4, seed=0)
        return p, psis, 4, None
    if name == "voids3d_partial":
        p, psis = si.ellipsoidal_voids_amr(base=8, levels=3, block=4, seed=1)
        b1 = np.zeros((4, 4, 4), np.uint8)
        b1[:2, 1:3, :3] = 1
        b1[3, 3, 3] = 1
        b2 = np.zeros((8, 8, 8), np.uint8)
        b2[1:3, 3:5, 1:5] = 1
        return p, psis, 4, [b1, b2]
    if name == "plate2d":
        p, psis = si.plate_void_amr_2d(base=16, levels=3, block=8)
        return p, psis, 8, None
    if name == "wide3d":
        # base 112 x 16 x 8 cells, two levels: the finest is 224 x 32 x 16
        # cells (225 x 33 x 17 nodes), wide enough for the tiled kernels
        p, psis = si.ellipsoidal_voids_amr(base=64, levels=2, block=8, seed=3, shape=(112, 16, 8))
        return p, psis, 8, None
    if name == "wide3d_sparse":
        # the same level with a few blocks: the block at cells x 56..64,
        # y 0..8 has its ghost faces x = 64 and y = 8 in the next tiles
        # (64 x 8 node columns), which hold no unknowns
        p, psis = si.ellipsoidal_voids_amr(base=64, levels=2, block=8, seed=3, shape=(112, 16, 8))
        b1 = np.zeros((2, 4, 28), np.uint8)
        b1[:, 0, 7] = 1
        b1[1, 2:4, 20:22] = 1
        return p, psis, 8, [b1]
    raise KeyError(name)


def _oracle(name, **opts):
    key = (name, tuple(sorted(opts.items())))
    if key not in _CACHE:
        p, psis, block, blocks = _case(name)
        _CACHE[key] = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind,
                                        p.val, block=block, blocks=blocks, **opts)
    return _CACHE[key]


def _oracle_solution(name, **opts):
    key = ("sol", name, tuple(sorted(opts.items())))
    if key not in _CACHE:
        m = _oracle(name, **opts)
        _CACHE[key] = m.solve(rtol=1e-10, max_cycles=200)
    return _CACHE[key]


def _gpu(name, **opts):
    from paper_2212_02362_amd import AmrSolver
    p, psis, block, blocks = _case(name)
    S = AmrSolver(p.ncell, p.h, len(psis), block, **opts)
    S.set_problem(psis, p.lam, p.mu, p.psi_floor, p.kind, p.val, blocks=blocks)
    return S


CASES = ["voids3d", "voids3d_partial", "plate2d", "wide3d", "wide3d_sparse"]
RHO_ATOL = 1e-13  # rounding floor of the composite residual evaluation


@pytest.mark.parametrize("name", CASES)
def test_setup_blocks_classes_psi(name):
    say("amr setup", name)
    m = _oracle(name)
    S = _gpu(name)
    levels = len(_case(name)[1])
    for a in range(levels):
        blk_o, cls_o, psi_o = m.info(a)
        blk_g, cls_g, psi_g = S.level_info(a)
        assert np.array_equal(to_np(psi_g), psi_o), a
        if a >= 1:
            assert np.array_equal(blk_g, blk_o), a
            assert np.array_equal(to_np(cls_g), cls_o), a
    # composite unknowns: class 1 (every node at the base), not covered by a
    # finer class-1 node, free DOF
    p = _case(name)[0]
    n = 0
    for a in range(levels):
        mask, _ = oracle.dirichlet(m.ncell(a), p.kind, p.val)
        use = np.ones(m.node_shape(a)[1:], bool) if a == 0 else (m.info(a)[1] == 1)
        if a + 1 < levels:
            cf = m.info(a + 1)[1]
            sl = tuple(slice(None, None, 2) for _ in range(m.dim))
            use &= cf[sl] != 1
        n += int(((mask == 0) & use[None]).sum())
    dof, fnorm = S.stats()
    assert dof == n
    assert abs(fnorm - m.fnorm()) <= 1e-12 * m.fnorm()


@pytest.mark.parametrize("name", CASES)
def test_ghost_fill(name):
    m = _oracle(name)
    S = _gpu(name)
    rng = np.random.default_rng(5)
    for a in range(1, len(_case(name)[1])):
        say("amr ghost", name, a)
        xc = rng.standard_normal(m.node_shape(a - 1))
        xf = rng.standard_normal(m.node_shape(a))
        got = to_np(S.ghost_fill(a, xc, xf))
        ref = m.ghost_fill(a, xc, xf)
        assert np.array_equal(got, ref), rel_max(got, ref)


@pytest.mark.parametrize("name", CASES)
def test_composite_residual(name):
    m = _oracle(name)
    S = _gpu(name)
    rng = np.random.default_rng(7)
    u = [rng.standard_normal(m.node_shape(a)) for a in range(len(_case(name)[1]))]
    say("amr residual", name)
    r_o, n_o, u_o = m.residual(u)
    r_g, n_g, u_g = S.residual(u)
    for a in range(len(u)):
        assert np.array_equal(to_np(u_g[a]), u_o[a]), a  # ghosts refilled identically
        assert rel_max(to_np(r_g[a]), r_o[a]) < 1e-12, a
    assert abs(n_g - n_o) <= 1e-12 * n_o
    # a level's r passed as its u is rejected before any launch
    import ctypes

    from paper_2212_02362_amd._lib import lib
    arr = (ctypes.c_void_p * len(u_g))(*[t.data_ptr() for t in u_g])
    assert lib().sbm_amr_residual(S._ctx, arr, arr, None) == -1
    assert b"alias" in lib().sbm_last_error()


@pytest.mark.parametrize("name", CASES)
def test_solve_parity_fp64(name):
    """Exactly the oracle's m* composite cycles, the whole residual history and
    every level's displacement."""
    u_o, h_o, st_o = _oracle_solution(name)
    assert st_o == 0
    m = len(h_o) - 1
    S = _gpu(name, rtol=0.0, max_cycles=m)
    say("amr solve fp64", name, "m*", m)
    u_g, h_g, st_g = S.solve()
    assert len(h_g) == m + 1, (len(h_g), m + 1)
    dh = np.abs(np.asarray(h_g) - np.asarray(h_o))
    assert np.all(dh <= 1e-6 * np.asarray(h_o) + RHO_ATOL), (dh.max(), h_g, h_o)
    assert h_g[-1] <= 1e-10
    for a in range(len(u_o)):
        assert rel_l2(to_np(u_g[a]), u_o[a]) < 1e-9, (a, rel_l2(to_np(u_g[a]), u_o[a]))
    # the returned solution satisfies the composite system
    _, nrm, _ = S.residual(u_g)
    assert nrm <= 1.01e-10 * S.stats()[1]


@pytest.mark.parametrize("name", ["wide3d", "wide3d_sparse"])
def test_wide_case_takes_the_tiled_path(name):
    """The wide cases' finest level passes the tiled kernels' size test
    (more than 192 nodes in x, more than 24 in y) and has inactive tiles; the
    sparse one has 64 x 8 node columns with ghost nodes and no unknown, so
    whatever its z chunks, the smoother's tile list leaves ghosts out."""
    p, psis, block, _ = _case(name)
    nz, ny, nx = psis[-1].shape
    assert nx + 1 > 192 and ny + 1 > 24
    m = _oracle(name)
    blk, cls, _ = m.info(1)
    assert 0 < blk.mean() < 1, blk.mean()
    ghost_only = 0
    for y0 in range(0, cls.shape[1], 8):
        for x0 in range(0, cls.shape[2], 64):
            col = cls[:, y0:y0 + 8, x0:x0 + 64]
            ghost_only += int((col >= 2).any() and not (col == 1).any())
    assert (ghost_only > 0) == (name == "wide3d_sparse"), ghost_only


def test_solve_parity_jacobi_trajectory():
    """Damped-Jacobi smoothing: the first cycles follow the oracle's."""
    name = "voids3d_partial"
    m = _oracle(name, smoother=1)
    u_o, h_o, _ = m.solve(rtol=0.0, max_cycles=6)
    S = _gpu(name, smoother=1, max_cycles=6, rtol=0.0)
    say("amr solve jacobi", name)
    u_g, h_g, st = S.solve()
    assert len(h_g) == len(h_o) == 7
    assert np.allclose(h_g, h_o, rtol=1e-9, atol=0), (h_g, h_o)
    for a in range(len(u_o)):
        assert rel_l2(to_np(u_g[a]), u_o[a]) < 1e-11, a


@pytest.mark.parametrize("name", ["voids3d", "plate2d", "wide3d_sparse"])
def test_solve_mixed(name):
    u_o, h_o, _ = _oracle_solution(name)
    S = _gpu(name, precision=1)
    say("amr solve mixed", name)
    u_g, h_g, st = S.solve()
    assert st == 0 and h_g[-1] <= 1e-10
    assert len(h_g) <= len(h_o) + 3, (len(h_g), len(h_o))
    for a in range(len(u_o)):
        err = rel_l2(to_np(u_g[a]), u_o[a])
        say("mixed level", a, "rel L2 vs FP64 oracle", err)
        assert err < 1e-8, (a, err)


def test_midsize_first_cycle():
    """Base 64^3 with a 129^3-node finest level (32^3-cell blocks, 56 % of
    them active): the first composite cycle follows the oracle's."""
    from paper_2212_02362_amd import AmrSolver
    p, psis = si.ellipsoidal_voids_amr(base=64, levels=2, block=32, seed=4)
    m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=32)
    say("amr mid-size: oracle cycle")
    u_o, h_o, _ = m.solve(rtol=0.0, max_cycles=1)
    for prec in (0, 1):
        S = AmrSolver(p.ncell, p.h, 2, 32, max_cycles=1, rtol=0.0, precision=prec)
        S.set_problem(psis, p.lam, p.mu, p.psi_floor, p.kind, p.val)
        say("amr mid-size: GPU cycle, precision", prec)
        u_g, h_g, _ = S.solve()
        tol = 1e-11 if prec == 0 else 1e-5
        assert np.allclose(h_g, h_o, rtol=tol, atol=0), (h_g, h_o)
        for a in range(2):
            assert rel_l2(to_np(u_g[a]), u_o[a]) < tol, (prec, a, rel_l2(to_np(u_g[a]), u_o[a]))


def test_full_coverage_matches_uniform_fine_solve():
    """A refined level covering the whole box: the composite solve reproduces
    the uniform solve of the fine grid cycle by cycle."""
    from paper_2212_02362_amd import AmrSolver, Solver
    p, psis = si.ellipsoidal_voids_amr(base=8, levels=2, block=8, seed=2)
    S = AmrSolver(p.ncell, p.h, 2, 8)
    S.set_problem(psis, p.lam, p.mu, p.psi_floor, p.kind, p.val, blocks=[np.ones((2, 2, 2), np.uint8)])
    say("amr full coverage")
    u_a, h_a, st_a = S.solve()
    U = Solver((16, 16, 16), tuple(x / 2 for x in p.h))
    U.set_problem(psis[1], p.lam, p.mu, p.psi_floor, p.kind, p.val)
    u_u, h_u, st_u = U.solve()
    assert st_a == 0 and st_u == 0
    assert len(h_a) == len(h_u)
    assert np.allclose(h_a, h_u, rtol=1e-7, atol=0)
    assert rel_l2(to_np(u_a[1]), to_np(u_u)) < 1e-10


def test_errors():
    from paper_2212_02362_amd import AmrSolver, SbmError
    say("amr errors")
    with pytest.raises(SbmError):
        AmrSolver((8, 8, 8), (1 / 8,) * 3, 3, 3)  # odd block
    with pytest.raises(SbmError):
        AmrSolver((8, 8, 8), (1 / 8,) * 3, 3, 4, krylov=1)
    S = AmrSolver((8, 8, 8), (1 / 8,) * 3, 2, 4)
    with pytest.raises(SbmError):
        S.solve()
    p, psis = si.ellipsoidal_voids_amr(base=8, levels=2, block=4, seed=0)
    bad = [x.copy() for x in psis]
    bad[1][0, 0, 0] = np.nan
    with pytest.raises(SbmError) as ei:
        S.set_problem(bad, p.lam, p.mu, p.psi_floor, p.kind, p.val)
    assert ei.value.status == -4
