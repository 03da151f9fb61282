"""Full-solve parity with the FP64 oracle at sizes the oracle finishes in
seconds (the 2D plate with a void at its full 65x65 size, and reduced
versions of the 3D workloads).

Protocol: the oracle solves to a relative residual of 1e-10 in m* V-cycles;
the GPU runs exactly m* cycles (rtol 0, max_cycles m*) with the same options.
Bar: every residual of the history agrees to 1e-6 relative plus an absolute
1e-13, and the displacement to 1e-9 relative L2.  The absolute term is the
FP64 rounding floor of evaluating rho = ||f - K u|| / ||f||: each entry of
K u is a sum of O(20) stencil terms of size up to ~1e3 |f|, so summation
order alone moves rho by ~1e-15..1e-14 whatever the iterate; 1e-13 leaves a
decade of margin above the largest difference observed (5e-15).  The mixed-precision solve converges to the
same tolerance; its error against the FP64 oracle is reported and bounded."""
import numpy as np
import pytest

import sbm_inputs as si
from _util import oracle_solve, random_problem, rel_l2, say, solver_for, to_np

pytestmark = pytest.mark.gpu

RHO_ATOL = 1e-13  # rounding floor of the FP64 residual evaluation (module docstring)

CASES = {
    "plate_void_2d_64": lambda: si.plate_void_2d(64),
    "spherical_voids_16": lambda: si.spherical_voids_3d(16),
    "spherical_voids_32": lambda: si.spherical_voids_3d(32),
    "diffuse_crack_32": lambda: si.diffuse_crack_3d(32),
    "cantilever_24x12x12": lambda: si.cantilever_density_3d(24, 12, 12),
    "random_mixed_2d_40x24": lambda: random_problem((40, 24), seed=3),
    "random_mixed_3d_16x8x12": lambda: random_problem((16, 8, 12), seed=4, floor=1e-3),
    # 624-node bottom (LDS CG)
    "random_mixed_2d_50x46": lambda: random_problem((50, 46), seed=5, floor=1e-2),
    # odd cell counts: the grid is its own 1224-node bottom (global-memory CG)
    "random_mixed_2d_35x33": lambda: random_problem((35, 33), seed=7, floor=1e-2),
}


def _run_pair(p, smoother, **kw):
    """Oracle to rtol 1e-10 in m* iterations, then the GPU for exactly m*."""
    u_o, hist_o, st_o = oracle_solve(p, smoother=smoother, rtol=1e-10, max_cycles=400, **kw)
    assert st_o == 0, "oracle did not converge"
    m = len(hist_o) - 1
    S = solver_for(p, smoother=smoother, rtol=0.0, max_cycles=m, **kw)
    u_g, hist_g, st_g = S.solve()
    return S, u_o, hist_o, to_np(u_g), hist_g, st_g, m


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_fp64_trajectory_parity(case, smoother):
    p = CASES[case]()
    say("fp64 parity", case, "smoother", smoother)
    S, u_o, hist_o, u_g, hist_g, st_g, m = _run_pair(p, smoother)
    assert len(hist_g) == m + 1
    dh = np.abs(hist_g - hist_o)
    assert np.all(dh <= 1e-6 * hist_o + RHO_ATOL), dh.max()
    assert rel_l2(u_g, u_o) <= 1e-9, rel_l2(u_g, u_o)


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("case", ["plate_void_2d_64", "spherical_voids_32", "diffuse_crack_32",
                                  "cantilever_24x12x12", "random_mixed_2d_40x24"])
def test_krylov_trajectory_parity(case, smoother):
    """V-cycle-preconditioned flexible CG: same iterates as the oracle's."""
    p = CASES[case]()
    say("krylov parity", case, smoother)
    S, u_o, hist_o, u_g, hist_g, st_g, m = _run_pair(p, smoother, krylov=1)
    assert len(hist_g) == m + 1
    dh = np.abs(hist_g - hist_o)
    assert np.all(dh <= 1e-6 * hist_o + RHO_ATOL), dh.max()
    assert rel_l2(u_g, u_o) <= 1e-9, rel_l2(u_g, u_o)


@pytest.mark.parametrize("shape", ["208x32x16", "256x32x16 cubic"])
@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("krylov", [0, 1])
def test_wide_grid_first_iterations(krylov, fused, shape):
    """209 x 33 x 17 nodes: the finest level takes the LDS-tiled half-sweep
    (or, with fused_sweep, the one-launch two-colour sweep, also from zero in
    the preconditioner), residual and (Krylov) Apply; the first iterations
    follow the oracle's.  257 x 33 x 17 nodes with cubic cells: the last node
    column and row of the level in the edge tiles or the face blocks, and the
    kernels' 4-coefficient form."""
    cubic = shape.endswith("cubic")
    ncell = tuple(int(n) for n in shape.split()[0].split("x"))
    p = random_problem(ncell, seed=6, floor=1e-3, cubic=cubic)
    say("wide grid", krylov, fused, shape)
    u_o, hist_o, _ = oracle_solve(p, rtol=0.0, max_cycles=5, krylov=krylov)
    S = solver_for(p, rtol=0.0, max_cycles=5, krylov=krylov, fused_sweep=fused)
    u_g, hist_g, _ = S.solve()
    assert len(hist_g) == len(hist_o) == 6
    dh = np.abs(hist_g - hist_o)
    assert np.all(dh <= 1e-9 * hist_o + RHO_ATOL), dh.max()
    assert rel_l2(to_np(u_g), u_o) <= 1e-11, rel_l2(to_np(u_g), u_o)


@pytest.mark.parametrize("case", ["plate_void_2d_64", "spherical_voids_32", "cantilever_24x12x12",
                                  "random_mixed_3d_16x8x12", "random_mixed_2d_50x46",
                                  "random_mixed_2d_35x33"])
def test_mixed_precision_converges_to_fp64_solution(case):
    p = CASES[case]()
    say("mixed", case)
    u_o, hist_o, st_o = oracle_solve(p, rtol=1e-10, max_cycles=400)
    for krylov in (0, 1):
        S = solver_for(p, precision=1, rtol=1e-10, max_cycles=400, krylov=krylov)
        u_g, hist_g, st = S.solve()
        assert st == 0
        assert hist_g[-1] <= 1e-10
        err = rel_l2(to_np(u_g), u_o)
        print(f"[mixed] {case} krylov {krylov}: iterations {len(hist_g) - 1} (fp64 oracle "
              f"{len(hist_o) - 1}), rel L2 error vs FP64 oracle {err:.3e}")
        assert err <= 1e-7


@pytest.mark.parametrize("fused", [0, 1])
def test_wide_grid_trajectory_to_tolerance(fused):
    """The wide grid solved to 1e-10 by preconditioned CG in exactly the
    oracle's iteration count m*, FP64 (half-sweeps or fused sweeps), and the
    mixed solve to the same tolerance within 1e-7 of the FP64 oracle."""
    p = random_problem((208, 32, 16), seed=8, floor=1e-3)
    say("wide grid to tolerance", fused)
    u_o, hist_o, st_o = oracle_solve(p, rtol=1e-10, max_cycles=400, krylov=1)
    assert st_o == 0
    m = len(hist_o) - 1
    S = solver_for(p, rtol=0.0, max_cycles=m, krylov=1, fused_sweep=fused)
    u_g, hist_g, _ = S.solve()
    assert len(hist_g) == m + 1
    dh = np.abs(hist_g - hist_o)
    assert np.all(dh <= 1e-6 * hist_o + RHO_ATOL), dh.max()
    assert rel_l2(to_np(u_g), u_o) <= 1e-9, rel_l2(to_np(u_g), u_o)
    say("wide grid mixed", fused)
    Sm = solver_for(p, precision=1, rtol=1e-10, max_cycles=400, krylov=1, fused_sweep=fused)
    u_m, hist_m, st_m = Sm.solve()
    assert st_m == 0 and hist_m[-1] <= 1e-10
    assert rel_l2(to_np(u_m), u_o) <= 1e-7, rel_l2(to_np(u_m), u_o)


def test_warm_start_and_history():
    p = CASES["spherical_voids_16"]()
    S = solver_for(p, rtol=1e-10)
    say("warm start")
    u, hist, st = S.solve()
    assert st == 0 and hist[0] == pytest.approx(1.0, rel=1e-12)
    assert np.all(np.diff(np.log(hist)) < 0)
    u2, hist2, st2 = S.solve(u0=u)
    assert st2 == 0 and len(hist2) == 1 and hist2[0] <= 1e-10


def test_not_converged_and_diverged_statuses():
    from paper_2212_02362_amd import SbmError
    p = CASES["spherical_voids_16"]()
    S = solver_for(p, rtol=1e-10, max_cycles=2)
    say("not converged")
    u, hist, st = S.solve()
    assert st == 1 and len(hist) == 3
    # an over-relaxed Jacobi smoother amplifies the error: reported as divergence
    S.set_options(smoother=1, omega=1.95, max_cycles=200)
    say("diverged")
    with pytest.raises(SbmError) as ei:
        S.solve()
    assert ei.value.status == -5


@pytest.mark.parametrize("case", ["spherical_voids_16", "random_mixed_2d_40x24"])
def test_adjoint_solve_parity(case):
    """solve_rhs(g): K x = g on free DOF, x = 0 on displacement DOF, equals the
    oracle's solve with that load, homogeneous data and no traction."""
    p = CASES[case]()
    g = np.random.default_rng(3).standard_normal((p.dim,) + p.node_shape)
    q = si.Problem(p.name, p.ncell, p.h, p.lam, p.mu, p.psi_floor, p.psi_raw, p.kind,
                   np.zeros_like(p.val), b=g)
    u_o, hist_o, st_o = oracle_solve(q, rtol=1e-10, max_cycles=400)
    m = len(hist_o) - 1
    S = solver_for(p, rtol=0.0, max_cycles=m)
    say("adjoint", case)
    x, hist, st = S.solve_rhs(g)
    assert np.all(np.abs(hist - hist_o) <= 1e-6 * hist_o + RHO_ATOL)
    assert rel_l2(to_np(x), u_o) <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager(precision):
    """Captured V-cycles replayed from a HIP graph give bit-identical
    histories and solutions to kernel-by-kernel launches, across repeated
    solves with eager work (problem setup, norms, copies) in between; a timed
    solve afterwards (launch by launch) still agrees."""
    p = CASES["spherical_voids_32"]()
    say("graph vs eager", precision)
    S1 = solver_for(p, precision=precision, use_graphs=0, rtol=1e-10)
    S2 = solver_for(p, precision=precision, use_graphs=1, rtol=1e-10)
    u1, h1, _ = S1.solve()
    u1 = to_np(u1)
    for rep in range(3):
        S2.set_problem_from(p)
        if rep == 2:
            S2.profile(True)
        u2, h2, _ = S2.solve()
        assert np.array_equal(h2, h1), rep
        assert np.array_equal(to_np(u2), u1), rep
    prof = S2.profile_read()
    S2.profile(False)
    ncyc = len(h1) - 1
    captures, launches = S2.graph_info()
    assert S1.graph_info() == (0, 0)
    assert captures == 1 and launches == 2 * ncyc  # the timed solve runs launch by launch
    # V(2,2): 8 finest half-sweeps per cycle, the first of them made by the
    # convergence test's pass (FP64) or by the cast of its residual (mixed)
    per = 2 * 4 - 1
    assert prof["smooth"][1] == per * ncyc and prof["smooth"][0] > 0
    assert prof["bottom"][1] == ncyc
