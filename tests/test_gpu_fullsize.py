"""Parity at the full workload sizes, in the launch configuration the
benchmark times (default options, FP64 and mixed).  The oracle cannot run a
whole solve there in seconds, so the checks are properties it can evaluate:

* the oracle's own FP64 Apply of the GPU solution gives a relative residual
  within the tolerance (any size);
* Apply parity on the full grid;
* the first two V-cycles match the oracle's two cycles (129^3 only);
* at 129^3 the whole solve under the trajectory protocol: the oracle's solve
  to 1e-10 in m* V-cycles (about a minute and a half of the oracle on the
  host), the GPU for exactly m* cycles, every residual of the history to
  1e-6 relative plus 1e-13 and the displacement to 1e-9 relative L2;
* central differences of the GPU compliance at the 32 drawn cells of the
  193x97x97 density workload."""
import numpy as np
import pytest

import oracle
import sbm_inputs as si
from _util import oracle_solve, rel_l2, rel_max, say, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _oracle_rel_residual(p, u):
    psi = oracle.floor_psi(p.psi_raw, p.psi_floor)
    fA, fB, _ = oracle.rhs(p.ncell, p.h, p.lam, p.mu, psi, p.kind, p.val, p.b)
    mask, _ = oracle.dirichlet(p.ncell, p.kind, p.val)
    r = oracle.residual(p.ncell, p.h, p.lam, p.mu, psi, mask, u, fA)
    return np.linalg.norm(r) / np.linalg.norm(fB[mask == 0])


WORKLOADS = {
    "spherical_voids_129": lambda: si.spherical_voids_3d(128),
    "cantilever_193x97x97": lambda: si.cantilever_density_3d(),
    "diffuse_crack_257": lambda: si.diffuse_crack_3d(256),
}


# The 257^3 crack with 40 % voids converges too slowly for plain V-cycles
# (about 0.996 per cycle); it is solved by V-cycle-preconditioned CG.
KRYLOV = {"spherical_voids_129": 0, "cantilever_193x97x97": 0, "diffuse_crack_257": 1}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_solution_residual(name, precision):
    p = WORKLOADS[name]()
    say("full size", name, "precision", precision)
    S = solver_for(p, precision=precision, rtol=1e-10, max_cycles=400, krylov=KRYLOV[name])
    u, hist, st = S.solve()
    assert st == 0, hist[-5:]
    un = to_np(u)
    del u
    rho = _oracle_rel_residual(p, un)
    print(f"[fullsize] {name} precision {precision}: {len(hist) - 1} cycles, "
          f"GPU rho {hist[-1]:.3e}, oracle-evaluated rho {rho:.3e}")
    assert rho <= 1.05e-10


def test_fullsize_trajectory_parity_129():
    """Spherical voids at the full 129^3: exactly the oracle's m* V-cycles."""
    p = WORKLOADS["spherical_voids_129"]()
    say("full size 129 trajectory: oracle solve")
    u_o, hist_o, st_o = oracle_solve(p, rtol=1e-10, max_cycles=400)
    assert st_o == 0
    m = len(hist_o) - 1
    S = solver_for(p, rtol=0.0, max_cycles=m)
    say("full size 129 trajectory: GPU, m*", m)
    u_g, hist_g, _ = S.solve()
    assert len(hist_g) == m + 1
    dh = np.abs(np.asarray(hist_g) - np.asarray(hist_o))
    assert np.all(dh <= 1e-6 * np.asarray(hist_o) + 1e-13), dh.max()
    err = rel_l2(to_np(u_g), u_o)
    print(f"[fullsize] spherical_voids_129: m* = {m}, rel L2 vs oracle {err:.3e}")
    assert err <= 1e-9


def test_fullsize_apply_and_first_cycles_129():
    p = WORKLOADS["spherical_voids_129"]()
    S = solver_for(p, rtol=0.0, max_cycles=2)
    psi = oracle.floor_psi(p.psi_raw, p.psi_floor)
    u = np.random.default_rng(0).standard_normal((3,) + p.node_shape)
    say("full apply 129")
    assert rel_max(to_np(S.apply(u)), oracle.apply(p.ncell, p.h, p.lam, p.mu, psi, u)) < 1e-13
    say("two cycles 129")
    ug, hg, _ = S.solve()
    uo, ho, _ = oracle_solve(p, rtol=0.0, max_cycles=2)
    assert np.all(np.abs(hg - ho) <= 1e-9 * ho + 1e-13)
    assert rel_l2(to_np(ug), uo) <= 1e-11


def test_fullsize_compliance_fd_193():
    from paper_2212_02362_amd import compliance_grad
    from test_gpu_grad import _fd_check
    p = WORKLOADS["cantilever_193x97x97"]()
    S = solver_for(p, rtol=1e-10, max_cycles=400)
    say("compliance grad full size")
    J, g, u = compliance_grad(S, p.rho, p, return_u=True)
    _fd_check(S, p, to_np(g), u, p.fd_cells, step=1e-6)


_AMR = {}


def _amr_c4():
    """Base 64^3, 3 levels, 32^3-cell blocks, threshold 0.05, 10 ellipsoidal
    voids, floor 1e-5: the inputs and the oracle's setup (tags, blocks,
    classes, averaged psi, loads) at full size, built once."""
    if not _AMR:
        say("amr full size: generating inputs")
        p, psis = si.ellipsoidal_voids_amr(base=64, levels=3, block=32, seed=0)
        say("amr full size: oracle setup")
        m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val,
                              block=32, thresh=0.05)
        _AMR.update(p=p, psis=psis, m=m)
    return _AMR["p"], _AMR["psis"], _AMR["m"]


@pytest.mark.parametrize("precision", [0, 1])
def test_fullsize_amr_c4(precision):
    """Setup bit-exact against the oracle at full size; the GPU composite
    solution's composite residual, evaluated by the oracle, within the
    tolerance."""
    from paper_2212_02362_amd import AmrSolver
    p, psis, m = _amr_c4()
    say("amr full size: GPU setup, precision", precision)
    S = AmrSolver(p.ncell, p.h, 3, 32, precision=precision, rtol=1e-10, max_cycles=400)
    S.set_problem(psis, p.lam, p.mu, p.psi_floor, p.kind, p.val, thresh=0.05)
    for a in range(3):
        blk_o, cls_o, psi_o = m.info(a)
        blk_g, cls_g, psi_g = S.level_info(a)
        assert np.array_equal(to_np(psi_g), psi_o), a
        if a >= 1:
            assert np.array_equal(blk_g, blk_o), a
            assert np.array_equal(to_np(cls_g), cls_o), a
        del cls_g, psi_g
    dof, fnorm = S.stats()
    assert abs(fnorm - m.fnorm()) <= 1e-12 * m.fnorm()
    say("amr full size: GPU solve")
    u, hist, st = S.solve()
    assert st == 0, hist[-5:]
    un = [to_np(x) for x in u]
    del u
    say("amr full size: oracle composite residual of the GPU solution")
    _, nrm, _ = m.residual(un)
    rho = nrm / m.fnorm()
    print(f"[fullsize] amr C4 precision {precision}: {dof} composite DOF, {len(hist) - 1} cycles, "
          f"GPU rho {hist[-1]:.3e}, oracle-evaluated rho {rho:.3e}", flush=True)
    assert rho <= 1.05e-10
