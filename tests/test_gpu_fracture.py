"""Parity of the GPU phase-field fracture kernels (Sec. 3.2) with the FP64
oracle, through the C ABI.

Bars: the crack driving force updates H to 1e-12 relative (max norm; the
principal strains come from rotations that may round differently) and marks
the same intact cells (random strains: no ties); the Ginzburg-Landau step
agrees to 1e-12 relative in c and psi; a staggered Mode-I sequence (solve to
a 1e-10 residual, driving force, crack step, warm-started next solve) keeps c
within 1e-8 and H within 1e-7 relative L2 of the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import random_problem, rel_l2, rel_max, say, solver_for, to_np

pytestmark = pytest.mark.gpu

GRIDS = [(6, 5), (67, 45), (5, 4, 6), (17, 9, 13), (40, 33, 24)]


def _node_u(p, seed, scale=1e-3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((p.dim,) + p.node_shape) * scale


@pytest.mark.parametrize("ncell", GRIDS)
def test_crack_drive(ncell):
    p = random_problem(ncell, seed=11, body=False)
    S = solver_for(p)
    shape = tuple(reversed(ncell))
    u = _node_u(p, 12)
    rng = np.random.default_rng(13)
    # half of the cells start with a history above what this strain gives
    H0 = np.where(rng.uniform(size=shape) < 0.5, 0.0, 10.0 * p.mu * 1e-6)
    Href, iref = oracle.crack_drive(p.ncell, p.h, p.lam, p.mu, u, H0)
    say("crack drive", ncell)
    H, intact = S.crack_drive(u, H0)
    assert rel_max(to_np(H), Href) < 1e-12, rel_max(to_np(H), Href)
    assert np.array_equal(to_np(intact), iref)
    assert 0 < iref.sum() < iref.size
    Ht = torch.tensor(H0, device="cuda")
    out = S.crack_drive(u, Ht, inplace=True)
    assert out[0] is Ht and rel_max(to_np(Ht), Href) < 1e-12


@pytest.mark.parametrize("ncell", GRIDS)
def test_phase_step(ncell):
    p = random_problem(ncell, seed=14, body=False)
    S = solver_for(p)
    shape = tuple(reversed(ncell))
    rng = np.random.default_rng(15)
    c = rng.uniform(0.0, 1.0, shape)
    H = rng.uniform(0.0, 3.0, shape)
    intact = (rng.uniform(size=shape) < 0.2).astype(np.uint8)
    prm = dict(Gc=2.7, xi=2.0 * min(p.h), M=0.3, dt=1e-3 * min(p.h) ** 2, eta=1e-4)
    cref, psiref = oracle.phase_step(p.ncell, p.h, c, H, intact, **prm)
    say("phase step", ncell)
    c1, psi = S.phase_step(c, H, intact, **prm)
    assert rel_max(to_np(c1), cref) < 1e-12, rel_max(to_np(c1), cref)
    assert rel_max(to_np(psi), psiref) < 1e-12
    assert np.all(to_np(c1)[intact == 1] == 1.0)


def test_phase_step_errors():
    from paper_2212_02362_amd import SbmError, Solver
    p = random_problem((6, 5), seed=1, body=False)
    S = solver_for(p)
    c = torch.ones((5, 6), dtype=torch.float64, device="cuda")
    i8 = torch.zeros((5, 6), dtype=torch.uint8, device="cuda")
    say("phase step errors")
    with pytest.raises(SbmError):
        S.phase_step(c, c, i8, 1.0, 0.0, 1.0, 1.0)   # xi must be positive
    with pytest.raises(SbmError):
        S.phase_step(c, c, i8, 1.0, 0.1, 1.0, -1.0)  # dt must be non-negative
    with pytest.raises(ValueError):
        S.crack_drive(np.zeros((2, 5, 6)), c)        # u has the node shape (2, 6, 7)
    S2 = Solver((6, 5), (0.1, 0.1))
    with pytest.raises(SbmError) as ei:
        S2.crack_drive(np.zeros((2, 6, 7)), c)       # needs lambda, mu of a problem
    assert ei.value.status == -1


def _mode1():
    n = 64
    L = 0.02
    return si.pf_mode1_2d(n, L=L, notch=0.25 * L, xi=2.0 * L / n, uy=1.5e-5)


def _oracle_initial_psi(p):
    """psi = g(c0) + eta from the oracle's own crack step with dt = 0."""
    e = p.extra
    z = np.zeros_like(e["c0"])
    c, psi = oracle.phase_step(p.ncell, p.h, e["c0"], z, z.astype(np.uint8), e["Gc"], e["xi"],
                               e["M"], 0.0, e["eta"])
    assert np.array_equal(c, e["c0"])
    return psi


def _gpu_initial_psi(S, p):
    """psi = g(c0) + eta from the library's crack step with dt = 0."""
    e = p.extra
    c = torch.tensor(e["c0"], device="cuda")
    z = torch.zeros_like(c)
    c1, psi = S.phase_step(c, z, z.to(torch.uint8), e["Gc"], e["xi"], e["M"], 0.0, e["eta"])
    assert torch.equal(c1, c)
    return psi


def _stagger_oracle(p, nstep):
    e = p.extra
    c, H, psi, u = e["c0"].copy(), np.zeros_like(e["c0"]), _oracle_initial_psi(p), None
    small = []
    for _ in range(nstep):
        u, hist, st = oracle.solve(p.ncell, p.h, p.lam, p.mu, psi, p.psi_floor, p.kind, p.val,
                                   None, rtol=1e-10, u0=u)
        assert st == 0
        H, intact = oracle.crack_drive(p.ncell, p.h, p.lam, p.mu, u, H)
        c, psi = oracle.phase_step(p.ncell, p.h, c, H, intact, e["Gc"], e["xi"], e["M"], e["dt"],
                                   e["eta"])
        small.append(int((c < 0.5).sum()))
    return c, H, small


def test_staggered_mode1_sequence():
    """Solve, drive, crack step, next solve warm-started: the crack grows."""
    p = _mode1()
    e = p.extra
    nstep = 6
    c_o, H_o, small_o = _stagger_oracle(p, nstep)
    assert small_o[-1] > small_o[0], small_o           # the crack advances
    assert H_o.max() > e["Gc"] / (2.0 * e["xi"])         # above the growth threshold
    from paper_2212_02362_amd import Solver
    S = Solver(p.ncell, p.h)
    c = torch.tensor(e["c0"], device="cuda")
    H = torch.zeros_like(c)
    psi = _gpu_initial_psi(S, p)
    u = None
    small = []
    for k in range(nstep):
        say("staggered mode-I step", k)
        S.set_problem(psi, p.lam, p.mu, p.psi_floor, p.kind, p.val)
        u, hist, st = S.solve(u0=u)
        assert st == 0
        H, intact = S.crack_drive(u, H, inplace=True)
        c, psi = S.phase_step(c, H, intact, e["Gc"], e["xi"], e["M"], e["dt"], e["eta"])
        small.append(int((c < 0.5).sum().item()))
    assert all(abs(a - b) <= 1 for a, b in zip(small, small_o)), (small, small_o)
    assert rel_l2(to_np(c), c_o) < 1e-8, rel_l2(to_np(c), c_o)
    assert rel_l2(to_np(H), H_o) < 1e-7, rel_l2(to_np(H), H_o)


def test_phase_step_projection():
    """Steps that overshoot 0 or 1 land on the ends, as in the oracle."""
    p = random_problem((33, 17), seed=16, body=False)
    S = solver_for(p)
    shape = tuple(reversed(p.ncell))
    rng = np.random.default_rng(17)
    c = rng.uniform(-0.2, 1.2, shape)
    H = rng.uniform(0.0, 50.0, shape)
    intact = (rng.uniform(size=shape) < 0.1).astype(np.uint8)
    prm = dict(Gc=1.0, xi=0.1, M=1.0, dt=0.005, eta=1e-4)
    cref, psiref = oracle.phase_step(p.ncell, p.h, c, H, intact, **prm)
    assert (cref == 0.0).sum() > 10 and ((cref == 1.0) & (intact == 0)).sum() > 10
    say("phase step projection")
    out = (torch.full(shape, 7.0, dtype=torch.float64, device="cuda"),
           torch.full(shape, 7.0, dtype=torch.float64, device="cuda"))
    c1, psi = S.phase_step(c, H, intact, **prm, out=out)
    assert c1 is out[0] and psi is out[1]
    assert rel_max(to_np(c1), cref) < 1e-12 and rel_max(to_np(psi), psiref) < 1e-12
    assert np.array_equal(to_np(c1) == 0.0, cref == 0.0)


def test_fracture_calls_reject_aliased_buffers():
    import ctypes

    from paper_2212_02362_amd._lib import SbmPf, lib
    p = random_problem((6, 5), seed=2, body=False)
    S = solver_for(p)
    c = torch.full((5, 6), 0.5, dtype=torch.float64, device="cuda")
    H = torch.zeros_like(c)
    i8 = torch.zeros((5, 6), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(c)
    pf = SbmPf(1.0, 0.1, 1.0, 1e-3, 1e-4)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    say("phase step aliasing")
    for co, po in ((c, out), (out, c), (out, out), (H, out), (out, H)):
        st = lib().sbm_phase_step(S._ctx, P(c), P(H), P(i8), ctypes.byref(pf), P(co), P(po))
        assert st == -1
    say("crack drive aliasing")
    u = torch.zeros((2, 6, 7), dtype=torch.float64, device="cuda")
    for uu, hh, ii in ((u, u, i8), (u, H, u), (u, H, H)):
        assert lib().sbm_crack_drive(S._ctx, P(uu), P(hh), P(ii)) == -1
