"""The model kernels at the benchmark's full sizes, on the states the
benchmark's steps produce: the oracle evaluates these pointwise kernels on
the whole grid in about a second, so they are compared element by element.

* Mode-I fracture, 4096^2 cells: after a warm-started solve of the specimen,
  the crack driving force and the crack step against the oracle on the GPU
  displacement (H to 1e-12 relative, identical intact cells, c and psi to
  1e-12), and the oracle's relative residual of that displacement below
  1.1e-10.
* J2 void tension, 128^3 cells: plastic load and radial return on a
  displacement from a solve past first yield (load to 1e-13, state to 1e-12,
  identical yield counts).
* Pressurised voids, 129^3 nodes: the diffuse traction load (1e-13) and the
  oracle's residual of the GPU solution loaded by it."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import rel_max, say, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _oracle_rel_residual(p, psi_raw, u, b=None):
    psi = oracle.floor_psi(psi_raw, p.psi_floor)
    fA, fB, _ = oracle.rhs(p.ncell, p.h, p.lam, p.mu, psi, p.kind, p.val, b)
    mask, _ = oracle.dirichlet(p.ncell, p.kind, p.val)
    r = oracle.residual(p.ncell, p.h, p.lam, p.mu, psi, mask, u, fA)
    return np.linalg.norm(r) / np.linalg.norm(fB[mask == 0])


def test_fracture_4096():
    from paper_2212_02362_amd import Solver
    p = si.pf_mode1_2d(4096)
    e = p.extra
    S = Solver(p.ncell, p.h, krylov=1, rtol=1e-10, max_cycles=400)
    say("full size fracture solve")
    # the initial indicator psi = g(c0) + eta, each side from its own crack
    # step with dt = 0
    c0 = torch.tensor(e["c0"], device="cuda")
    z = torch.zeros_like(c0)
    _, psi0 = S.phase_step(c0, z, z.to(torch.uint8), e["Gc"], e["xi"], e["M"], 0.0, e["eta"])
    zh = np.zeros_like(e["c0"])
    _, psi0_ref = oracle.phase_step(p.ncell, p.h, e["c0"], zh, zh.astype(np.uint8), e["Gc"],
                                    e["xi"], e["M"], 0.0, e["eta"])
    assert rel_max(to_np(psi0), psi0_ref) < 1e-14
    S.set_problem(psi0, p.lam, p.mu, p.psi_floor, p.kind, p.val)
    u, hist, st = S.solve()
    assert st == 0
    u_h = to_np(u)
    assert _oracle_rel_residual(p, psi0_ref, u_h) < 1.1e-10
    rng = np.random.default_rng(0)
    H0 = rng.uniform(0.0, 2.0 * e["Gc"] / (2.0 * e["xi"]), e["c0"].shape)
    say("full size crack drive / step")
    H, intact = S.crack_drive(u, H0)
    Href, iref = oracle.crack_drive(p.ncell, p.h, p.lam, p.mu, u_h, H0)
    assert rel_max(to_np(H), Href) < 1e-12
    assert np.array_equal(to_np(intact), iref)
    c1, psi1 = S.phase_step(e["c0"], H, intact, e["Gc"], e["xi"], e["M"], e["dt"], e["eta"])
    cref, psiref = oracle.phase_step(p.ncell, p.h, e["c0"], Href, iref, e["Gc"], e["xi"], e["M"],
                                     e["dt"], e["eta"])
    assert rel_max(to_np(c1), cref) < 1e-12 and rel_max(to_np(psi1), psiref) < 1e-12


def test_j2_128():
    from paper_2212_02362_amd import Solver
    p = si.j2_void_tension(128)
    j2 = p.extra
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=400)
    val = p.val.copy()
    val[1, 0] = 0.08                     # past first yield
    say("full size j2 solve")
    S.set_problem(p.psi_raw, p.lam, p.mu, p.psi_floor, p.kind, val)
    u, hist, st = S.solve()
    assert st == 0
    u_h = to_np(u)
    shape = tuple(reversed(p.ncell))
    rng = np.random.default_rng(1)
    ep = rng.standard_normal((6,) + shape) * 1e-4
    ep[:3] -= ep[:3].mean(axis=0, keepdims=True)
    al = np.abs(rng.standard_normal(shape)) * 1e-4
    bt = np.zeros((6,) + shape)
    say("full size plastic load / return")
    fp = to_np(S.plastic_source(ep))
    psi = oracle.floor_psi(p.psi_raw, p.psi_floor)
    fref = oracle.plastic_source(p.ncell, p.h, p.lam, p.mu, psi, ep)
    assert rel_max(fp, fref) < 1e-13
    got = S.return_map(u, ep, al, bt, j2["sigma_y"], j2["hbar"], j2["theta"])
    ref = oracle.return_map(p.ncell, p.h, p.lam, p.mu, j2["sigma_y"], j2["hbar"], j2["theta"],
                            u_h, ep, al, bt)
    assert got[3] == ref[3] and ref[3] > 0
    for a in range(3):
        assert rel_max(to_np(got[a]), ref[a]) < 1e-12


def test_pressurised_voids_129():
    from paper_2212_02362_amd import Solver
    p = si.pressurised_voids_3d(128)
    pr = p.extra["pressure"]
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=400)
    say("full size diffuse traction")
    b = S.diffuse_traction(p.psi_raw, p.psi_floor, pressure=pr)
    bref = oracle.diffuse_traction(p.ncell, p.h, p.psi_raw, p.psi_floor, pressure=pr)
    assert rel_max(to_np(b), bref) < 1e-13
    S.set_problem(p.psi_raw, p.lam, p.mu, p.psi_floor, p.kind, p.val, b)
    u, hist, st = S.solve()
    assert st == 0
    assert _oracle_rel_residual(p, p.psi_raw, to_np(u), bref) < 1.1e-10
