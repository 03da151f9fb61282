"""Differentiation parity: the autograd Function's backward (re-solve, adjoint
multigrid solve, fused sensitivity kernel) against the oracle's adjoint
gradient, against central finite differences of the GPU compliance, and the
Euler identity sum psi dJ/dpsi = -J."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import oracle_solve, rel_l2, rel_max, say, solver_for, to_np

pytestmark = pytest.mark.gpu


def _small_cantilever():
    return si.cantilever_density_3d(24, 12, 12, n_fd=8)


def test_autograd_matches_oracle_adjoint():
    from paper_2212_02362_amd import SBMSolve, Solver
    p = random_problem_with_traction()
    S = Solver(p.ncell, p.h, rtol=1e-12, max_cycles=400)
    psi = torch.tensor(p.psi_raw, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(p.b, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor(np.random.default_rng(2).standard_normal((p.dim,) + p.node_shape),
                     dtype=torch.float64, device="cuda")
    say("autograd forward/backward")
    u = SBMSolve.apply(psi, b, S, p.lam, p.mu, p.psi_floor, p.kind, p.val)
    loss = (w * u).sum()
    loss.backward()
    # oracle: u, adjoint lam = K^-1 w (homogeneous), g = sensitivity, floor mask
    u_o, _, st = oracle_solve(p, rtol=1e-12, max_cycles=400)
    q = si.Problem(p.name, p.ncell, p.h, p.lam, p.mu, p.psi_floor, p.psi_raw, p.kind,
                   np.zeros_like(p.val), b=to_np(w))
    lam_o, _, _ = oracle_solve(q, rtol=1e-12, max_cycles=400)
    g_o = oracle.sensitivity(p.ncell, p.h, p.lam, p.mu, p.kind, p.val, u_o, lam_o)
    g_o = np.where(p.psi_raw > p.psi_floor, g_o, 0.0)
    assert rel_max(to_np(psi.grad), g_o) < 1e-8
    mask, _ = oracle.dirichlet(p.ncell, p.kind, p.val)
    assert rel_l2(to_np(b.grad)[mask == 0], lam_o[mask == 0]) < 1e-9
    assert (to_np(b.grad)[mask == 1] == 0).all()


def random_problem_with_traction():
    from _util import random_problem
    p = random_problem((12, 8, 10), seed=11, floor=1e-3, zero_frac=0.1)
    return p


def test_compliance_gradient_fd_and_euler():
    from paper_2212_02362_amd import compliance_grad
    p = _small_cantilever()
    S = solver_for(p, rtol=1e-12, max_cycles=400)
    say("compliance grad small")
    J, g, u = compliance_grad(S, p.rho, p, return_u=True)
    assert J > 0 and (to_np(g) <= 1e-14 * np.abs(to_np(g)).max()).all()
    # oracle gradient with the oracle's own solution
    u_o, _, _ = oracle_solve(p, rtol=1e-12, max_cycles=400)
    hd = np.prod(p.h)
    g_o = oracle.sensitivity(p.ncell, p.h, p.lam, p.mu, p.kind, p.val, u_o, hd * u_o, rho=p.rho,
                             psi_floor=p.psi_floor)
    assert rel_max(to_np(g), g_o) < 1e-8
    # Euler identity on psi (homogeneous degree one, f independent of psi)
    gpsi = to_np(S.sensitivity(u, u, lam_scale=hd))
    psi = np.maximum(p.rho ** 3, p.psi_floor)
    assert abs(np.sum(psi * gpsi) + J) < 1e-9 * J
    # central differences in correction form at the drawn cells
    _fd_check(S, p, to_np(g), u, p.fd_cells, step=1e-6)


def _fd_check(S, p, g, u, cells, step):
    """dJ/drho_c by central differences: for rho +- step e_c solve
    K(rho') w = f - K(rho') u from w = 0 (the RHS is O(step), so the solve's
    relative tolerance applies to the correction, not to u), then
    dJ = h^d f.(w+ - w-)."""
    errs = []
    for c in cells:
        idx = np.unravel_index(int(c), p.rho.shape)
        Js = []
        for sgn in (1.0, -1.0):
            rho = p.rho.copy()
            rho[idx] += sgn * step
            S.set_problem(rho, p.lam, p.mu, p.psi_floor, p.kind, p.val, p.b, density=True)
            r, _ = S.residual(u)
            w, hist, st = S.solve_rhs(r)
            Js.append(S.compliance(w))
        fd = (Js[0] - Js[1]) / (2 * step)
        errs.append(abs(fd - g[idx]))
    scale = np.abs(g).max()
    print(f"[fd] max abs err {max(errs):.3e}, max |g| {scale:.3e}")
    assert max(errs) <= 1e-6 * scale
