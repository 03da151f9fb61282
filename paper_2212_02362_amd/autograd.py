"""Differentiable solve: ``SBMSolve`` (a torch.autograd.Function) and the
compliance gradient of the topology-optimisation workload (Sec. 3.3).

The backward pass stores no multigrid state.  It recomputes the forward
solution from the saved inputs, solves the adjoint problem K lam = dL/du with
the same multigrid (K is symmetric), and evaluates the fused per-cell
sensitivity dL/dpsi_c = -lam_c^T K_c u_c + lam^T df/dpsi_c in one kernel.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import CHAIN_FLOOR, CHAIN_RHO3
from .solver import Solver


class SBMSolve(torch.autograd.Function):
    """u = K(psi)^-1 f(psi, b).

    ``SBMSolve.apply(psi_raw, b, solver, lam, mu, psi_floor, kind, val)``
    returns the node displacement; gradients flow to ``psi_raw`` (through the
    floor: zero where psi_raw <= psi_floor) and to ``b`` (dL/db = lam on free
    DOF)."""

    @staticmethod
    def forward(ctx, psi_raw, b, solver: Solver, lam, mu, psi_floor, kind, val):
        solver.set_problem(psi_raw.detach(), lam, mu, psi_floor, kind, val,
                           None if b is None else b.detach())
        u, hist, st = solver.solve()
        ctx.solver = solver
        ctx.args = (lam, mu, psi_floor, kind, val)
        ctx.has_b = b is not None
        ctx.forward_hist = hist
        ctx.save_for_backward(psi_raw.detach(), b.detach() if b is not None else None)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        psi_raw, b = ctx.saved_tensors
        solver: Solver = ctx.solver
        lam_, mu, psi_floor, kind, val = ctx.args
        solver.set_problem(psi_raw, lam_, mu, psi_floor, kind, val, b)
        u, _, _ = solver.solve()                       # recomputed, not stored
        adj, _, _ = solver.solve_rhs(grad_u.contiguous())  # K lam = dL/du (symmetric K)
        g_psi = solver.sensitivity(u, adj, design=psi_raw, chain=CHAIN_FLOOR)
        g_b = adj if ctx.has_b else None
        return g_psi, g_b, None, None, None, None, None, None


def compliance_grad(solver: Solver, rho, problem, *, return_u=False):
    """J = h^d sum_free f.u and dJ/drho for psi = max(rho^3, floor).

    ``problem`` supplies the moduli, floor, boundary table and body force.
    With homogeneous displacement data the adjoint is lam = h^d u (compliance
    is self-adjoint) and no second solve is needed; otherwise the adjoint is
    solved with the same multigrid.  When traction loads are present J also
    depends on psi explicitly through f, and that term is added.
    Returns (J, dJ/drho[, u])."""
    kind = np.asarray(problem.kind)
    val = np.asarray(problem.val)
    d = solver.dim
    if np.any((kind[: 2 * d, :d] == 0) & (val[: 2 * d, :d] != 0.0)):
        raise NotImplementedError("compliance_grad covers body-force loads; use SBMSolve for "
                                  "traction loads")
    rho_t = torch.as_tensor(rho, dtype=torch.float64, device=solver.device).contiguous()
    solver.set_problem(rho_t, problem.lam, problem.mu, problem.psi_floor, problem.kind,
                       problem.val, problem.b, density=True)
    u, hist, st = solver.solve()
    J = solver.compliance(u)
    hd = float(np.prod(solver.h))
    if not np.any((kind[: 2 * d, :d] == 1) & (val[: 2 * d, :d] != 0.0)):
        # self-adjoint: lam = h^d u, and u is 0 on the displacement DOF
        g = solver.sensitivity(u, u, lam_scale=hd, design=rho_t, chain=CHAIN_RHO3)
    else:
        fA, _ = solver.rhs()
        adj, _, _ = solver.solve_rhs(fA)
        g = solver.sensitivity(u, adj, lam_scale=hd, design=rho_t, chain=CHAIN_RHO3)
    return (J, g, u) if return_u else (J, g)
