"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np

import oracle
import sbm_inputs as si


def say(*a):
    """Names the case before each GPU step, flushed, so a failing run says where it was."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def solver_for(p, **opts):
    from paper_2212_02362_amd import Solver
    S = Solver(p.ncell, p.h, **opts)
    S.set_problem_from(p)
    return S


def to_np(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def random_problem(ncell, seed=0, floor=1e-6, zero_frac=0.2, body=True, traction=True, cubic=False):
    """Random indicator with a fraction of empty cells, a mixed boundary table
    and a random body force; cells of slightly different sizes per axis, or
    cubic cells (the same spacing on every axis)."""
    rng = np.random.default_rng(seed)
    d = len(ncell)
    psi = rng.uniform(0.05, 1.0, tuple(reversed(ncell)))
    psi[rng.uniform(size=psi.shape) < zero_frac] = 0.0
    kind, val = si.mixed_bc(d, seed=seed)
    if not traction:
        val[kind == si.TRACTION] = 0.0
    b = rng.standard_normal((d,) + tuple(n + 1 for n in reversed(ncell))) if body else None
    h = (tuple(1.0 / max(ncell) for _ in ncell) if cubic else
         tuple(1.0 / n * (1.0 + 0.05 * a) for a, n in enumerate(ncell)))
    lam, mu = si.lame(1.0, 0.3)
    return si.Problem("random", tuple(ncell), h, lam, mu, floor, psi, kind, val, b=b)


def oracle_solve(p, **kw):
    return oracle.solve(p.ncell, p.h, p.lam, p.mu, p.psi_raw, p.psi_floor, p.kind, p.val, p.b, **kw)
