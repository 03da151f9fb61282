"""Pins of the oracle's multigrid pieces (transfers, smoothers, bottom CG,
V-cycle solve) and of its sensitivity, against dense linear algebra, exact
interpolation identities, the Kirsch solution and finite differences."""
import itertools

import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)


def _free_dense(ncell, h, psi, mask):
    K = oracle.assemble(ncell, h, LAM, MU, psi)
    free = mask.ravel() == 0
    return K, free


# ----------------------------------------------------------------- transfers

@pytest.mark.parametrize("ncc", [(3, 2), (2, 3, 2)])
def test_prolongation_reproduces_multilinear(ncc):
    d = len(ncc)
    ncf = tuple(2 * n for n in ncc)
    rng = np.random.default_rng(0)
    coef = rng.standard_normal((d, 2 ** d))

    def field(nc):
        X = si.node_coords(nc, (1.0,) * d)
        out = []
        for k in range(d):
            v = 0.0
            for t, bits in enumerate(itertools.product((0, 1), repeat=d)):
                term = coef[k, t]
                for a, bt in enumerate(bits):
                    if bt:
                        term = term * X[a]
                v = v + term
            out.append(v * np.ones_like(X[0]))
        return np.stack(out)

    ec = field(ncc)
    # fine coordinates measured in coarse units: x_f = n/2
    Xf = si.node_coords(ncf, (0.5,) * d)
    ef = []
    for k in range(d):
        v = 0.0
        for t, bits in enumerate(itertools.product((0, 1), repeat=d)):
            term = coef[k, t]
            for a, bt in enumerate(bits):
                if bt:
                    term = term * Xf[a]
            v = v + term
        ef.append(v * np.ones_like(Xf[0]))
    ef = np.stack(ef)
    mask = np.zeros(ef.shape, np.uint8)
    got = oracle.prolong_add(ncc, ec, mask, np.zeros_like(ef))
    assert np.abs(got - ef).max() < 1e-13 * np.abs(ef).max()


@pytest.mark.parametrize("ncf", [(6, 4), (4, 6, 4)])
def test_restriction_is_scaled_transpose(ncf):
    d = len(ncf)
    ncc = tuple(n // 2 for n in ncf)
    rng = np.random.default_rng(1)
    r = rng.standard_normal((d,) + tuple(n + 1 for n in reversed(ncf)))
    e = rng.standard_normal((d,) + tuple(n + 1 for n in reversed(ncc)))
    zf = np.zeros(r.shape, np.uint8)
    zc = np.zeros(e.shape, np.uint8)
    Rr = oracle.restrict(ncf, r, zc)
    Pe = oracle.prolong_add(ncc, e, zf, np.zeros_like(r))
    assert abs(np.vdot(Rr, e) * 2 ** d - np.vdot(r, Pe)) < 1e-12 * abs(np.vdot(r, Pe))
    const = np.ones_like(r)
    Rc = oracle.restrict(ncf, const, zc)
    inner = (slice(None),) + tuple(slice(1, -1) for _ in range(d))
    assert np.allclose(Rc[inner], 1.0, rtol=1e-15)
    # Dirichlet DOF of the coarse grid receive nothing
    zc2 = zc.copy()
    zc2[0, ...] = 1
    assert (oracle.restrict(ncf, r, zc2)[0] == 0).all()


def test_coarsen_psi_is_mean_of_children():
    psi = np.arange(4 * 6 * 8, dtype=float).reshape(4, 6, 8)
    c = oracle.coarsen_psi((8, 6, 4), psi)
    assert c.shape == (2, 3, 4)
    assert np.allclose(c, psi.reshape(2, 2, 3, 2, 4, 2).mean(axis=(1, 3, 5)))


# ----------------------------------------------------------------- smoothers

def _small_problem(ncell, seed=0):
    h = tuple(1.0 / n for n in ncell)
    psi, u, f = si.random_fields(ncell, seed=seed, psi_lo=1e-3)
    psi[psi < 0.1] = 1e-6
    kind, val = si.mixed_bc(len(ncell), seed=seed)
    mask, uD = oracle.dirichlet(ncell, kind, val)
    u[mask == 1] = uD[mask == 1]
    f[mask == 1] = 0.0
    return h, psi, u, f, mask


@pytest.mark.parametrize("ncell", [(5, 4), (3, 4, 3)])
def test_diagonal_matches_dense(ncell):
    h, psi, _, _, _ = _small_problem(ncell)
    K = oracle.assemble(ncell, h, LAM, MU, psi)
    assert np.allclose(oracle.diag(ncell, h, LAM, MU, psi).ravel(), np.diag(K), rtol=1e-13)


@pytest.mark.parametrize("ncell", [(5, 4), (3, 4, 3)])
def test_jacobi_and_rb_against_dense(ncell):
    """One damped-Jacobi sweep and one colour-synchronous half-sweep equal
    their definitions written with the dense matrix, and both fix the exact
    solution."""
    h, psi, u, f, mask = _small_problem(ncell, seed=2)
    K, free = _free_dense(ncell, h, psi, mask)
    D = np.diag(K)
    uf, ff = u.ravel(), f.ravel()
    r = np.where(free, ff - K @ uf, 0.0)
    w = 0.8
    jac = np.where(free, uf + w * r / D, uf)
    assert np.allclose(oracle.jacobi(ncell, h, LAM, MU, psi, mask, w, u, f).ravel(), jac,
                       rtol=1e-12, atol=1e-12 * np.abs(jac).max())
    idx = np.indices(tuple(reversed([n + 1 for n in ncell]))).sum(0) % 2
    colour = np.broadcast_to(idx, u.shape).ravel()
    for c in (0, 1):
        rb = np.where(free & (colour == c), uf + 1.0 * r / D, uf)
        got = oracle.rb_half(ncell, h, LAM, MU, psi, mask, 1.0, c, u, f).ravel()
        assert np.allclose(got, rb, rtol=1e-12, atol=1e-12 * np.abs(rb).max())
    # exact solution is a fixed point
    ustar = uf.copy()
    A = K[np.ix_(free, free)]
    rhs = ff[free] - K[np.ix_(free, ~free)] @ uf[~free]
    ustar[free] = np.linalg.solve(A, rhs)
    ustar = ustar.reshape(u.shape)
    for out in (oracle.jacobi(ncell, h, LAM, MU, psi, mask, w, ustar, f),
                oracle.rb_half(ncell, h, LAM, MU, psi, mask, 1.0, 0, ustar, f)):
        assert np.abs(out - ustar).max() < 1e-8 * np.abs(ustar).max()


def test_cg_matches_direct_solve():
    ncell = (3, 3, 2)
    h, psi, u, f, mask = _small_problem(ncell, seed=3)
    psi = np.maximum(psi, 0.05)
    K, free = _free_dense(ncell, h, psi, mask)
    x, it = oracle.cg(ncell, h, LAM, MU, psi, mask, f, rtol=1e-14)
    A = K[np.ix_(free, free)]
    ref = np.linalg.solve(A, f.ravel()[free])
    assert np.abs(x.ravel()[free] - ref).max() < 1e-10 * np.abs(ref).max()
    assert (x.ravel()[~free] == 0).all()
    assert it <= 4 * free.sum()


# --------------------------------------------------------------------- solve

@pytest.mark.parametrize("ncell,smoother,krylov", [((8, 8), 0, 0), ((16, 16), 0, 0),
                                                   ((16, 16), 1, 0), ((4, 4, 4), 0, 0),
                                                   ((8, 8, 8), 0, 0), ((8, 8, 8), 1, 0),
                                                   ((16, 16), 0, 1), ((8, 8, 8), 0, 1),
                                                   ((8, 8, 8), 1, 1)])
def test_vcycle_solve_matches_dense(ncell, smoother, krylov):
    """Multigrid solution (stationary V-cycles, or V-cycle-preconditioned
    flexible CG) equals the dense direct solution of the same discrete problem
    (random psi with floor cells, mixed boundary table)."""
    d = len(ncell)
    h = tuple(1.0 / n for n in ncell)
    rng = np.random.default_rng(11)
    psi = rng.uniform(0.05, 1.0, tuple(reversed(ncell)))
    psi[rng.uniform(size=psi.shape) < 0.15] = 0.0  # floored below
    floor = 1e-3
    kind, val = si.mixed_bc(d, seed=5)
    b = rng.standard_normal((d,) + tuple(n + 1 for n in reversed(ncell)))
    u, hist, st = oracle.solve(ncell, h, LAM, MU, psi, floor, kind, val, b,
                               smoother=smoother, rtol=1e-12, max_cycles=300, krylov=krylov)
    assert st == 0
    psi_f = np.maximum(psi, floor)
    mask, uD = oracle.dirichlet(ncell, kind, val)
    fA, fB, _ = oracle.rhs(ncell, h, LAM, MU, psi_f, kind, val, b)
    K, free = _free_dense(ncell, h, psi_f, mask)
    ref = uD.ravel().copy()
    ref[free] = np.linalg.solve(K[np.ix_(free, free)], fB.ravel()[free])
    cond = np.linalg.cond(K[np.ix_(free, free)])
    err = np.abs(u.ravel() - ref).max() / np.abs(ref).max()
    assert err < max(1e-9, cond * 1e-13), (err, cond)
    assert hist[-1] <= 1e-12
    if not krylov:  # geometric decrease of the stationary iteration's residual
        assert np.all(np.diff(np.log(hist[1:])) < 0)


def test_krylov_accelerates_near_singular_case():
    """On a diffuse crack in a 40 % void field the stationary V-cycle
    converges slowly; flexible CG preconditioned by the same V-cycle needs
    far fewer iterations to the same tolerance and reaches the same
    solution."""
    import sbm_inputs as si
    p = si.diffuse_crack_3d(16)
    args = (p.ncell, p.h, p.lam, p.mu, p.psi_raw, p.psi_floor, p.kind, p.val)
    u0, h0, s0 = oracle.solve(*args, rtol=1e-10, max_cycles=400)
    u1, h1, s1 = oracle.solve(*args, rtol=1e-10, max_cycles=400, krylov=1)
    assert s0 == 0 and s1 == 0
    assert len(h1) < 0.6 * len(h0), (len(h0), len(h1))
    assert np.linalg.norm(u1 - u0) <= 1e-6 * np.linalg.norm(u0)


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_psi_vcycle_contracts(dim):
    ncell = (32, 32) if dim == 2 else (16, 16, 16)
    h = tuple(1.0 / n for n in ncell)
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    kind[0, :] = oracle.DISPLACEMENT
    val[1, 0] = 1e-3
    u, hist, st = oracle.solve(ncell, h, LAM, MU, np.ones(tuple(reversed(ncell))), 0.0, kind, val,
                               rtol=1e-10, max_cycles=100)
    assert st == 0
    rate = (hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2))
    assert rate < 0.5, rate


@pytest.mark.slow
def test_kirsch_stress_concentration_trend():
    """Plate with a hole under remote uniaxial stress (Sec. 3.1): as the
    diffuse width shrinks (at fixed, fine grid), the hoop stress at the top of
    the hole approaches the Kirsch value 3 sigma and the L2 error of sigma_xx
    along the line y = a decreases."""
    sigma, a = 1e-3, 1.0
    errs, peaks = [], []
    for width in (1.0, 0.5, 0.25):
        p = si.kirsch_quarter_plate(n=256, width=width, sigma=sigma)
        u, hist, st = oracle.solve(p.ncell, p.h, p.lam, p.mu, p.psi_raw, p.psi_floor, p.kind, p.val,
                                   rtol=1e-9, max_cycles=400)
        assert st == 0
        h = p.h[0]
        ux, uy = u[0], u[1]
        # cell-centred strain from the four corner nodes
        exx = 0.5 * ((ux[:-1, 1:] - ux[:-1, :-1]) + (ux[1:, 1:] - ux[1:, :-1])) / h
        eyy = 0.5 * ((uy[1:, :-1] - uy[:-1, :-1]) + (uy[1:, 1:] - uy[:-1, 1:])) / h
        sxx = (p.lam + 2 * p.mu) * exx + p.lam * eyy
        Xc, Yc = si.cell_centres(p.ncell, p.h)
        row = int(round(a / h - 0.5))  # cells whose centre is nearest y = a
        x = Xc[row]
        sel = (x > 0) & (x < 4.0) & (p.psi_raw[row] > 0.5)
        r = np.hypot(x[sel], Yc[row][sel])
        th = np.arctan2(Yc[row][sel], x[sel])
        srr = sigma / 2 * (1 - a * a / r ** 2) + sigma / 2 * (1 - 4 * a * a / r ** 2 + 3 * a ** 4 / r ** 4) * np.cos(2 * th)
        stt = sigma / 2 * (1 + a * a / r ** 2) - sigma / 2 * (1 + 3 * a ** 4 / r ** 4) * np.cos(2 * th)
        srt = -sigma / 2 * (1 + 2 * a * a / r ** 2 - 3 * a ** 4 / r ** 4) * np.sin(2 * th)
        c, s = np.cos(th), np.sin(th)
        kxx = srr * c * c + stt * s * s - 2 * srt * s * c
        errs.append(np.linalg.norm(sxx[row][sel] - kxx) / np.linalg.norm(kxx))
        peaks.append(sxx[row][sel][0] / sigma)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.1, errs
    assert abs(peaks[2] - 3.0) < abs(peaks[0] - 3.0), peaks


# --------------------------------------------------------------- sensitivity

def _tiny_topopt(ncell=(4, 3, 3), seed=0, traction=False):
    d = len(ncell)
    h = tuple(1.0 / n for n in ncell)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.2, 1.0, tuple(reversed(ncell)))
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    kind[0, :] = oracle.DISPLACEMENT
    if traction:
        val[1, :d] = rng.uniform(-1, 1, d)
    b = rng.standard_normal((d,) + tuple(n + 1 for n in reversed(ncell)))
    return d, h, rho, kind, val, b


def _compliance(ncell, h, psi, kind, val, b):
    d = len(ncell)
    mask, uD = oracle.dirichlet(ncell, kind, val)
    fA, fB, _ = oracle.rhs(ncell, h, LAM, MU, psi, kind, val, b)
    K, free = _free_dense(ncell, h, psi, mask)
    u = uD.ravel().copy()
    u[free] = np.linalg.solve(K[np.ix_(free, free)], fB.ravel()[free])
    J = np.prod(h) * np.dot(fA.ravel()[free], u[free])
    return J, u.reshape((d,) + tuple(n + 1 for n in reversed(ncell))), fA


@pytest.mark.parametrize("traction", [False, True])
def test_sensitivity_fd_and_euler(traction):
    """dJ/dpsi for the compliance J = h^d f.u: central finite differences of
    dense solves, the Euler identity sum psi dJ/dpsi = -J (no traction, since
    then f does not depend on psi) and the sign dJ/dpsi <= 0."""
    ncell = (4, 3, 3)
    d, h, rho, kind, val, b = _tiny_topopt(ncell, traction=traction)
    psi = rho ** 3
    J, u, fA = _compliance(ncell, h, psi, kind, val, b)
    mask, _ = oracle.dirichlet(ncell, kind, val)
    adj = np.where(mask == 1, 0.0, np.prod(h) * u)  # compliance is self-adjoint
    g = oracle.sensitivity(ncell, h, LAM, MU, kind, val, u, adj)
    fd = np.zeros_like(g)
    step = 1e-6
    for c in itertools.product(*[range(s) for s in psi.shape]):
        pp, pm = psi.copy(), psi.copy()
        pp[c] += step
        pm[c] -= step
        fd[c] = (_compliance(ncell, h, pp, kind, val, b)[0] - _compliance(ncell, h, pm, kind, val, b)[0]) / (2 * step)
    # With a traction load f depends on psi, and J = h^d f(psi).u(psi) also
    # depends on psi explicitly: dJ = (adjoint formula with lam = h^d u) +
    # h^d u.df/dpsi.  The second term is the adjoint formula with zero moduli.
    if traction:
        g_src = oracle.sensitivity(ncell, h, 0.0, 0.0, kind, val, u, adj)
        g = g + g_src
    assert np.abs(g - fd).max() < 1e-6 * np.abs(fd).max()
    if not traction:
        assert abs(np.sum(psi * g) + J) < 1e-12 * abs(J)
        assert (g <= 1e-15 * np.abs(g).max()).all()


def test_sensitivity_dense_and_rho_chain():
    """-u^T (dK/dpsi_c) u with dK/dpsi_c assembled densely from a unit-cell psi,
    and the chain to rho for psi = max(rho^3, floor)."""
    ncell = (3, 3)
    d, h, rho, kind, val, b = _tiny_topopt(ncell, seed=4)
    rho[0, 0] = 0.01  # rho^3 below the floor
    u = np.random.default_rng(5).standard_normal((d, 4, 4))
    lam_adj = np.random.default_rng(6).standard_normal((d, 4, 4))
    mask, _ = oracle.dirichlet(ncell, kind, val)
    lam_adj[mask == 1] = 0.0
    g = oracle.sensitivity(ncell, h, LAM, MU, kind, val, u, lam_adj)
    for c in itertools.product(range(3), range(3)):
        e = np.zeros((3, 3))
        e[c] = 1.0
        dK = oracle.assemble(ncell, h, LAM, MU, e)
        assert abs(g[c] + lam_adj.ravel() @ dK @ u.ravel()) < 1e-12 * np.abs(g).max()
    floor = 1e-4
    gr = oracle.sensitivity(ncell, h, LAM, MU, kind, val, u, lam_adj, rho=rho, psi_floor=floor)
    expect = np.where(rho ** 3 > floor, 3 * rho ** 2 * g, 0.0)
    assert np.allclose(gr, expect, rtol=1e-14, atol=0)
    assert gr[0, 0] == 0.0
