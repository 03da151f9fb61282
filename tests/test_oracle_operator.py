"""Pins of the oracle's operator K and load f against facts fixed outside it.

Each test checks the oracle (``oracle/``) against the continuum equation, a
textbook stencil, the paper's 1D operator, an exact elastic solution or an
algebraic invariant -- never against a retyped copy of its own formula.
"""
import itertools

import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)


def _nodes(ncell, h):
    return si.node_coords(ncell, h)


def _cells(ncell, h):
    return si.cell_centres(ncell, h)


def _interior(ncell, margin=1):
    """Boolean node mask of nodes whose whole 3^d neighbourhood is inside."""
    shp = tuple(n + 1 for n in reversed(ncell))
    m = np.zeros(shp, bool)
    m[tuple(slice(margin, s - margin) for s in shp)] = True
    return m


def _C(lam, mu, d):
    I = np.eye(d)
    return (lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))


@pytest.mark.parametrize("ncell", [(7, 6), (5, 6, 4)])
@pytest.mark.parametrize("psi_kind", ["constant", "linear"])
def test_quadratic_exact(ncell, psi_kind):
    """Eq. K is exact for quadratic u with constant or linear psi: compare with
    the continuum -div(psi C grad u) evaluated analytically at interior nodes."""
    d = len(ncell)
    h = tuple(1.0 / n * (1 + 0.1 * a) for a, n in enumerate(ncell))  # anisotropic spacing
    rng = np.random.default_rng(3)
    a0 = rng.standard_normal(d)
    B = rng.standard_normal((d, d))
    Q = rng.standard_normal((d, d, d))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))  # u_k = a_k + B_k.x + x.Q_k.x
    psi0 = 0.7
    gpsi = rng.uniform(-0.3, 0.3, d) if psi_kind == "linear" else np.zeros(d)
    Xc = _cells(ncell, h)
    psi = psi0 + sum(gpsi[a] * Xc[a] for a in range(d))
    Xn = _nodes(ncell, h)
    u = np.stack([a0[k] + sum(B[k, l] * Xn[l] for l in range(d))
                  + sum(Q[k, l, m] * Xn[l] * Xn[m] for l in range(d) for m in range(d))
                  for k in range(d)])
    Ku = oracle.apply(ncell, h, LAM, MU, psi, u)
    C = _C(LAM, MU, d)
    # grad u_k (l) = B_kl + 2 (Q_k x)_l ; d_j d_l u_k = 2 Q_k[j,l]
    psi_n = psi0 + sum(gpsi[a] * Xn[a] for a in range(d))
    exact = np.zeros_like(u)
    for i, j, k, l in itertools.product(range(d), repeat=4):
        if C[i, j, k, l] == 0:
            continue
        grad_kl = B[k, l] + 2 * sum(Q[k, l, m] * Xn[m] for m in range(d))
        exact[i] -= C[i, j, k, l] * (gpsi[j] * grad_kl + psi_n * 2 * Q[k, j, l])
    m = _interior(ncell)
    err = np.abs(Ku[:, m] - exact[:, m]).max() / np.abs(exact[:, m]).max()
    assert err < 1e-11, err


@pytest.mark.parametrize("ncell", [(6, 5), (4, 3, 5)])
def test_symmetry(ncell):
    """<v, K u> = <u, K v> for random psi including floor values."""
    d = len(ncell)
    h = tuple(1.0 / n for n in ncell)
    psi, u, _ = si.random_fields(ncell, seed=1)
    psi[psi < 0.2] = 1e-6
    v = np.random.default_rng(2).standard_normal(u.shape)
    a = np.vdot(v, oracle.apply(ncell, h, LAM, MU, psi, u))
    b = np.vdot(u, oracle.apply(ncell, h, LAM, MU, psi, v))
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0) * u.size
    K = oracle.assemble(ncell, h, LAM, MU, psi)
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()


@pytest.mark.parametrize("ncell", [(6, 5), (4, 3, 5)])
def test_rigid_modes(ncell):
    """Translations and infinitesimal rotations lie in the kernel of K for any
    psi (all faces traction-free)."""
    d = len(ncell)
    h = tuple(1.0 / n for n in ncell)
    psi, _, _ = si.random_fields(ncell, seed=4)
    X = _nodes(ncell, h)
    modes = [np.stack([np.full_like(X[0], float(k == a)) for k in range(d)]) for a in range(d)]
    for a, b in itertools.combinations(range(d), 2):
        w = [np.zeros_like(X[0]) for _ in range(d)]
        w[a] = -X[b]
        w[b] = X[a]
        modes.append(np.stack(w))
    K1 = oracle.apply(ncell, h, LAM, MU, psi, np.ones((d,) + X[0].shape))
    scale = np.abs(K1).max() + np.abs(oracle.apply(ncell, h, LAM, MU, psi,
                                                    np.random.default_rng(0).standard_normal(K1.shape))).max()
    for m in modes:
        assert np.abs(oracle.apply(ncell, h, LAM, MU, psi, m)).max() < 1e-13 * scale


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("nu", [0.3, 0.45, 0.49])
def test_cell_matrix_psd_rigid_nullspace(dim, nu):
    """K on a single cell with psi=1 is that cell's matrix K_c: PSD with a
    null space of exactly the rigid modes (3 in 2D, 6 in 3D)."""
    lam, mu = si.lame(1.0, nu)
    ncell = (1,) * dim
    Kc = oracle.assemble(ncell, (1.0,) * dim, lam, mu, np.ones((1,) * dim))
    ev = np.linalg.eigvalsh(Kc)
    tol = 1e-12 * ev.max()
    assert ev.min() > -tol
    assert int((ev < tol).sum()) == (3 if dim == 2 else 6)


@pytest.mark.parametrize("ncell", [(6, 7), (5, 6, 4)])
def test_constant_psi_textbook_stencil(ncell):
    """With psi = 1 the interior rows are the second-order Navier-Lame stencil
    -[mu lap u + (lam+mu) grad div u] with central differences."""
    d = len(ncell)
    h = tuple(1.0 / n * (1 + 0.2 * a) for a, n in enumerate(ncell))
    _, u, _ = si.random_fields(ncell, seed=5)
    Ku = oracle.apply(ncell, h, LAM, MU, np.ones(tuple(reversed(ncell))), u)
    ax = lambda a: d - 1 - a  # numpy axis of spatial axis a

    def sh(f, offs):
        out = f
        for a, o in offs:
            out = np.roll(out, -o, axis=ax(a))
        return out

    ref = np.zeros_like(u)
    for i in range(d):
        for j in range(d):
            coef = MU + (LAM + MU) * (i == j)
            ref[i] -= coef * (sh(u[i], [(j, 1)]) - 2 * u[i] + sh(u[i], [(j, -1)])) / h[j] ** 2
        for l in range(d):
            if l == i:
                continue
            cross = (sh(u[l], [(i, 1), (l, 1)]) - sh(u[l], [(i, 1), (l, -1)])
                     - sh(u[l], [(i, -1), (l, 1)]) + sh(u[l], [(i, -1), (l, -1)])) / (4 * h[i] * h[l])
            ref[i] -= (LAM + MU) * cross
    m = _interior(ncell)
    assert np.abs(Ku[:, m] - ref[:, m]).max() < 1e-12 * np.abs(ref[:, m]).max()
    # diagonal of the constant-psi interior row: (2(lam+2mu) + 2(d-1)mu)/h^2 for equal h
    hh = (1.0 / 8,) * d
    D = oracle.diag((8,) * d, hh, LAM, MU, np.ones((8,) * d))
    centre = (slice(None),) + (4,) * d
    assert np.allclose(D[centre], (2 * (LAM + 2 * MU) + 2 * (d - 1) * MU) / hh[0] ** 2, rtol=1e-14)


def test_reduces_to_paper_1d_cell_operator():
    """u = (u_x(x), 0) and psi = psi(x): the u_x row is the paper's 1D
    cell-based operator (Sec. 2.3) with modulus lam+2mu, and its diagonal is
    C (psi_{i+1/2} + psi_{i-1/2}) / dx^2 (the true value of the Jacobi
    prefactor, which the printed update garbles by a constant factor)."""
    nx, ny = 12, 5
    h = (1.0 / nx, 0.7 / ny)
    rng = np.random.default_rng(6)
    psi_x = rng.uniform(0.0, 1.0, nx)
    psi_x[3:5] = 0.0  # a void in the middle
    psi = np.tile(psi_x, (ny, 1))
    ux = rng.standard_normal(nx + 1)
    u = np.zeros((2, ny + 1, nx + 1))
    u[0] = ux[None, :]
    Ku = oracle.apply((nx, ny), h, LAM, MU, psi, u)
    C = LAM + 2 * MU
    dx = h[0]
    i = np.arange(1, nx)
    pp, pm = psi_x[i], psi_x[i - 1]
    paper = C * ((pp - pm) / dx * (ux[i + 1] - ux[i - 1]) / (2 * dx)
                 + 0.5 * (pp + pm) * (ux[i + 1] - 2 * ux[i] + ux[i - 1]) / dx ** 2)
    for j in range(1, ny):
        assert np.allclose(Ku[0, j, 1:nx], -paper, rtol=1e-12, atol=1e-12 * np.abs(paper).max())
        assert np.abs(Ku[1, j, 1:nx]).max() < 1e-12 * np.abs(paper).max()
    D = oracle.diag((nx, ny), h, LAM, MU, psi)
    # the u_x diagonal at interior nodes: C (psi+ + psi-)/dx^2 + mu (psi+ + psi-) / dy^2
    # (the y edges of an x-only field see the same two cells)
    expect = C * (pp + pm) / dx ** 2 + MU * (pp + pm) / h[1] ** 2
    assert np.allclose(D[0, 2, 1:nx], expect, rtol=1e-13)


def test_node_psi_jacobi_breaks_cell_psi_does_not():
    """Sec. 2.3: with psi on nodes, the Jacobi diagonal -2 C psi_i / dx^2
    vanishes at a node with psi_i = 0 next to non-zero neighbours while the
    off-diagonal part does not; with psi in cells the diagonal vanishes only
    where both adjacent cells vanish."""
    C, dx = 1.0, 0.1
    psi_node = np.array([1.0, 0.5, 0.0, 0.5, 1.0])
    i = 2
    diag_node = -2 * C * psi_node[i] / dx ** 2
    offdiag_node = C * (psi_node[i + 1] - psi_node[i - 1]) / (2 * dx) / (2 * dx)
    assert diag_node == 0.0 and offdiag_node == 0.0  # symmetric neighbours: degenerate
    psi_node = np.array([1.0, 0.8, 0.0, 0.3, 1.0])
    offdiag_node = C * (psi_node[i + 1] - psi_node[i - 1]) / (2 * dx) / (2 * dx)
    assert -2 * C * psi_node[i] / dx ** 2 == 0.0 and offdiag_node != 0.0  # D^-1 undefined
    # the oracle's cell-based diagonal in the same situation (one adjacent cell empty)
    nx, ny = 4, 3
    psi = np.tile(np.array([1.0, 0.0, 0.4, 1.0]), (ny, 1))
    D = oracle.diag((nx, ny), (dx, dx), LAM, MU, psi)
    assert (D[:, 1:ny, 1:nx] > 0).all()
    psi = np.tile(np.array([1.0, 0.0, 0.0, 1.0]), (ny, 1))
    D = oracle.diag((nx, ny), (dx, dx), LAM, MU, psi)
    assert (D[:, :, 2] == 0).all()  # both adjacent cells empty: an isolated, well-posed zero row
    u = np.random.default_rng(0).standard_normal((2, ny + 1, nx + 1))
    assert np.abs(oracle.apply((nx, ny), (dx, dx), LAM, MU, psi, u)[:, :, 2]).max() == 0.0


@pytest.mark.parametrize("ncell", [(6, 5), (4, 3, 5)])
def test_linear_in_psi_and_moduli(ncell):
    """K is linear in psi and in (lambda, mu) (material models form a vector
    space over the Lame constants, Sec. 2.4)."""
    h = tuple(1.0 / n for n in ncell)
    p1, u, _ = si.random_fields(ncell, seed=7)
    p2, _, _ = si.random_fields(ncell, seed=8)
    A = lambda lam, mu, psi: oracle.apply(ncell, h, lam, mu, psi, u)
    ref = np.abs(A(LAM, MU, p1)).max()
    assert np.abs(A(LAM, MU, 2 * p1 + 3 * p2) - 2 * A(LAM, MU, p1) - 3 * A(LAM, MU, p2)).max() < 1e-13 * ref * 10
    assert np.abs(A(2 * LAM + 0.5, 3 * MU + 0.25, p1)
                  - 2 * A(LAM, 0.0, p1) - A(0.5, 0.0, p1) - 3 * A(0.0, MU, p1) - A(0.0, 0.25, p1)).max() < 1e-12 * ref
    assert np.abs(A(0.0, 0.0, p1)).max() == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_uniaxial_traction_exact(dim):
    """psi = 1, rollers on the low faces (u_a = 0 on x_a = 0), uniform normal
    traction t on the top face: the exact uniaxial field (with Poisson
    contraction) satisfies the discrete equations, including the traction
    source of every boundary row, to rounding."""
    ncell = (5, 4) if dim == 2 else (4, 5, 3)
    h = tuple(1.0 / n for n in ncell)
    t = 1e-3
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    for a in range(dim):
        kind[2 * a, a] = oracle.DISPLACEMENT
    top = dim - 1
    val[2 * top + 1, top] = t
    psi = np.ones(tuple(reversed(ncell)))
    # stress sigma = t e_top (x) e_top  ->  strain = S sigma with the isotropic compliance
    C = _C(LAM, MU, dim).reshape(dim * dim, dim * dim)
    sig = np.zeros((dim, dim))
    sig[top, top] = t
    eps = np.linalg.lstsq(C, sig.ravel(), rcond=None)[0].reshape(dim, dim)
    X = _nodes(ncell, h)
    u = np.stack([eps[k, k] * X[k] for k in range(dim)])
    fA, fB, uD = oracle.rhs(ncell, h, LAM, MU, psi, kind, val)
    mask, _ = oracle.dirichlet(ncell, kind, val)
    r = oracle.residual(ncell, h, LAM, MU, psi, mask, u, fA)
    assert np.abs(r).max() < 1e-12 * np.abs(fA).max()
    us, hist, st = oracle.solve(ncell, h, LAM, MU, psi, 0.0, kind, val, rtol=1e-13, max_cycles=400)
    assert st == 0
    assert np.abs(us - u).max() < 1e-9 * np.abs(u).max()


def test_traction_source_shares_and_1d_bar():
    """The traction source is t/h times the fraction of the adjacent boundary
    cells that are solid: 1 inside a face, 1/2 on its edges, 1/4 at corners;
    and a bar with traction t at its free end stretches as u = t x / C."""
    ncell = (3, 4, 2)
    h = (0.5, 0.25, 0.5)
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    val[1, 0] = 2.0  # traction in x on face x+
    fA, _, _ = oracle.rhs(ncell, h, LAM, MU, np.ones((2, 4, 3)), kind, val)
    face = fA[0, :, :, 3] * h[0] / 2.0
    expect = np.ones((3, 5))
    expect[0, :] *= 0.5
    expect[-1, :] *= 0.5
    expect[:, 0] *= 0.5
    expect[:, -1] *= 0.5
    assert np.allclose(face, expect, rtol=0, atol=1e-15)
    # 1D bar (a strip with one cell across, rollers keep it uniaxial in y)
    nx = 8
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    kind[0, :2] = oracle.DISPLACEMENT
    kind[2, 1] = oracle.DISPLACEMENT
    kind[3, 1] = oracle.DISPLACEMENT
    val[1, 0] = 1e-3
    lam, mu = si.lame(1.0, 0.0)  # nu = 0: no Poisson coupling, C = lam + 2 mu = E
    u, hist, st = oracle.solve((nx, 1), (1.0 / nx, 1.0), lam, mu, np.ones((1, nx)), 0.0, kind, val,
                               rtol=1e-14, max_cycles=50)
    x = np.arange(nx + 1) / nx
    assert np.allclose(u[0, 0], 1e-3 * x / (lam + 2 * mu), rtol=1e-10, atol=1e-16)


def test_rhs_dirichlet_and_lifting():
    """Dirichlet DOF take their values (the last face in x-,x+,y-,y+,z-,z+
    order wins on shared edges), carry no load, and the lifted load is
    fA - K uD on the free DOF."""
    ncell = (4, 3, 3)
    h = (0.25, 1 / 3, 1 / 3)
    psi, _, _ = si.random_fields(ncell, seed=9)
    kind, val = si.mixed_bc(3, seed=3)
    mask, uD = oracle.dirichlet(ncell, kind, val)
    fA, fB, uD2 = oracle.rhs(ncell, h, LAM, MU, psi, kind, val)
    assert np.array_equal(uD, uD2)
    assert (fA[mask == 1] == 0).all() and (fB[mask == 1] == 0).all()
    KuD = oracle.apply(ncell, h, LAM, MU, psi, uD)
    free = mask == 0
    assert np.allclose(fB[free], fA[free] - KuD[free], rtol=0, atol=1e-15 * np.abs(KuD).max())
    # explicit precedence check at a node on faces x- and y-
    for k in range(3):
        if kind[2, k] == oracle.DISPLACEMENT:
            assert uD[k, 1, 0, 0] == val[2, k]
        elif kind[0, k] == oracle.DISPLACEMENT:
            assert uD[k, 1, 0, 0] == val[0, k]
