"""Seeded synthetic inputs for the SBM elasticity solve.

This module builds problem *inputs* only: cell indicator fields, boundary
tables, body forces and grid sizes.  It holds none of the solver's arithmetic
(no operator, no floor, no source terms) and is the only module shared by the
HIP library's tests and the CPU oracle.

The workloads stand in for the geometries of arXiv:2212.02362 (no public
dataset exists): a 2D plate with a circular void (Sec. 3.1), a 3D block with
spherical voids (Sec. 3.1), a near-singular diffuse crack in a random void
field (Sec. 3.2), ellipsoidal voids for the adaptive case, and a SIMP-like
random density for the topology-optimisation gradient (Sec. 3.3).  Every
generator draws from ``numpy.random.default_rng(seed)`` in the order written.

Array conventions: cells ``(ny, nx)`` / ``(nz, ny, nx)``; node vectors
``(d, ny+1, nx+1)`` / ``(d, nz+1, ny+1, nx+1)``; ``ncell = (nx, ny[, nz])``.
Boundary tables are ``(6, 3)`` over faces x-, x+, y-, y+, z-, z+.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

TRACTION = 0
DISPLACEMENT = 1


def lame(E: float, nu: float):
    """(lambda, mu) from Young's modulus and Poisson's ratio."""
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


@dataclasses.dataclass
class Problem:
    name: str
    ncell: tuple
    h: tuple
    lam: float
    mu: float
    psi_floor: float
    psi_raw: np.ndarray            # cells, before the floor
    kind: np.ndarray               # (6, 3) int32
    val: np.ndarray                # (6, 3) float64
    b: Optional[np.ndarray] = None  # node body force or None
    rho: Optional[np.ndarray] = None  # density (topology-optimisation input)
    fd_cells: Optional[np.ndarray] = None
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def dim(self):
        return len(self.ncell)

    @property
    def node_shape(self):
        return tuple(n + 1 for n in reversed(self.ncell))

    @property
    def n_nodes(self):
        return int(np.prod(self.node_shape))


def _bc_table():
    return np.zeros((6, 3), np.int32), np.zeros((6, 3), np.float64)


def cell_centres(ncell, h):
    """Coordinate arrays of the cell centres, numpy axis order (z, y, x)."""
    axes = [(np.arange(n) + 0.5) * hh for n, hh in zip(ncell, h)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))  # [X, Y(, Z)] each shaped like the cells


def node_coords(ncell, h):
    axes = [np.arange(n + 1) * hh for n, hh in zip(ncell, h)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))


def plate_void_2d(n: int = 64, floor: float = 1e-4) -> Problem:
    """Unit square, centred circular void of radius 0.25 with tanh width 2h.
    Bottom edge clamped, uniform normal traction 1e-3 on the top edge, sides
    traction-free."""
    h = 1.0 / n
    X, Y = cell_centres((n, n), (h, h))
    r = np.hypot(X - 0.5, Y - 0.5)
    psi = 0.5 * (1 + np.tanh((r - 0.25) / (2 * h)))
    kind, val = _bc_table()
    kind[2, :2] = DISPLACEMENT
    val[3, 1] = 1e-3
    lam, mu = lame(1.0, 0.3)
    return Problem("plate_void_2d", (n, n), (h, h), lam, mu, floor, psi, kind, val)


def plate_void_amr_2d(base: int = 16, levels: int = 3, block: int = 8, floor: float = 1e-4):
    """The plate with a centred circular void for the adaptive solve in 2D:
    the indicator 0.5 (1 + tanh((r - 0.25) / (2 h_f))), h_f the finest
    spacing, sampled at the cell centres of every level (level a: base * 2^a
    cells per axis).  Bottom edge clamped, normal traction 1e-3 on the top.
    Returns (Problem of the base level, list of per-level raw psi)."""
    hf = 1.0 / (base << (levels - 1))
    psis = []
    for a in range(levels):
        n = base << a
        X, Y = cell_centres((n, n), (1.0 / n, 1.0 / n))
        r = np.hypot(X - 0.5, Y - 0.5)
        psis.append(0.5 * (1 + np.tanh((r - 0.25) / (2 * hf))))
    kind, val = _bc_table()
    kind[2, :2] = DISPLACEMENT
    val[3, 1] = 1e-3
    lam, mu = lame(1.0, 0.3)
    h0 = 1.0 / base
    p = Problem("plate_void_amr_2d", (base, base), (h0, h0), lam, mu, floor, psis[0], kind, val,
                extra={"levels": levels, "block": block})
    return p, psis


def spherical_voids_3d(n: int = 128, seed: int = 0, nvoid: int = 20,
                       floor: float = 1e-6) -> Problem:
    """Unit cube with seeded spherical voids (centres U[0,1]^3, radii
    U[0.05,0.15], tanh width 2h).  z=0 clamped, u=(0,0,1e-3) on z=1."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (nvoid, 3))
    radii = rng.uniform(0.05, 0.15, nvoid)
    h = 1.0 / n
    X, Y, Z = cell_centres((n, n, n), (h, h, h))
    psi = np.ones_like(X)
    for c, R in zip(centres, radii):
        dist = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        psi *= 0.5 * (1 + np.tanh((dist - R) / (2 * h)))
    kind, val = _bc_table()
    kind[4, :] = DISPLACEMENT
    kind[5, :] = DISPLACEMENT
    val[5, 2] = 1e-3
    lam, mu = lame(1.0, 0.3)
    return Problem("spherical_voids_3d", (n, n, n), (h, h, h), lam, mu, floor, psi, kind, val,
                   extra={"centres": centres, "radii": radii})


def pressurised_voids_3d(n: int = 128, seed: int = 0, nvoid: int = 20, pressure: float = 1e-3,
                         floor: float = 1e-6) -> Problem:
    """The voids of ``spherical_voids_3d`` (same draws) under an internal
    pressure instead of a displacement load: z=0 clamped, every other box
    face traction free, the load a pressure ``pressure`` on the diffuse void
    surfaces (Sec. 2.1 diffuse traction; in ``extra``, the load itself is not
    formed here)."""
    p = spherical_voids_3d(n, seed, nvoid, floor)
    kind, val = _bc_table()
    kind[4, :] = DISPLACEMENT
    return Problem("pressurised_voids_3d", p.ncell, p.h, p.lam, p.mu, floor, p.psi_raw, kind, val,
                   extra=dict(p.extra, pressure=pressure))


def pressurised_hole_quarter(n: int = 64, L: float = 16.0, a: float = 1.0, width=None,
                             pressure: float = 1e-3, floor: float = 1e-6) -> Problem:
    """Quarter plate [0, L]^2 with a circular hole of radius a at the origin
    under an internal pressure: rollers on x=0 (u_x=0) and y=0 (u_y=0), outer
    edges free, indicator 0.5(1+tanh((r-a)/width)) (width 2h by default);
    the pressure is in ``extra``."""
    h = L / n
    w = 2.0 * h if width is None else width
    X, Y = cell_centres((n, n), (h, h))
    psi = 0.5 * (1 + np.tanh((np.hypot(X, Y) - a) / w))
    kind, val = _bc_table()
    kind[0, 0] = DISPLACEMENT
    kind[2, 1] = DISPLACEMENT
    lam, mu = lame(1.0, 0.3)
    return Problem("pressurised_hole_quarter", (n, n), (h, h), lam, mu, floor, psi, kind, val,
                   extra={"L": L, "a": a, "width": w, "pressure": pressure})


def _smooth_field(rng, shape, sigma_cells):
    from scipy.ndimage import gaussian_filter
    g = rng.standard_normal(shape)
    g = gaussian_filter(g, sigma_cells, mode="reflect")
    return (g - g.mean()) / g.std()


def diffuse_crack_3d(n: int = 256, seed: int = 0, floor: float = 1e-6) -> Problem:
    """Planar disc crack (radius 0.3, centre (1/2,1/2,1/2), seeded normal) with
    crack factor 1-exp(-d/2h), times a random void field in which 40% of the
    cells fall below 0.01.  Mode-I displacement loading on the faces normal to
    the dominant normal axis."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(3)
    nrm = v / np.linalg.norm(v)
    h = 1.0 / n
    X, Y, Z = cell_centres((n, n, n), (h, h, h))
    dx, dy, dz = X - 0.5, Y - 0.5, Z - 0.5
    z = dx * nrm[0] + dy * nrm[1] + dz * nrm[2]
    px, py, pz = dx - z * nrm[0], dy - z * nrm[1], dz - z * nrm[2]
    rho_par = np.sqrt(px * px + py * py + pz * pz)
    dist = np.sqrt(z * z + np.maximum(rho_par - 0.3, 0.0) ** 2)
    psi_cr = 1.0 - np.exp(-dist / (2 * h))
    del X, Y, Z, dx, dy, dz, z, px, py, pz, rho_par, dist
    g = _smooth_field(rng, (n, n, n), 8.0 / math.sqrt(2.0))
    tau = np.quantile(g, 0.4)
    psi_v = 1.0 / (1.0 + np.exp(-((g - tau) / 0.05 - math.log(99.0))))
    psi = psi_cr * psi_v
    a = int(np.argmax(np.abs(nrm)))
    kind, val = _bc_table()
    kind[2 * a, :] = DISPLACEMENT
    kind[2 * a + 1, :] = DISPLACEMENT
    val[2 * a + 1, a] = 1e-3
    lam, mu = lame(1.0, 0.3)
    return Problem("diffuse_crack_3d", (n, n, n), (h, h, h), lam, mu, floor, psi, kind, val,
                   extra={"normal": nrm, "axis": a, "void_fraction": float((psi_v < 0.01).mean())})


def cantilever_density_3d(nx: int = 192, ny: int = 96, nz: int = 96, seed: int = 0,
                          floor: float = 1e-4, n_fd: int = 32) -> Problem:
    """Topology-optimisation gradient workload: domain [0,2]x[0,1]x[0,1],
    density rho = sigmoid of a standardised Gaussian random field (correlation
    length 8h), psi = rho^3 (raw), x=0 clamped, unit load (0,0,-1) smoothed
    over a 4h ball at the far corner (2,1,1) with weights (1-(r/4h)^2)^2
    normalised so that h^3 sum(b) = F."""
    rng = np.random.default_rng(seed)
    h = 1.0 / ny
    g = _smooth_field(rng, (nz, ny, nx), 8.0 / math.sqrt(2.0))
    rho = 1.0 / (1.0 + np.exp(-g))
    fd = rng.choice(nx * ny * nz, size=n_fd, replace=False)
    Xn, Yn, Zn = node_coords((nx, ny, nz), (h, h, h))
    r = np.sqrt((Xn - nx * h) ** 2 + (Yn - ny * h) ** 2 + (Zn - nz * h) ** 2)
    w = np.where(r < 4 * h, (1 - (r / (4 * h)) ** 2) ** 2, 0.0)
    F = np.array([0.0, 0.0, -1.0])
    b = np.zeros((3,) + w.shape)
    for k in range(3):
        b[k] = F[k] * w / (h ** 3 * w.sum())
    kind, val = _bc_table()
    kind[0, :] = DISPLACEMENT
    lam, mu = lame(1.0, 0.3)
    return Problem("cantilever_density_3d", (nx, ny, nz), (h, h, h), lam, mu, floor, rho ** 3,
                   kind, val, b=b, rho=rho, fd_cells=fd)


def kirsch_quarter_plate(n: int = 128, L: float = 16.0, a: float = 1.0, width: float = 0.5,
                         sigma: float = 1e-3, floor: float = 1e-6) -> Problem:
    """Quarter model of an infinite plate with a circular hole (radius a at the
    origin) under remote uniaxial stress sigma along x: rollers on x=0 (u_x=0)
    and y=0 (u_y=0), traction (sigma, 0) on x=L, y=L traction-free.  The
    indicator is 0.5(1+tanh((r-a)/width))."""
    h = L / n
    X, Y = cell_centres((n, n), (h, h))
    r = np.hypot(X, Y)
    psi = 0.5 * (1 + np.tanh((r - a) / width))
    kind, val = _bc_table()
    kind[0, 0] = DISPLACEMENT
    kind[2, 1] = DISPLACEMENT
    val[1, 0] = sigma
    lam, mu = lame(1.0, 0.3)
    return Problem("kirsch_quarter_plate", (n, n), (h, h), lam, mu, floor, psi, kind, val,
                   extra={"L": L, "a": a, "sigma": sigma, "width": width})


def random_fields(ncell, seed=0, psi_lo=1e-6, psi_hi=1.0):
    """Random psi (cells) and u, f (nodes) for kernel-level parity tests."""
    rng = np.random.default_rng(seed)
    d = len(ncell)
    cs = tuple(reversed(ncell))
    ns = (d,) + tuple(n + 1 for n in reversed(ncell))
    psi = rng.uniform(psi_lo, psi_hi, cs)
    u = rng.standard_normal(ns)
    f = rng.standard_normal(ns)
    return psi, u, f


def mixed_bc(dim, seed=0):
    """A boundary table mixing traction and displacement faces/components."""
    rng = np.random.default_rng(seed)
    kind, val = _bc_table()
    for F in range(2 * dim):
        for k in range(dim):
            kind[F, k] = int(rng.integers(0, 2))
            val[F, k] = rng.uniform(-1e-3, 1e-3)
    kind[0, :dim] = DISPLACEMENT  # something always pins the rigid modes
    return kind, val


def _quat_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def ellipsoidal_voids_amr(base: int = 64, levels: int = 3, block: int = 32, seed: int = 0,
                          nvoid: int = 10, floor: float = 1e-5, shape=None):
    """Unit cube with seeded ellipsoidal voids for the adaptive solve: centres
    U[0,1]^3, then semi-axes U[0.04,0.12] (nvoid x 3), then orientations from
    unit quaternions drawn from N(0, I4).  The indicator is the product of
    0.5 (1 + tanh(d / (2 h_f))) with d = (q - 1)/|grad q|, q = |A^-1 R^T (x - c)|
    and h_f the finest spacing, sampled at the cell centres of every level
    (level a: base * 2^a cells per axis).  z=0 clamped, u=(0,0,1e-3) on z=1.
    ``shape`` (cells per axis x, y, z of the base level) makes the box
    shape[a] / base long along axis a, with the same spacing 1 / base and
    the centres scaled to the box (the same draws).
    Returns (Problem of the base level, list of per-level raw psi)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (nvoid, 3))
    axes = rng.uniform(0.04, 0.12, (nvoid, 3))
    quats = rng.standard_normal((nvoid, 4))
    shape = (base, base, base) if shape is None else tuple(int(n) for n in shape)
    centres = centres * (np.asarray(shape, np.float64) / base)
    hf = 1.0 / (base << (levels - 1))
    psis = []
    for a in range(levels):
        ns = tuple(n << a for n in shape)
        h = 1.0 / (base << a)
        X, Y, Z = cell_centres(ns, (h, h, h))
        psi = np.ones_like(X)
        for c, ax, q in zip(centres, axes, quats):
            M = np.diag(1.0 / ax) @ _quat_rot(q).T
            dx, dy, dz = X - c[0], Y - c[1], Z - c[2]
            y0 = M[0, 0] * dx + M[0, 1] * dy + M[0, 2] * dz
            y1 = M[1, 0] * dx + M[1, 1] * dy + M[1, 2] * dz
            y2 = M[2, 0] * dx + M[2, 1] * dy + M[2, 2] * dz
            qn = np.sqrt(y0 * y0 + y1 * y1 + y2 * y2)
            MtM = M.T @ M
            gx = (MtM[0, 0] * dx + MtM[0, 1] * dy + MtM[0, 2] * dz)
            gy = (MtM[1, 0] * dx + MtM[1, 1] * dy + MtM[1, 2] * dz)
            gz = (MtM[2, 0] * dx + MtM[2, 1] * dy + MtM[2, 2] * dz)
            gq = np.sqrt(gx * gx + gy * gy + gz * gz) / np.maximum(qn, 1e-300)
            dist = (qn - 1.0) / np.maximum(gq, 1e-300)
            psi *= 0.5 * (1 + np.tanh(dist / (2 * hf)))
        psis.append(psi)
    kind, val = _bc_table()
    kind[4, :] = DISPLACEMENT
    kind[5, :] = DISPLACEMENT
    val[5, 2] = 1e-3
    lam, mu = lame(1.0, 0.3)
    h0 = 1.0 / base
    p = Problem("ellipsoidal_voids_amr", shape, (h0, h0, h0), lam, mu, floor, psis[0],
                kind, val, extra={"levels": levels, "block": block, "centres": centres,
                                  "axes": axes, "quats": quats})
    return p, psis


def j2_void_tension(n: int = 32, radii=(7.5, 4.08, 4.08), floor: float = 1e-4) -> Problem:
    """The plastic-void tension specimen of the J2 example (Sec. 3.1): the
    cube [-16, 16]^3 with an ellipsoidal void of semi-axes ``radii`` centred
    at the origin, indicator 0.5 (1 + tanh(d / eps)) with eps = 0.4 and
    d = (q - 1)/|grad q|, q = |x / r|; E = 210 (GPa), nu = 0.3.  Face x = -16
    clamped, the x-displacement of face x = +16 prescribed (``val[1, 0]``, 0
    here; the caller sets each load step), its other components free.  The
    J2 parameters sigma_Y = 0.2, Hbar = 50, theta = 1 are in ``extra``."""
    h = 32.0 / n
    X, Y, Z = cell_centres((n, n, n), (h, h, h))
    X, Y, Z = X - 16.0, Y - 16.0, Z - 16.0
    r = np.asarray(radii, np.float64)
    qn = np.sqrt((X / r[0]) ** 2 + (Y / r[1]) ** 2 + (Z / r[2]) ** 2)
    gq = np.sqrt((X / r[0] ** 2) ** 2 + (Y / r[1] ** 2) ** 2 + (Z / r[2] ** 2) ** 2) / np.maximum(qn, 1e-300)
    dist = (qn - 1.0) / np.maximum(gq, 1e-300)
    psi = 0.5 * (1.0 + np.tanh(dist / 0.4))
    kind, val = _bc_table()
    kind[0, :] = DISPLACEMENT
    kind[1, 0] = DISPLACEMENT
    lam, mu = lame(210.0, 0.3)
    return Problem("j2_void_tension", (n, n, n), (h, h, h), lam, mu, floor, psi, kind, val,
                   extra={"sigma_y": 0.2, "hbar": 50.0, "theta": 1.0, "radii": tuple(radii)})


def pf_mode1_2d(n: int = 4096, L: float = 0.02, notch: float = 1.5e-4, xi: float = 1e-5,
                uy: float = 1.5e-5, floor: float = 1e-4) -> Problem:
    """The Mode-I phase-field fracture specimen (Sec. 3.2) on a uniform grid:
    the square [-L/2, L/2]^2 with n x n cells, lambda = 121.15e9, mu =
    80.77e9 (Pa), a notch of length ``notch`` along y = 0 from the centre of
    the left edge.  The initial crack field is c0 = 1 - exp(-d / xi), d the
    distance of the cell centre to the notch segment.  The indicator the solve
    needs, psi = g(c0) + eta, is NOT formed here (``psi_raw`` is None): it is
    model arithmetic, so each path computes it with its own degradation
    function (its crack step with dt = 0).  Bottom edge clamped,
    y-displacement ``uy`` prescribed on the top edge (x free), left and right
    edges traction free.  ``extra`` holds c0 and the Ginzburg-Landau
    parameters Gc = 2700, xi, M = 1e-5, dt = 1e-4, eta = 1e-4."""
    h = L / n
    X, Y = cell_centres((n, n), (h, h))
    X, Y = X - 0.5 * L, Y - 0.5 * L
    x1 = -0.5 * L + notch
    dx = np.maximum(X - x1, 0.0)
    d = np.sqrt(dx * dx + Y * Y)
    c0 = 1.0 - np.exp(-d / xi)
    eta = 1e-4
    kind, val = _bc_table()
    kind[2, :] = DISPLACEMENT
    kind[3, 1] = DISPLACEMENT
    val[3, 1] = uy
    return Problem("pf_mode1_2d", (n, n), (h, h), 121.15e9, 80.77e9, floor, None, kind, val,
                   extra={"c0": c0, "Gc": 2700.0, "xi": xi, "M": 1e-5, "dt": 1e-4, "eta": eta,
                          "notch": notch, "uy": uy})
