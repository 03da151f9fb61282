"""Pins of the oracle's phase-field fracture pieces (Sec. 3.2).

The crack driving force is checked on strains whose principal values are
known (a rotated diagonal strain, pure tension, pure compression) and for the
history property of H; the Ginzburg-Landau step by its fixed point, its
closed form for a uniform field, its projection onto [0, 1] (the range of
the crack field), and the discrete Laplacian it contains (exact for a
quadratic in the interior, summing to zero over the box with the zero-flux
faces)."""
import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q


def _linear_u(ncell, h, E):
    X = si.node_coords(ncell, h)
    d = len(ncell)
    return np.stack([sum(E[k, l] * X[l] for l in range(d)) for k in range(d)])


def _w_plus_minus(e):
    ep, em = np.clip(e, 0, None), np.clip(e, None, 0)
    return (0.5 * LAM * ep.sum() ** 2 + MU * (ep ** 2).sum(),
            0.5 * LAM * em.sum() ** 2 + MU * (em ** 2).sum())


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_driving_force_of_a_rotated_principal_strain(dim, seed):
    """u = R D R^T x: every cell has the principal strains D."""
    ncell = (3, 4) if dim == 2 else (3, 2, 4)
    h = (0.3, 0.2, 0.25)[:dim]
    D = np.random.default_rng(10 + seed).standard_normal(dim) * 1e-3
    R = _rot(seed)[:dim, :dim]
    if dim == 2:
        R, _ = np.linalg.qr(R)
    E = R @ np.diag(D) @ R.T
    u = _linear_u(ncell, h, E)
    H0 = np.zeros(tuple(reversed(ncell)))
    H, intact = oracle.crack_drive(ncell, h, LAM, MU, u, H0)
    wp, wm = _w_plus_minus(D)
    assert np.allclose(H, wp, rtol=1e-10, atol=1e-18)
    assert np.all(intact == (wp < wm))


def test_tension_compression_and_history():
    ncell, h = (3, 3, 2), (0.5, 0.5, 0.5)
    E = np.diag([1e-3, 2e-3, 5e-4])
    shape = tuple(reversed(ncell))
    H, intact = oracle.crack_drive(ncell, h, LAM, MU, _linear_u(ncell, h, E), np.zeros(shape))
    W0 = 0.5 * LAM * np.trace(E) ** 2 + MU * np.sum(E * E)
    assert np.allclose(H, W0, rtol=1e-12) and not intact.any()   # pure tension: W0+ = W0
    H2, intact2 = oracle.crack_drive(ncell, h, LAM, MU, _linear_u(ncell, h, -E), H)
    assert np.array_equal(H2, H) and intact2.all()               # compression: W0+ = 0
    Hbig = np.full(shape, 1.0)
    H3, _ = oracle.crack_drive(ncell, h, LAM, MU, _linear_u(ncell, h, E), Hbig)
    assert np.array_equal(H3, Hbig)                              # history keeps the maximum


def _lap_from_step(ncell, h, c, dt):
    """With H = 0, Gc = M = 1, xi = 1/2 the step is c + dt (lap(c) + w'(c)),
    w' = -g' = -(12 c^2 - 12 c^3): read lap(c) back (dt small enough that
    the step stays inside [0, 1])."""
    shape = tuple(reversed(ncell))
    c1, _ = oracle.phase_step(ncell, h, c, np.zeros(shape), np.zeros(shape, np.uint8), 1.0, 0.5,
                              1.0, dt)
    assert 0.0 < c1.min() and c1.max() < 1.0
    return (c1 - c) / dt + (12 * c ** 2 - 12 * c ** 3)


@pytest.mark.parametrize("ncell", [(7, 5), (6, 5, 4)])
def test_laplacian_in_the_step(ncell):
    h = (0.2, 0.25, 0.3)[:len(ncell)]
    cc = si.cell_centres(ncell, h)
    q = 0.4 + 0.02 * sum((a + 1.0) * x * x for a, x in enumerate(cc))  # lap q = 0.04 sum (a+1)
    lap = _lap_from_step(ncell, h, q, 1e-2)
    inner = tuple(slice(1, -1) for _ in ncell)
    assert np.allclose(lap[inner], 0.04 * sum(a + 1.0 for a in range(len(ncell))), rtol=1e-9)
    c = np.random.default_rng(3).uniform(0.4, 0.6, size=tuple(reversed(ncell)))
    lap = _lap_from_step(ncell, h, c, 1e-4)
    assert abs(lap.sum()) <= 1e-10 * np.abs(lap).sum()      # zero flux through the box faces


def test_step_closed_form_and_fixed_point():
    ncell, h = (4, 3), (0.1, 0.1)
    shape = tuple(reversed(ncell))
    Gc, xi, M, dt, eta = 2.7, 0.05, 0.3, 0.01, 1e-4
    c0, H0 = 0.6, 5.0
    c1, psi = oracle.phase_step(ncell, h, np.full(shape, c0), np.full(shape, H0),
                                np.zeros(shape, np.uint8), Gc, xi, M, dt, eta)
    gp = 12 * c0 ** 2 - 12 * c0 ** 3
    ref = c0 - dt * M * (gp * H0 - Gc * (-gp) / (2 * xi))
    assert np.allclose(c1, ref, rtol=1e-14)
    assert np.allclose(psi, 4 * ref ** 3 - 3 * ref ** 4 + eta, rtol=1e-14)
    ones, _ = oracle.phase_step(ncell, h, np.ones(shape), np.full(shape, H0),
                                np.zeros(shape, np.uint8), Gc, xi, M, dt, eta)
    assert np.array_equal(ones, np.ones(shape))              # intact material stays intact
    held, _ = oracle.phase_step(ncell, h, np.full(shape, 0.2), np.full(shape, H0),
                                np.ones(shape, np.uint8), Gc, xi, M, dt, eta)
    assert np.array_equal(held, np.ones(shape))              # W0+ < W0- forces c = 1


def test_step_stays_in_the_unit_interval():
    """A driving force far above the threshold takes c below 0 in one explicit
    step and a field above 1 is pushed further up: both are projected onto
    [0, 1]; a NaN is not hidden."""
    ncell, h = (3, 2), (0.1, 0.1)
    shape = tuple(reversed(ncell))
    Gc, xi, M, dt = 1.0, 0.1, 1.0, 1.0
    free = np.zeros(shape, np.uint8)
    c0 = 0.5
    gp = 12 * c0 ** 2 - 12 * c0 ** 3
    H = 10.0
    raw = c0 - dt * M * (gp * H + Gc * gp / (2 * xi))
    assert raw < 0
    c1, psi = oracle.phase_step(ncell, h, np.full(shape, c0), np.full(shape, H), free, Gc, xi, M,
                                dt, 1e-4)
    assert np.array_equal(c1, np.zeros(shape)) and np.allclose(psi, 1e-4, rtol=0, atol=1e-18)
    c0 = 1.2
    gp = 12 * c0 ** 2 - 12 * c0 ** 3
    assert c0 - dt * M * (gp * H + Gc * gp / (2 * xi)) > 1
    c1, _ = oracle.phase_step(ncell, h, np.full(shape, c0), np.full(shape, H), free, Gc, xi, M,
                              dt, 1e-4)
    assert np.array_equal(c1, np.ones(shape))
    c = np.full(shape, 0.5)
    c[0, 0] = np.nan
    c1, _ = oracle.phase_step(ncell, h, c, np.zeros(shape), free, Gc, xi, M, 1e-3, 1e-4)
    assert np.isnan(c1[0, 0])
