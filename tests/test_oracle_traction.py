"""Pins of the oracle's diffuse traction load (Sec. 2.1, eq.
SBMLinearElasticity): the sharp limit of a slab (the load of the box-face
traction), the balance of a pressure on a closed void (no net force, no net
torque, first moment = pressure x dimension x void volume, all exact in the
discrete sums), and the pressurised circular hole of plane-strain elasticity
approached as the diffuse width shrinks."""
import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)


@pytest.mark.parametrize("ncell", [(9, 6), (7, 5, 6)])
def test_slab_is_the_box_face_traction(ncell):
    """Cells x < m solid, x >= m empty (floor 0): a traction t on that
    interface loads its interior nodes with t / h_x, as the box-face source of
    a box that ends at x = m; a pressure loads them with -p / h_x along x."""
    d = len(ncell)
    h = (0.3, 0.25, 0.2)[:d]
    m = 4
    shape = tuple(reversed(ncell))
    psi = np.zeros(shape)
    psi[..., :m] = 1.0
    t = np.array([0.7, -0.4, 0.25])[:d]
    t_hat = np.broadcast_to(t.reshape((d,) + (1,) * d), (d,) + tuple(n + 1 for n in shape)).copy()
    f = oracle.diffuse_traction(ncell, h, psi, 0.0, t_hat=t_hat)
    inner = (slice(1, -1),) * (d - 1)
    for k in range(d):
        face = f[k][inner + (m,)]
        assert np.allclose(face, t[k] / h[0], rtol=1e-14)
        rest = np.delete(f[k], m, axis=d - 1)
        assert np.all(rest == 0.0)
    # the box-face source of the box of m cells, traction t on x+
    small = (m,) + tuple(ncell[1:])
    kind, val = si._bc_table()
    val[1, :d] = t
    fA, _, _ = oracle.rhs(small, h, LAM, MU, np.ones(tuple(reversed(small))), kind, val)
    for k in range(d):
        assert np.allclose(f[k][inner + (m,)], fA[k][inner + (m,)], rtol=1e-14)
    fp = oracle.diffuse_traction(ncell, h, psi, 0.0, pressure=2.0)
    assert np.allclose(fp[0][inner + (m,)], -2.0 / h[0], rtol=1e-14)
    for k in range(1, d):
        assert np.all(fp[k][inner + (m,)] == 0.0)


def _compact_void(ncell, h, centre, a, w):
    cc = si.cell_centres(ncell, h)
    r = np.sqrt(sum((x - c) ** 2 for x, c in zip(cc, centre)))
    s = np.clip((r - a) / w, 0.0, 1.0)
    return s * s * (3.0 - 2.0 * s)   # exactly 1 beyond r = a + w, 0 inside r = a


@pytest.mark.parametrize("ncell", [(40, 43), (14, 12, 16)])
def test_pressure_on_a_closed_void_balances(ncell):
    d = len(ncell)
    h = (0.1, 0.12, 0.09)[:d]
    centre = (1.7, 2.3) if d == 2 else (0.7, 0.72, 0.7)
    a, w, p = (0.8, 0.5, 2.0) if d == 2 else (0.3, 0.25, 1.5)
    psi = _compact_void(ncell, h, centre, a, w)
    assert psi.min() == 0.0 and np.all(psi[0] == 1.0) and np.all(psi[-1] == 1.0)
    f = oracle.diffuse_traction(ncell, h, psi, 1e-6, pressure=p)
    X = si.node_coords(ncell, h)
    scale = np.abs(f).sum() * max(max(x.max() for x in X), 1.0)
    for k in range(d):
        assert abs(f[k].sum()) <= 1e-13 * scale                # no net force
    for i in range(d):
        for j in range(i + 1, d):
            tq = (X[i] * f[j] - X[j] * f[i]).sum()
            assert abs(tq) <= 1e-13 * scale                     # no net torque
    vol = np.prod(h)
    moment = sum((X[k] * f[k]).sum() for k in range(d)) * vol
    void = (1.0 - np.maximum(psi, 1e-6)).sum() * vol
    assert np.isclose(moment, p * d * void, rtol=1e-12)         # p d V (divergence theorem)


@pytest.mark.slow
def test_pressurised_hole_approaches_the_elastic_solution():
    """Quarter plate [0,16]^2 with rollers on x = 0 and y = 0, a hole of radius 1
    at the origin under pressure p, outer edges free: the radial displacement at
    1.5 <= r <= 2.5 approaches the thick-cylinder solution (outer radius 16)
    as the diffuse width shrinks."""
    L, a, p, n = 16.0, 1.0, 1e-3, 256
    h = L / n
    X, Y = si.cell_centres((n, n), (h, h))
    r = np.hypot(X, Y)
    kind, val = si._bc_table()
    kind[0, 0] = si.DISPLACEMENT
    kind[2, 1] = si.DISPLACEMENT
    Xn, Yn = si.node_coords((n, n), (h, h))
    rn = np.hypot(Xn, Yn)
    sel = (rn > 1.5 * a) & (rn < 2.5 * a)
    b = L
    B = p * a * a * b * b / (2 * MU * (b * b - a * a))
    A = p * a * a / (2 * (LAM + MU) * (b * b - a * a))
    exact = A * rn[sel] + B / rn[sel]
    errs = []
    for width in (0.25, 0.125):
        psi = 0.5 * (1 + np.tanh((r - a) / width))
        load = oracle.diffuse_traction((n, n), (h, h), psi, 1e-6, pressure=p)
        u, hist, st = oracle.solve((n, n), (h, h), LAM, MU, psi, 1e-6, kind, val, load,
                                   rtol=1e-10, max_cycles=300)
        assert st == 0
        ur = (u[0] * Xn + u[1] * Yn)[sel] / rn[sel]
        errs.append(np.linalg.norm(ur - exact) / np.linalg.norm(exact))
    assert errs[1] < errs[0] and errs[1] < 0.03, errs
