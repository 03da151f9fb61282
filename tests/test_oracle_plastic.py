"""Pins of the oracle's plastic-strain load and J2 radial return (Sec. 3.1).

The load -div(psi C eps_p) is tied to eq. K (a uniform eigenstrain is the
strain of a linear field), to global equilibrium (no net force) and to its
first moment (a closed form over the cells).  The return map is checked
against the properties the J2 update must have: no change below yield, the
consistency condition of the updated state, normality and plastic
incompressibility, the hardening rates of the flow rule, and the exact cell
strain of a linear displacement.
"""
import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)
VI = [0, 1, 2, 1, 0, 0]
VJ = [0, 1, 2, 2, 2, 1]


def _mat(v):
    """(6, ...) Voigt-ordered components -> (3, 3, ...) symmetric tensor."""
    m = np.empty((3, 3) + v.shape[1:])
    for q in range(6):
        m[VI[q], VJ[q]] = v[q]
        m[VJ[q], VI[q]] = v[q]
    return m


def _C_apply(e):
    tr = e[0, 0] + e[1, 1] + e[2, 2]
    out = 2.0 * MU * e
    for i in range(3):
        out[i, i] = out[i, i] + LAM * tr
    return out


def _psi(ncell, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, tuple(reversed(ncell)))
    p[p < 0.2] = 0.0
    return p


@pytest.mark.parametrize("ncell", [(4, 3, 5), (6, 5, 4)])
def test_uniform_eigenstrain_is_the_strain_of_a_linear_field(ncell):
    """fp = -div(psi C eps) for a uniform eps equals K applied to u = eps x at
    every node, box faces included."""
    h = (0.3, 0.25, 0.2)
    psi = _psi(ncell, 1)
    rng = np.random.default_rng(2)
    ev = rng.standard_normal(6)
    eps_p = np.broadcast_to(ev[:, None, None, None], (6,) + psi.shape).copy()
    E = _mat(ev)
    X = si.node_coords(ncell, h)
    u = np.stack([sum(E[k, l] * X[l] for l in range(3)) for k in range(3)])
    fp = oracle.plastic_source(ncell, h, LAM, MU, psi, eps_p)
    Ku = oracle.apply(ncell, h, LAM, MU, psi, u)
    assert np.max(np.abs(fp - Ku)) <= 1e-12 * np.max(np.abs(Ku))


def test_no_net_force_and_moment_is_the_cell_sum():
    """sum_n fp(n) = 0 and sum_n x_a(n) fp_i(n) = sum_c psi_c (C eps_p,c)_ia
    (symmetric: no net torque) for an arbitrary plastic strain field."""
    ncell, h = (5, 4, 6), (0.2, 0.3, 0.25)
    psi = _psi(ncell, 3)
    eps_p = np.random.default_rng(4).standard_normal((6,) + psi.shape)
    fp = oracle.plastic_source(ncell, h, LAM, MU, psi, eps_p)
    scale = np.abs(fp).max()
    assert np.all(np.abs(fp.reshape(3, -1).sum(axis=1)) <= 1e-12 * scale * fp[0].size)
    X = si.node_coords(ncell, h)
    M = np.array([[np.sum(X[a] * fp[i]) for i in range(3)] for a in range(3)])
    S = _C_apply(_mat(eps_p)) * psi[None, None]
    ref = S.reshape(3, 3, -1).sum(axis=2)
    assert np.allclose(M, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(M, M.T, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _state(shape, seed, scale=1e-3):
    rng = np.random.default_rng(seed)
    ep = rng.standard_normal((6,) + shape) * scale
    tr = ep[0] + ep[1] + ep[2]
    for q in range(3):
        ep[q] -= tr / 3.0  # plastic strain is deviatoric
    al = np.abs(rng.standard_normal(shape)) * scale
    bt = rng.standard_normal((6,) + shape) * scale * 0.1
    trb = bt[0] + bt[1] + bt[2]
    for q in range(3):
        bt[q] -= trb / 3.0
    return ep, al, bt


def _cell_strain_linear(E):
    return 0.5 * (E + E.T)


def test_cell_strain_of_a_linear_field_is_exact():
    """With sigma_Y = Hbar = 0 and a zero state every cell yields fully and
    eps_p becomes dev(eps): a linear u = E x exposes eps = sym(E) exactly."""
    ncell, h = (3, 4, 2), (0.5, 0.25, 0.4)
    E = np.random.default_rng(5).standard_normal((3, 3)) * 1e-2
    X = si.node_coords(ncell, h)
    u = np.stack([sum(E[k, l] * X[l] for l in range(3)) for k in range(3)])
    shape = tuple(reversed(ncell))
    z6 = np.zeros((6,) + shape)
    ep, al, bt, n = oracle.return_map(ncell, h, LAM, MU, 0.0, 0.0, 1.0, u, z6, np.zeros(shape), z6)
    assert n == np.prod(ncell)
    e = _cell_strain_linear(E)
    dev = e - np.trace(e) / 3.0 * np.eye(3)
    for q in range(6):
        assert np.allclose(ep[q], dev[VI[q], VJ[q]], rtol=1e-12, atol=1e-15)


def _eta(ncell, h, u, ep, bt):
    """Relative stress dev(C(eps - eps_p)) - beta per cell, with eps from the
    displacement of a linear-per-cell field (recomputed here from u by the
    cell gradient of the corner nodes)."""
    shape = tuple(reversed(ncell))
    G = np.zeros((3, 3) + shape)
    for k in range(3):
        uk = u[k]
        # d/dx (axis 2 in numpy order), d/dy (axis 1), d/dz (axis 0)
        dx = (uk[:, :, 1:] - uk[:, :, :-1]) / h[0]
        dy = (uk[:, 1:, :] - uk[:, :-1, :]) / h[1]
        dz = (uk[1:, :, :] - uk[:-1, :, :]) / h[2]
        G[k, 0] = 0.25 * (dx[:-1, :-1] + dx[:-1, 1:] + dx[1:, :-1] + dx[1:, 1:])
        G[k, 1] = 0.25 * (dy[:-1, :, :-1] + dy[:-1, :, 1:] + dy[1:, :, :-1] + dy[1:, :, 1:])
        G[k, 2] = 0.25 * (dz[:, :-1, :-1] + dz[:, :-1, 1:] + dz[:, 1:, :-1] + dz[:, 1:, 1:])
    eps = 0.5 * (G + G.transpose(1, 0, *range(2, G.ndim)))
    ee = eps - _mat(ep)
    tr = ee[0, 0] + ee[1, 1] + ee[2, 2]
    s = 2.0 * MU * ee
    for i in range(3):
        s[i, i] -= 2.0 * MU * tr / 3.0
    return s - _mat(bt)


@pytest.mark.parametrize("theta", [1.0, 0.3])
def test_return_map_properties(theta):
    ncell, h = (4, 5, 3), (0.25, 0.2, 0.3)
    shape = tuple(reversed(ncell))
    rng = np.random.default_rng(6)
    u = rng.standard_normal((3,) + tuple(n + 1 for n in reversed(ncell))) * 2e-3
    ep0, al0, bt0 = _state(shape, 7)
    hb = 0.05
    eta0 = _eta(ncell, h, u, ep0, bt0)
    nrm0 = np.sqrt(np.einsum("ij...,ij...->...", eta0, eta0))
    # yield strength at the median trial state: about half of the cells yield
    sy = float(np.median(nrm0 / np.sqrt(2 / 3) - theta * hb * al0))
    ep, al, bt, n = oracle.return_map(ncell, h, LAM, MU, sy, hb, theta, u, ep0, al0, bt0)
    f0 = nrm0 - np.sqrt(2 / 3) * (sy + theta * hb * al0)
    yielded = f0 > 0
    assert n == int(yielded.sum()) and 0 < n < yielded.size
    # below yield: nothing changes
    assert np.array_equal(ep[:, ~yielded], ep0[:, ~yielded])
    assert np.array_equal(al[~yielded], al0[~yielded]) and np.array_equal(bt[:, ~yielded], bt0[:, ~yielded])
    # consistency of the updated state, and no cell left above yield
    eta1 = _eta(ncell, h, u, ep, bt)
    nrm1 = np.sqrt(np.einsum("ij...,ij...->...", eta1, eta1))
    f1 = nrm1 - np.sqrt(2 / 3) * (sy + theta * hb * al)
    assert np.all(np.abs(f1[yielded]) <= 1e-10 * nrm1[yielded])
    assert np.all(f1 <= 1e-10 * np.abs(nrm1).max())
    # normality (increment along the updated relative stress), incompressibility
    dep = _mat(ep - ep0)
    ndep = np.sqrt(np.einsum("ij...,ij...->...", dep, dep))
    cosang = np.einsum("ij...,ij...->...", dep, eta1) / (ndep * nrm1 + 1e-300)
    assert np.all(np.abs(cosang[yielded] - 1.0) <= 1e-10)
    assert np.all(np.abs((dep[0, 0] + dep[1, 1] + dep[2, 2])[yielded]) <= 1e-12 * ndep.max())
    # hardening rates of the flow rule
    assert np.allclose((al - al0)[yielded], np.sqrt(2 / 3) * ndep[yielded], rtol=1e-12, atol=0)
    assert np.allclose(bt - bt0, (2 / 3) * (1 - theta) * hb * (ep - ep0), rtol=1e-12, atol=1e-18)


def test_uniaxial_shear_closed_form():
    """Simple shear eps_xy = g/2 of a virgin cell (theta = 1): |eta| = sqrt(2)
    mu g, so dgamma = (sqrt(2) mu g - sqrt(2/3) sigma_Y) / (2 mu + 2 Hbar / 3)
    and eps_p,xy = dgamma / sqrt(2)."""
    ncell, h = (1, 1, 1), (1.0, 1.0, 1.0)
    g = 0.01
    X = si.node_coords(ncell, h)
    u = np.stack([g * X[1], np.zeros_like(X[0]), np.zeros_like(X[0])])
    z6, z1 = np.zeros((6, 1, 1, 1)), np.zeros((1, 1, 1))
    sy, hb = 1e-3, 0.2
    ep, al, bt, n = oracle.return_map(ncell, h, LAM, MU, sy, hb, 1.0, u, z6, z1, z6)
    dg = (np.sqrt(2) * MU * g - np.sqrt(2 / 3) * sy) / (2 * MU + 2 * hb / 3)
    assert n == 1
    assert abs(ep[5, 0, 0, 0] - dg / np.sqrt(2)) <= 1e-14
    assert np.all(ep[:5] == 0.0)
    assert abs(al[0, 0, 0] - np.sqrt(2 / 3) * dg) <= 1e-15
