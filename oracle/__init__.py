"""FP64 CPU oracle for the SBM elasticity multigrid solve (arXiv:2212.02362).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library under
``paper_2212_02362_amd`` never does, and the two share no code.

The arithmetic lives in ``sbm_oracle.c`` (plain loops, IEEE double, built with
``-ffp-contract=off``); this module only loads it and marshals numpy arrays.
Every function cites the passage of the paper it follows in the C source.

Conventions: node vectors have shape ``(d, *nodes)`` in numpy order, i.e.
``(d, ny+1, nx+1)`` in 2D and ``(d, nz+1, ny+1, nx+1)`` in 3D (x fastest in
memory); cell scalars have shape ``(ny, nx)`` / ``(nz, ny, nx)``.  ``ncell``
is given as ``(nx, ny[, nz])``.  Boundary kinds/values are ``(6, 3)`` arrays
over faces x-, x+, y-, y+, z-, z+ and components.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TRACTION = 0
DISPLACEMENT = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _u8(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_u8p)


def _long3(nc):
    v = list(nc) + [0] * (3 - len(nc))
    return (ctypes.c_long * 3)(*v)


def _dbl3(h):
    v = list(h) + [1.0] * (3 - len(h))
    return (ctypes.c_double * 3)(*v)


def node_shape(ncell):
    return tuple(n + 1 for n in reversed(ncell))


def cell_shape(ncell):
    return tuple(reversed(ncell))


def _bc(kind, val):
    k = np.ascontiguousarray(kind, dtype=np.int32).reshape(6, 3)
    v = np.ascontiguousarray(val, dtype=np.float64).reshape(6, 3)
    return k, v


def apply(ncell, h, lam, mu, psi, u):
    """Ku by eq. K (node rows written out with the full C_ijkl tensor)."""
    d = len(ncell)
    psi = np.ascontiguousarray(psi, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    assert psi.shape == cell_shape(ncell) and u.shape == (d,) + node_shape(ncell)
    out = np.empty_like(u)
    lib().orc_apply(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                    _d(psi), _d(u), _d(out))
    return out


def diag(ncell, h, lam, mu, psi):
    d = len(ncell)
    psi = np.ascontiguousarray(psi, np.float64)
    out = np.empty((d,) + node_shape(ncell))
    lib().orc_diag(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                   _d(psi), _d(out))
    return out


def floor_psi(psi_raw, floor):
    return np.maximum(np.asarray(psi_raw, np.float64), floor)


def dirichlet(ncell, kind, val):
    """(mask uint8, uD) node vectors."""
    d = len(ncell)
    k, v = _bc(kind, val)
    mask = np.empty((d,) + node_shape(ncell), np.uint8)
    uD = np.empty((d,) + node_shape(ncell))
    lib().orc_dirichlet_mask(d, _long3(ncell), k.ctypes.data_as(_ip), _d(v), _u8(mask), _d(uD))
    return mask, uD


def rhs(ncell, h, lam, mu, psi, kind, val, b=None):
    """(fA, fB, uD): load with traction source, lifted load, prescribed values."""
    d = len(ncell)
    k, v = _bc(kind, val)
    psi = np.ascontiguousarray(psi, np.float64)
    shp = (d,) + node_shape(ncell)
    fA, fB, uD = np.empty(shp), np.empty(shp), np.empty(shp)
    bb = None if b is None else np.ascontiguousarray(b, np.float64)
    lib().orc_rhs(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                  _d(psi), k.ctypes.data_as(_ip), _d(v), _d(bb), _d(fA), _d(fB), _d(uD))
    return fA, fB, uD


def residual(ncell, h, lam, mu, psi, mask, u, f):
    d = len(ncell)
    out = np.empty((d,) + node_shape(ncell))
    lib().orc_residual(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                       _d(np.ascontiguousarray(psi, np.float64)), _u8(mask),
                       _d(np.ascontiguousarray(u, np.float64)),
                       _d(np.ascontiguousarray(f, np.float64)), _d(out))
    return out


def jacobi(ncell, h, lam, mu, psi, mask, omega, u, f):
    d = len(ncell)
    out = np.empty((d,) + node_shape(ncell))
    lib().orc_jacobi(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                     _d(np.ascontiguousarray(psi, np.float64)), _u8(mask), ctypes.c_double(omega),
                     _d(np.ascontiguousarray(u, np.float64)),
                     _d(np.ascontiguousarray(f, np.float64)), _d(out))
    return out


def rb_half(ncell, h, lam, mu, psi, mask, omega, colour, u, f):
    d = len(ncell)
    out = np.empty((d,) + node_shape(ncell))
    lib().orc_rb_half(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                      _d(np.ascontiguousarray(psi, np.float64)), _u8(mask), ctypes.c_double(omega),
                      int(colour), _d(np.ascontiguousarray(u, np.float64)),
                      _d(np.ascontiguousarray(f, np.float64)), _d(out))
    return out


def prolong_add(ncell_coarse, e, mask_fine, u_fine):
    d = len(ncell_coarse)
    u = np.array(u_fine, np.float64, copy=True, order="C")
    lib().orc_prolong_add(d, _long3(ncell_coarse), _d(np.ascontiguousarray(e, np.float64)),
                          _u8(mask_fine), _d(u))
    return u


def restrict(ncell_fine, r, mask_coarse):
    d = len(ncell_fine)
    ncc = tuple(n // 2 for n in ncell_fine)
    out = np.empty((d,) + node_shape(ncc))
    lib().orc_restrict(d, _long3(ncell_fine), _d(np.ascontiguousarray(r, np.float64)),
                       _u8(mask_coarse), _d(out))
    return out


def coarsen_psi(ncell_fine, psi):
    d = len(ncell_fine)
    ncc = tuple(n // 2 for n in ncell_fine)
    out = np.empty(cell_shape(ncc))
    lib().orc_coarsen_psi(d, _long3(ncell_fine), _d(np.ascontiguousarray(psi, np.float64)),
                          _d(out))
    return out


def amr_tags(ncell, h, psi, thresh):
    """Refinement tags of a level's (floored) cell psi."""
    psi = np.ascontiguousarray(psi, np.float64)
    tags = np.empty(psi.shape, np.uint8)
    lib().orc_amr_tags(len(ncell), _long3(ncell), _dbl3(h), _d(psi), ctypes.c_double(thresh),
                       _u8(tags))
    return tags


def cg(ncell, h, lam, mu, psi, mask, f, x0=None, rtol=1e-12, maxit=None):
    d = len(ncell)
    x = np.zeros((d,) + node_shape(ncell)) if x0 is None else np.array(x0, np.float64, copy=True)
    if maxit is None:
        maxit = 4 * int((mask == 0).sum())
    it = lib().orc_cg(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                      _d(np.ascontiguousarray(psi, np.float64)), _u8(mask),
                      _d(np.ascontiguousarray(f, np.float64)), _d(x), ctypes.c_double(rtol),
                      int(maxit))
    return x, it


def num_levels(ncell):
    return lib().orc_num_levels(len(ncell), _long3(ncell))


def solve(ncell, h, lam, mu, psi_raw, psi_floor, kind, val, b=None, *, smoother=0,
          omega=None, nu_pre=2, nu_post=2, rtol=1e-10, max_cycles=200, bottom_rtol=1e-12,
          bottom_max_iter=0, krylov=0, u0=None):
    """FP64 solve by V-cycles (krylov=0) or V-cycle-preconditioned flexible
    CG (krylov=1).  Returns (u, hist, status)."""
    d = len(ncell)
    if omega is None:
        omega = 1.0 if smoother == 0 else 0.8
    k, v = _bc(kind, val)
    u = np.zeros((d,) + node_shape(ncell)) if u0 is None else np.array(u0, np.float64, copy=True)
    hist = np.zeros(max_cycles + 1)
    ncyc = ctypes.c_int(0)
    bb = None if b is None else np.ascontiguousarray(b, np.float64)
    st = lib().orc_solve(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                         _d(np.ascontiguousarray(psi_raw, np.float64)), ctypes.c_double(psi_floor),
                         k.ctypes.data_as(_ip), _d(v), _d(bb), int(smoother),
                         ctypes.c_double(omega), int(nu_pre), int(nu_post), ctypes.c_double(rtol),
                         int(max_cycles), ctypes.c_double(bottom_rtol), int(bottom_max_iter),
                         int(krylov), _d(u), _d(hist), int(max_cycles + 1), ctypes.byref(ncyc))
    return u, hist[: ncyc.value + 1].copy(), st


def sensitivity(ncell, h, lam, mu, kind, val, u, adj, rho=None, psi_floor=0.0):
    """dL/dpsi per cell (or dL/drho when rho is given, psi = max(rho^3, floor))."""
    d = len(ncell)
    k, v = _bc(kind, val)
    g = np.empty(cell_shape(ncell))
    rr = None if rho is None else np.ascontiguousarray(rho, np.float64)
    lib().orc_sensitivity(d, _long3(ncell), _dbl3(h), ctypes.c_double(lam), ctypes.c_double(mu),
                          k.ctypes.data_as(_ip), _d(v), _d(np.ascontiguousarray(u, np.float64)),
                          _d(np.ascontiguousarray(adj, np.float64)), _d(rr),
                          ctypes.c_double(psi_floor), _d(g))
    return g


def plastic_source(ncell, h, lam, mu, psi, eps_p):
    """Nodal load -div(psi C eps_p) of a cell plastic strain (3D; eps_p of
    shape (6, nz, ny, nx), components xx, yy, zz, yz, xz, xy)."""
    fp = np.empty((3,) + node_shape(ncell))
    st = lib().orc_plastic_source(len(ncell), _long3(ncell), _dbl3(h), ctypes.c_double(lam),
                                  ctypes.c_double(mu), _d(np.ascontiguousarray(psi, np.float64)),
                                  _d(np.ascontiguousarray(eps_p, np.float64)), _d(fp))
    if st != 0:
        raise ValueError("plastic_source: 3D only")
    return fp


def return_map(ncell, h, lam, mu, sigma_y, hbar, theta, u, eps_p, alpha, beta):
    """One radial-return update of the cell state (eps_p, alpha, beta) for the
    displacement u; returns (eps_p, alpha, beta, cells that yielded)."""
    ep = np.array(eps_p, np.float64, copy=True, order="C")
    al = np.array(alpha, np.float64, copy=True, order="C")
    bt = np.array(beta, np.float64, copy=True, order="C")
    n = lib().orc_return_map(len(ncell), _long3(ncell), _dbl3(h), ctypes.c_double(lam),
                             ctypes.c_double(mu), ctypes.c_double(sigma_y), ctypes.c_double(hbar),
                             ctypes.c_double(theta), _d(np.ascontiguousarray(u, np.float64)),
                             _d(ep), _d(al), _d(bt))
    if n < 0:
        raise ValueError("return_map: 3D only")
    return ep, al, bt, n


def crack_drive(ncell, h, lam, mu, u, H):
    """Crack driving force (Sec. 3.2): returns (H updated to max(H, W0+), the
    cells held intact where W0+ < W0-) for the strain of u."""
    Hn = np.array(H, np.float64, copy=True, order="C")
    intact = np.empty(cell_shape(ncell), np.uint8)
    lib().orc_crack_drive(len(ncell), _long3(ncell), _dbl3(h), ctypes.c_double(lam),
                          ctypes.c_double(mu), _d(np.ascontiguousarray(u, np.float64)), _d(Hn),
                          _u8(intact))
    return Hn, intact


def phase_step(ncell, h, c, H, intact, Gc, xi, M, dt, eta=1e-4):
    """One explicit Ginzburg-Landau step of the crack field; returns
    (c_new, psi = g(c_new) + eta)."""
    c1 = np.empty(cell_shape(ncell))
    psi = np.empty(cell_shape(ncell))
    lib().orc_phase_step(len(ncell), _long3(ncell), _dbl3(h),
                         _d(np.ascontiguousarray(c, np.float64)),
                         _d(np.ascontiguousarray(H, np.float64)),
                         _u8(np.ascontiguousarray(intact, np.uint8)), ctypes.c_double(Gc),
                         ctypes.c_double(xi), ctypes.c_double(M), ctypes.c_double(dt),
                         ctypes.c_double(eta), _d(c1), _d(psi))
    return c1, psi


def diffuse_traction(ncell, h, psi_raw, floor, t_hat=None, pressure=0.0):
    """Load of a diffuse traction (Sec. 2.1, eq. SBMLinearElasticity):
    t_hat |grad psi| + pressure grad psi at every node (psi floored)."""
    d = len(ncell)
    f = np.empty((d,) + node_shape(ncell))
    th = None if t_hat is None else np.ascontiguousarray(t_hat, np.float64)
    lib().orc_diffuse_traction(d, _long3(ncell), _dbl3(h),
                               _d(np.ascontiguousarray(psi_raw, np.float64)),
                               ctypes.c_double(floor), _d(th) if th is not None else None,
                               ctypes.c_double(pressure), _d(f))
    return f


def assemble(ncell, h, lam, mu, psi):
    """Dense K (small grids only) built column by column from ``apply``."""
    d = len(ncell)
    shp = (d,) + node_shape(ncell)
    n = int(np.prod(shp))
    K = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        K[:, j] = apply(ncell, h, lam, mu, psi, e.reshape(shp)).ravel()
        e[j] = 0.0
    return K


# ------------------------------------------------------------------ BSAMR

def br_cluster(flags, eff):
    """Berger-Rigoutsos clustering of a block flag array (numpy axis order
    (z, y, x) or (y, x)): returns (flags of the blocks inside the accepted
    boxes, boxes as [(lo, hi)] with (x, y, z) block indices, inclusive)."""
    f = np.ascontiguousarray(flags, np.uint8)
    d = f.ndim
    nb = tuple(reversed(f.shape))
    out = np.empty_like(f)
    cap = int(f.size) + 1
    boxes = np.zeros(6 * cap, np.int64)
    L = lib()
    L.orc_br_cluster.restype = ctypes.c_long
    n = L.orc_br_cluster(d, _long3(nb), _u8(f), ctypes.c_double(eff), _u8(out),
                         boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), cap)
    bx = [(tuple(boxes[6 * i:6 * i + 3][:d]), tuple(boxes[6 * i + 3:6 * i + 6][:d]))
          for i in range(n)]
    return out, bx


class AmrProblem:
    """Oracle of the block-structured adaptive composite solve.  psi_levels
    are the raw indicators sampled at each level's cell centres (dense,
    level a has ncell0 * 2^a cells per axis)."""

    def __init__(self, ncell0, h0, lam, mu, psi_levels, psi_floor, kind, val, *, block=32,
                 thresh=0.05, smoother=0, omega=None, nu_pre=2, nu_post=2, bottom_rtol=1e-12,
                 bottom_max_iter=0, blocks=None, cluster_eff=0.0):
        L = lib()
        L.orc_amr_new.restype = ctypes.c_void_p
        L.orc_amr_fnorm.restype = ctypes.c_double
        L.orc_amr_residual.restype = ctypes.c_double
        self.dim = len(ncell0)
        self.A = len(psi_levels) - 1
        self.ncell0 = tuple(ncell0)
        self.h0 = tuple(h0)
        self.block = block
        if omega is None:
            omega = 1.0 if smoother == 0 else 0.8
        self._psi = [np.ascontiguousarray(p, np.float64) for p in psi_levels]
        for a, p in enumerate(self._psi):
            assert p.shape == cell_shape(self.ncell(a)), (a, p.shape)
        arr = (_dp * len(self._psi))(*[_d(p) for p in self._psi])
        k, v = _bc(kind, val)
        blk = None
        if blocks is not None:  # block flags of levels 1..A, shape (nbz, nby, nbx) each
            self._blk = [np.ascontiguousarray(b, np.uint8) for b in blocks]
            blk = (_u8p * len(self._blk))(*[_u8(b) for b in self._blk])
        self._ctx = L.orc_amr_new(self.dim, self.A, int(block), _long3(ncell0), _dbl3(h0),
                                  ctypes.c_double(lam), ctypes.c_double(mu), arr,
                                  ctypes.c_double(psi_floor), k.ctypes.data_as(_ip), _d(v),
                                  ctypes.c_double(thresh), int(smoother), ctypes.c_double(omega),
                                  int(nu_pre), int(nu_post), ctypes.c_double(bottom_rtol),
                                  int(bottom_max_iter), blk, ctypes.c_double(cluster_eff))

    def __del__(self):
        if getattr(self, "_ctx", None):
            lib().orc_amr_free(ctypes.c_void_p(self._ctx))
            self._ctx = None

    def ncell(self, a):
        return tuple(n << a for n in self.ncell0)

    def h(self, a):
        return tuple(x / (1 << a) for x in self.h0)

    def node_shape(self, a):
        return (self.dim,) + node_shape(self.ncell(a))

    def info(self, a):
        """(block flags, node classes, psi) of level a (flags/classes None at a = 0)."""
        nc = self.ncell(a)
        nb = (ctypes.c_long * 3)()
        psi = np.empty(cell_shape(nc))
        if a == 0:
            lib().orc_amr_info(ctypes.c_void_p(self._ctx), 0, None, None, _d(psi), nb)
            return None, None, psi
        nbl = tuple(n // self.block for n in nc)
        blk = np.empty(tuple(reversed(nbl)), np.uint8)
        cls = np.empty(node_shape(nc), np.uint8)
        lib().orc_amr_info(ctypes.c_void_p(self._ctx), a, _u8(blk), _u8(cls), _d(psi), nb)
        return blk, cls, psi

    def fnorm(self):
        return lib().orc_amr_fnorm(ctypes.c_void_p(self._ctx))

    def _ptrs(self, arrs):
        return (_dp * len(arrs))(*[_d(x) for x in arrs])

    def residual(self, u_levels, f_levels=None):
        """(composite residual per level, norm over the composite unknowns);
        the ghosts of u are refilled in place."""
        u = [np.ascontiguousarray(x, np.float64) for x in u_levels]
        r = [np.zeros(self.node_shape(a)) for a in range(self.A + 1)]
        f = None if f_levels is None else self._ptrs(
            [np.ascontiguousarray(x, np.float64) for x in f_levels])
        nrm = lib().orc_amr_residual(ctypes.c_void_p(self._ctx), self._ptrs(u), f, self._ptrs(r))
        return r, nrm, u

    def ghost_fill(self, a, xc, xf):
        xf = np.array(xf, np.float64, copy=True)
        lib().orc_amr_ghost_fill(ctypes.c_void_p(self._ctx), int(a),
                                 _d(np.ascontiguousarray(xc, np.float64)), _d(xf))
        return xf

    def solve(self, rtol=1e-10, max_cycles=200, u0=None):
        u = [np.zeros(self.node_shape(a)) if u0 is None else np.array(u0[a], np.float64, copy=True)
             for a in range(self.A + 1)]
        hist = np.zeros(max_cycles + 1)
        n = ctypes.c_int(0)
        st = lib().orc_amr_solve(ctypes.c_void_p(self._ctx), ctypes.c_double(rtol), int(max_cycles),
                                 self._ptrs(u), _d(hist), int(max_cycles + 1), ctypes.byref(n))
        return u, hist[: n.value + 1].copy(), st
