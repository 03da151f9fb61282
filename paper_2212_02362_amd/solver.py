"""Python face of the C ABI: a ``Solver`` that owns one library context.

PyTorch supplies the device memory (the workspace is a uint8 tensor) and the
stream (the current torch stream); every arithmetic step runs in the HIP
library.  Array conventions follow include/sbm.h: cells ``(ny, nx)`` /
``(nz, ny, nx)``, node vectors ``(d, ny+1, nx+1)`` / ``(d, nz+1, ny+1, nx+1)``,
``ncell = (nx, ny[, nz])``, boundary tables ``(6, 3)`` over faces
x-, x+, y-, y+, z-, z+.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import (SbmJ2, SbmPf, CHAIN_FLOOR, CHAIN_PSI, CHAIN_RHO3, DISPLACEMENT, SBM_NOT_CONVERGED, SBM_OK,
                   TRACTION, SbmBc, SbmError, SbmGrid, SbmMaterial, SbmOptions, check, lib)

__all__ = ["Solver", "SbmError", "TRACTION", "DISPLACEMENT"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Solver:
    """One grid, one workspace, one library context.

    Options (the paper leaves them open): ``smoother`` 0 two-colour
    Gauss-Seidel / 1 damped Jacobi, ``omega`` (0 = default for the smoother),
    ``nu_pre``/``nu_post``, ``precision`` 0 FP64 / 1 FP32 cycles with FP64
    refinement, ``rtol``, ``max_cycles``, ``bottom_rtol``, ``bottom_max_iter``.
    """

    def __init__(self, ncell: Sequence[int], h: Sequence[float], *, device=None, stream=None,
                 **options):
        self.dim = len(ncell)
        if self.dim not in (2, 3):
            raise ValueError("ncell must have 2 or 3 entries")
        self.ncell = tuple(int(n) for n in ncell)
        self.h = tuple(float(x) for x in h)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the SBM library runs on a HIP device only")
        L = lib()
        g = SbmGrid()
        g.dim = self.dim
        for a in range(3):
            g.ncell[a] = self.ncell[a] if a < self.dim else 0
            g.h[a] = self.h[a] if a < self.dim else 1.0
        self._grid = g
        self._opts = SbmOptions()
        L.sbm_default_options(ctypes.byref(self._opts))
        self._apply_options(options)
        nbytes = L.sbm_workspace_bytes(ctypes.byref(g), ctypes.byref(self._opts))
        if nbytes == 0:
            raise SbmError(-2, f"invalid grid {self.ncell} / options")
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        ctx = ctypes.c_void_p()
        check(L.sbm_create(ctypes.byref(g), ctypes.byref(self._opts), ctypes.c_void_p(aligned),
                           self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                           ctypes.byref(ctx)))
        self._ctx = ctx
        self.nlevels = L.sbm_num_levels(ctypes.byref(g))
        self.problem = None

    # ------------------------------------------------------------ plumbing
    def _apply_options(self, options):
        for k, v in options.items():
            if not hasattr(self._opts, k):
                raise TypeError(f"unknown option {k}")
            setattr(self._opts, k, v)

    def set_options(self, **options):
        self._apply_options(options)
        check(lib().sbm_set_options(self._ctx, ctypes.byref(self._opts)))

    @property
    def options(self):
        return {name: getattr(self._opts, name) for name, _ in SbmOptions._fields_}

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                lib().sbm_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass

    @property
    def node_shape(self):
        return tuple(n + 1 for n in reversed(self.ncell))

    @property
    def cell_shape(self):
        return tuple(reversed(self.ncell))

    def _dev(self, a, dtype=torch.float64, shape=None):
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=dtype, device=self.device)
        if not t.is_contiguous():
            t = t.contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def new_nodes(self, dtype=torch.float64):
        return torch.zeros((self.dim,) + self.node_shape, dtype=dtype, device=self.device)

    def new_cells(self, dtype=torch.float64):
        return torch.zeros(self.cell_shape, dtype=dtype, device=self.device)

    def level_shape(self, level):
        nc = (ctypes.c_int64 * 3)()
        check(lib().sbm_level_shape(self._ctx, int(level), nc))
        return tuple(int(nc[a]) for a in range(self.dim))

    # -------------------------------------------------------------- problem
    def set_problem(self, psi_raw, lam, mu, psi_floor, kind, val, b=None, *, density=False):
        """Problem data (Sec. 2.1): raw cell indicator, Lame constants, floor,
        boundary table, optional node body force.  With density=True the cell
        field is a density rho and the library takes psi_raw = rho^3."""
        psi_t = self._dev(psi_raw, shape=self.cell_shape)
        b_t = self._dev(b, shape=(self.dim,) + self.node_shape)
        kind = np.asarray(kind).reshape(6, 3)
        val = np.asarray(val, dtype=np.float64).reshape(6, 3)
        bc = SbmBc()
        for F in range(6):
            for k in range(3):
                bc.kind[F][k] = int(kind[F, k])
                bc.value[F][k] = float(val[F, k])
        m = SbmMaterial(float(lam), float(mu), float(psi_floor))
        with torch.cuda.device(self.device):
            fn = lib().sbm_set_problem_density if density else lib().sbm_set_problem
            check(fn(self._ctx, _ptr(psi_t), ctypes.byref(m), ctypes.byref(bc), _ptr(b_t)))
        self.problem = dict(lam=float(lam), mu=float(mu), psi_floor=float(psi_floor),
                            kind=kind.copy(), val=val.copy())
        self._psi_ref, self._b_ref = psi_t, b_t  # inputs are copied by the library; kept for reuse
        return self

    def set_problem_from(self, p):
        """Takes an ``sbm_inputs.Problem``."""
        return self.set_problem(p.psi_raw, p.lam, p.mu, p.psi_floor, p.kind, p.val, p.b)

    # ---------------------------------------------------------------- solve
    def solve(self, u0=None, hist_cap=None, allow_not_converged=True):
        """Returns (u, hist, status): u on the device, the relative residual
        history rho_0..rho_m (numpy) and the status code."""
        u = self.new_nodes() if u0 is None else self._dev(u0, shape=(self.dim,) + self.node_shape).clone()
        cap = int(hist_cap or (self._opts.max_cycles + 1))
        hist = (ctypes.c_double * cap)()
        ncyc = ctypes.c_int(0)
        fin = ctypes.c_double(0.0)
        with torch.cuda.device(self.device):
            st = lib().sbm_solve(self._ctx, _ptr(u), hist, cap, ctypes.byref(ncyc), ctypes.byref(fin))
        check(st, (SBM_OK, SBM_NOT_CONVERGED) if allow_not_converged else (SBM_OK,))
        return u, np.array(hist[: min(cap, ncyc.value + 1)]), st

    def solve_rhs(self, g, x0=None, hist_cap=None, allow_not_converged=True):
        """Solves K x = g on the free DOF with x = 0 on displacement DOF."""
        g_t = self._dev(g, shape=(self.dim,) + self.node_shape)
        x = self.new_nodes() if x0 is None else self._dev(x0, shape=(self.dim,) + self.node_shape).clone()
        cap = int(hist_cap or (self._opts.max_cycles + 1))
        hist = (ctypes.c_double * cap)()
        ncyc = ctypes.c_int(0)
        fin = ctypes.c_double(0.0)
        with torch.cuda.device(self.device):
            st = lib().sbm_solve_rhs(self._ctx, _ptr(g_t), _ptr(x), hist, cap, ctypes.byref(ncyc),
                                     ctypes.byref(fin))
        check(st, (SBM_OK, SBM_NOT_CONVERGED) if allow_not_converged else (SBM_OK,))
        return x, np.array(hist[: min(cap, ncyc.value + 1)]), st

    def apply(self, u, out=None):
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        out = self.new_nodes() if out is None else out
        check(lib().sbm_apply(self._ctx, _ptr(u_t), _ptr(out)))
        return out

    def residual(self, u, want_r=True):
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        r = self.new_nodes() if want_r else None
        nrm = ctypes.c_double(0.0)
        check(lib().sbm_residual(self._ctx, _ptr(u_t), _ptr(r), ctypes.byref(nrm)))
        return r, nrm.value

    def rhs(self):
        fA, fB = self.new_nodes(), self.new_nodes()
        check(lib().sbm_rhs(self._ctx, _ptr(fA), _ptr(fB)))
        return fA, fB

    def sensitivity(self, u, lam, *, lam_scale=1.0, design=None, chain=CHAIN_PSI):
        """dL/dpsi per cell (chain CHAIN_PSI), masked by the floor against the
        raw psi given as design (CHAIN_FLOOR), or dL/drho for psi = rho^3
        with design = rho (CHAIN_RHO3)."""
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        l_t = self._dev(lam, shape=(self.dim,) + self.node_shape)
        d_t = self._dev(design, shape=self.cell_shape)
        g = self.new_cells()
        check(lib().sbm_sensitivity(self._ctx, _ptr(u_t), _ptr(l_t), float(lam_scale), _ptr(d_t),
                                    int(chain), _ptr(g)))
        return g

    # ------------------------------------------------- plastic strain (J2)
    def plastic_source(self, eps_p, out=None):
        """Nodal load -div(psi C eps_p) of a cell plastic strain (3D; eps_p
        of shape (6, nz, ny, nx), components xx, yy, zz, yz, xz, xy)."""
        e_t = self._dev(eps_p, shape=(6,) + self.cell_shape)
        out = self.new_nodes() if out is None else out
        check(lib().sbm_plastic_source(self._ctx, _ptr(e_t), _ptr(out)))
        return out

    def return_map(self, u, eps_p, alpha, beta, sigma_y, hbar, theta, *, inplace=False):
        """J2 radial return of the cell state for the strain of u.  Returns
        (eps_p, alpha, beta, number of yielding cells); with inplace=True the
        given device tensors (float64, contiguous) are updated and returned."""
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        state = []
        for a, shp in ((eps_p, (6,) + self.cell_shape), (alpha, self.cell_shape),
                       (beta, (6,) + self.cell_shape)):
            t = self._dev(a, shape=shp)
            if inplace:
                if t is not a:
                    raise ValueError("inplace needs contiguous float64 tensors on the solver's device")
            else:
                t = t.clone()
            state.append(t)
        m = SbmJ2(float(sigma_y), float(hbar), float(theta))
        n = ctypes.c_int64(0)
        check(lib().sbm_return_map(self._ctx, _ptr(u_t), ctypes.byref(m), _ptr(state[0]),
                                   _ptr(state[1]), _ptr(state[2]), ctypes.byref(n)))
        return state[0], state[1], state[2], int(n.value)

    # ---------------------------------------------------- diffuse traction
    def diffuse_traction(self, psi_raw, psi_floor, t_hat=None, pressure=0.0, out=None):
        """Node load t_hat |grad psi| + pressure grad psi of a traction on the
        diffuse boundary (psi = max(psi_raw, psi_floor)); pass it as b."""
        p_t = self._dev(psi_raw, shape=self.cell_shape)
        t_t = self._dev(t_hat, shape=(self.dim,) + self.node_shape)
        if out is None:
            out = torch.empty((self.dim,) + self.node_shape, dtype=torch.float64,
                              device=self.device)
        elif self._dev(out, shape=(self.dim,) + self.node_shape) is not out:
            raise ValueError("out: a contiguous float64 node tensor on the solver's device")
        check(lib().sbm_diffuse_traction(self._ctx, _ptr(p_t), float(psi_floor), _ptr(t_t),
                                         float(pressure), _ptr(out)))
        return out

    # ------------------------------------------------ phase-field fracture
    def crack_drive(self, u, H, *, inplace=False):
        """Crack driving force: returns (H updated to max(H, W0+), intact
        cells as uint8) for the strain of u."""
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        h_t = self._dev(H, shape=self.cell_shape)
        if inplace and h_t is not H:
            raise ValueError("inplace needs a contiguous float64 tensor on the solver's device")
        if not inplace:
            h_t = h_t.clone()
        intact = torch.empty(self.cell_shape, dtype=torch.uint8, device=self.device)
        check(lib().sbm_crack_drive(self._ctx, _ptr(u_t), _ptr(h_t), _ptr(intact)))
        return h_t, intact

    def phase_step(self, c, H, intact, Gc, xi, M, dt, eta=1e-4, out=None):
        """One explicit Ginzburg-Landau step of the crack field; returns
        (c_new, psi = g(c_new) + eta), written into ``out`` = (c_new, psi)
        when given (contiguous float64 cell tensors on the solver's device,
        c_new not aliasing c)."""
        c_t = self._dev(c, shape=self.cell_shape)
        h_t = self._dev(H, shape=self.cell_shape)
        i_t = self._dev(intact, dtype=torch.uint8, shape=self.cell_shape)
        if out is None:
            c1 = torch.empty(self.cell_shape, dtype=torch.float64, device=self.device)
            psi = torch.empty_like(c1)
        else:
            c1, psi = (self._dev(o, shape=self.cell_shape) for o in out)
            if c1 is not out[0] or psi is not out[1]:
                raise ValueError("out: contiguous float64 tensors on the solver's device")
        pf = SbmPf(float(Gc), float(xi), float(M), float(dt), float(eta))
        check(lib().sbm_phase_step(self._ctx, _ptr(c_t), _ptr(h_t), _ptr(i_t), ctypes.byref(pf),
                                   _ptr(c1), _ptr(psi)))
        return c1, psi

    def compliance(self, u):
        """J = h^d sum over free DOF of f.u."""
        u_t = self._dev(u, shape=(self.dim,) + self.node_shape)
        J = ctypes.c_double(0.0)
        check(lib().sbm_compliance(self._ctx, _ptr(u_t), ctypes.byref(J)))
        return J.value

    # ------------------------------------------------------- live timing
    def profile(self, enable=True):
        check(lib().sbm_profile(self._ctx, int(bool(enable))))

    def profile_read(self):
        """{class: (total_ms, launches)} of the finest-level launches timed
        with HIP events since profile(True)."""
        from ._lib import PROF_CLASSES
        n = len(PROF_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(lib().sbm_profile_read(self._ctx, ms, cnt))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(PROF_CLASSES)}

    def graph_info(self):
        """(captures, graph launches) of the V-cycle graphs of this context."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        check(lib().sbm_graph_info(self._ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # ----------------------------------------------------- component steps
    def _level_nodes(self, level, dtype=torch.float64):
        nc = self.level_shape(level)
        return torch.zeros((self.dim,) + tuple(n + 1 for n in reversed(nc)), dtype=dtype,
                           device=self.device)

    def level_psi(self, level):
        nc = self.level_shape(level)
        out = torch.zeros(tuple(reversed(nc)), dtype=torch.float64, device=self.device)
        check(lib().sbm_level_psi(self._ctx, int(level), _ptr(out)))
        return out

    def level_apply(self, level, u):
        u_t = self._dev(u)
        out = torch.empty_like(u_t)
        check(lib().sbm_level_apply(self._ctx, int(level), _ptr(u_t), _ptr(out)))
        return out

    def level_apply_f32(self, level, u):
        u_t = self._dev(u, dtype=torch.float32)
        out = torch.empty_like(u_t)
        check(lib().sbm_level_apply_f32(self._ctx, int(level), _ptr(u_t), _ptr(out)))
        return out

    def level_smooth(self, level, colour, omega, u, f):
        u_t, f_t = self._dev(u), self._dev(f)
        out = torch.empty_like(u_t)
        check(lib().sbm_level_smooth(self._ctx, int(level), int(colour), float(omega), _ptr(u_t),
                                     _ptr(f_t), _ptr(out)))
        return out

    def level_sweep(self, level, first_colour, omega, u, f, fp32=False):
        """One two-colour Gauss-Seidel sweep on `level` (u None: a zero iterate)."""
        dt = torch.float32 if fp32 else torch.float64
        shp = (self.dim,) + tuple(n + 1 for n in reversed(self.level_shape(level)))
        f_t = self._dev(f, dtype=dt, shape=shp)
        u_t = None if u is None else self._dev(u, dtype=dt, shape=shp)
        out = torch.empty_like(f_t)
        fn = lib().sbm_level_sweep_f32 if fp32 else lib().sbm_level_sweep
        check(fn(self._ctx, int(level), int(first_colour), float(omega),
                 None if u_t is None else _ptr(u_t), _ptr(f_t), _ptr(out)))
        return out

    def level_residual(self, level, u, f):
        u_t, f_t = self._dev(u), self._dev(f)
        out = torch.empty_like(u_t)
        check(lib().sbm_level_residual(self._ctx, int(level), _ptr(u_t), _ptr(f_t), _ptr(out)))
        return out

    def level_restrict(self, level, r):
        r_t = self._dev(r)
        out = self._level_nodes(level + 1)
        check(lib().sbm_level_restrict(self._ctx, int(level), _ptr(r_t), _ptr(out)))
        return out

    def level_prolong_add(self, level, e, u):
        e_t = self._dev(e)
        out = self._dev(u).clone()
        check(lib().sbm_level_prolong_add(self._ctx, int(level), _ptr(e_t), _ptr(out)))
        return out

    def bottom_solve(self, f, x0=None):
        f_t = self._dev(f)
        x = torch.zeros_like(f_t) if x0 is None else self._dev(x0).clone()
        it = ctypes.c_int(0)
        check(lib().sbm_bottom_solve(self._ctx, _ptr(f_t), _ptr(x), ctypes.byref(it)))
        return x, it.value


def stream_triad(a, b, c, s):
    """a = b + s c on device float64 tensors through the library's bandwidth
    probe kernel, enqueued on the current stream."""
    for t in (a, b, c):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("stream_triad needs contiguous float64 device tensors")
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("stream_triad arrays differ in size")
    st = torch.cuda.current_stream(a.device)
    check(lib().sbm_stream_triad(_ptr(a), _ptr(b), _ptr(c), a.numel(), float(s),
                                 ctypes.c_void_p(st.cuda_stream)))


def residual_static(ncell, h, lam, mu, kind, psi, u, f, want_r=True):
    """r = f - K u on free DOF and ||r|| without a solver context (the
    library's allocation-free entry point): psi the floored cell indicator,
    u and f node tensors on the current device; returns (r or None, norm)."""
    d = len(ncell)
    g = SbmGrid()
    g.dim = d
    for a in range(3):
        g.ncell[a] = int(ncell[a]) if a < d else 0
        g.h[a] = float(h[a]) if a < d else 1.0
    kind = np.asarray(kind).reshape(6, 3)
    bc = SbmBc()
    for F in range(6):
        for k in range(3):
            bc.kind[F][k] = int(kind[F, k])
    m = SbmMaterial(float(lam), float(mu), 0.0)
    node = (d,) + tuple(int(n) + 1 for n in reversed(ncell))
    cell = tuple(int(n) for n in reversed(ncell))
    ts = []
    for t, shp in ((psi, cell), (u, node), (f, node)):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape) != shp:
            raise ValueError(f"expected a contiguous float64 device tensor of shape {shp}")
        ts.append(t)
    r = torch.empty_like(u) if want_r else None
    nrm = ctypes.c_double(0.0)
    st = torch.cuda.current_stream(u.device)
    check(lib().sbm_residual_static(ctypes.byref(g), ctypes.byref(m), ctypes.byref(bc),
                                    _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2]), _ptr(r),
                                    ctypes.byref(nrm), ctypes.c_void_p(st.cuda_stream)))
    return r, nrm.value

