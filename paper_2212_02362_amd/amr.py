"""Python face of the adaptive composite solve (``sbm_amr_*`` in include/sbm.h).

Every level is a dense torch tensor in the library's layouts: cells
``(nz, ny, nx)`` and node vectors ``(d, nz+1, ny+1, nx+1)`` with level ``a``
holding ``ncell0 * 2**a`` cells per axis.  Per-level arguments are lists with
one entry per level (block flags: one per refined level).  Only argument
marshalling happens here; every step runs in the HIP library.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import SBM_NOT_CONVERGED, SBM_OK, SbmBc, SbmError, SbmGrid, SbmMaterial, SbmOptions, check, lib

__all__ = ["AmrSolver"]

_P = ctypes.c_void_p


def _ptr_array(tensors):
    arr = (_P * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def cluster_blocks(flags, efficiency):
    """Berger-Rigoutsos clustering of a uint8 block-flag array (numpy axis
    order (z, y, x) or (y, x)) on the host, by the library's own routine."""
    f = np.ascontiguousarray(flags, np.uint8)
    if f.ndim not in (2, 3):
        raise ValueError("flags must be 2D or 3D")
    nb = (ctypes.c_int64 * 3)(*(list(reversed(f.shape)) + [1] * (3 - f.ndim)))
    out = np.empty_like(f)
    check(lib().sbm_amr_cluster(f.ndim, ctypes.cast(nb, _P), f.ctypes.data_as(_P),
                                float(efficiency), out.ctypes.data_as(_P)))
    return out


class AmrSolver:
    """Base grid ``ncell0`` with spacing ``h0``, ``levels`` AMR levels (base
    included, refinement ratio 2) and cubic blocks of ``block`` cells.
    Options as for :class:`Solver` (``krylov`` must stay 0)."""

    def __init__(self, ncell0: Sequence[int], h0: Sequence[float], levels: int, block: int = 32, *,
                 device=None, stream=None, **options):
        self.dim = len(ncell0)
        self.ncell0 = tuple(int(n) for n in ncell0)
        self.h0 = tuple(float(x) for x in h0)
        self.levels = int(levels)
        self.block = int(block)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the SBM library runs on a HIP device only")
        L = lib()
        g = SbmGrid()
        g.dim = self.dim
        for a in range(3):
            g.ncell[a] = self.ncell0[a] if a < self.dim else 0
            g.h[a] = self.h0[a] if a < self.dim else 1.0
        self._grid = g
        self._opts = SbmOptions()
        L.sbm_default_options(ctypes.byref(self._opts))
        for k, v in options.items():
            if not hasattr(self._opts, k):
                raise TypeError(f"unknown option {k}")
            setattr(self._opts, k, v)
        nbytes = L.sbm_amr_workspace_bytes(ctypes.byref(g), self.levels, self.block,
                                           ctypes.byref(self._opts))
        if nbytes == 0:
            raise SbmError(-2, f"unsupported adaptive layout {self.ncell0} x {self.levels} levels, "
                               f"block {self.block}")
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        ctx = _P()
        check(L.sbm_amr_create(ctypes.byref(g), self.levels, self.block, ctypes.byref(self._opts),
                               _P(aligned), self.workspace_bytes, _P(self.stream.cuda_stream),
                               ctypes.byref(ctx)))
        self._ctx = ctx
        self.problem = None

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                lib().sbm_amr_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass

    def set_clustering(self, efficiency):
        """Berger-Rigoutsos clustering of the tagged blocks at the next
        ``set_problem`` without ``blocks`` (0 turns it off)."""
        check(lib().sbm_amr_set_clustering(self._ctx, float(efficiency)))
        return self

    def set_options(self, **options):
        for k, v in options.items():
            if not hasattr(self._opts, k):
                raise TypeError(f"unknown option {k}")
            setattr(self._opts, k, v)
        check(lib().sbm_amr_set_options(self._ctx, ctypes.byref(self._opts)))

    # ------------------------------------------------------------- shapes
    def ncell(self, a):
        return tuple(n << a for n in self.ncell0)

    def h(self, a):
        return tuple(x / (1 << a) for x in self.h0)

    def node_shape(self, a):
        return (self.dim,) + tuple(n + 1 for n in reversed(self.ncell(a)))

    def cell_shape(self, a):
        return tuple(reversed(self.ncell(a)))

    def _dev(self, x, shape, dtype=torch.float64):
        t = torch.as_tensor(x, dtype=dtype, device=self.device).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------ problem
    def set_problem(self, psi_levels, lam, mu, psi_floor, kind, val, *, thresh=0.05, blocks=None):
        """Raw indicators per level (cell centres of each level), Lame
        constants, floor, boundary table; refinement by tags at ``thresh`` or
        by the given block flags of the refined levels."""
        if len(psi_levels) != self.levels:
            raise ValueError(f"need {self.levels} psi arrays")
        psi_t = [self._dev(p, self.cell_shape(a)) for a, p in enumerate(psi_levels)]
        kind = np.asarray(kind).reshape(6, 3)
        val = np.asarray(val, dtype=np.float64).reshape(6, 3)
        bc = SbmBc()
        for F in range(6):
            for k in range(3):
                bc.kind[F][k] = int(kind[F, k])
                bc.value[F][k] = float(val[F, k])
        m = SbmMaterial(float(lam), float(mu), float(psi_floor))
        blk_arr = None
        self._blk_in = None
        if blocks is not None:
            if len(blocks) != self.levels - 1:
                raise ValueError(f"need {self.levels - 1} block-flag arrays")
            self._blk_in = [np.ascontiguousarray(b, np.uint8) for b in blocks]
            blk_arr = (_P * len(self._blk_in))(*[b.ctypes.data for b in self._blk_in])
        with torch.cuda.device(self.device):
            check(lib().sbm_amr_set_problem(self._ctx, _ptr_array(psi_t), ctypes.byref(m),
                                            ctypes.byref(bc), ctypes.c_double(float(thresh)),
                                            blk_arr))
        self.problem = dict(lam=float(lam), mu=float(mu), psi_floor=float(psi_floor),
                            kind=kind.copy(), val=val.copy())
        return self

    def level_info(self, a):
        """(block flags as numpy (None at a = 0), node classes as a uint8
        tensor (None at a = 0), floored and averaged-down psi tensor)."""
        nc = (ctypes.c_int64 * 3)()
        nb = (ctypes.c_int64 * 3)()
        check(lib().sbm_amr_level_info(self._ctx, int(a), nc, nb, None, None, None))
        psi = torch.empty(self.cell_shape(a), dtype=torch.float64, device=self.device)
        if a == 0:
            check(lib().sbm_amr_level_info(self._ctx, 0, None, None, None, None, _P(psi.data_ptr())))
            return None, None, psi
        nbl = tuple(int(nb[x]) for x in range(self.dim))
        blk = np.empty(tuple(reversed(nbl)), np.uint8)
        cls = torch.empty(self.node_shape(a)[1:], dtype=torch.uint8, device=self.device)
        check(lib().sbm_amr_level_info(self._ctx, int(a), None, None, blk.ctypes.data_as(_P),
                                       _P(cls.data_ptr()), _P(psi.data_ptr())))
        return blk, cls, psi

    def stats(self):
        """(composite unknowns, norm of the lifted load)."""
        n = ctypes.c_int64()
        f = ctypes.c_double()
        check(lib().sbm_amr_stats(self._ctx, ctypes.byref(n), ctypes.byref(f)))
        return int(n.value), float(f.value)

    def new_levels(self):
        return [torch.zeros(self.node_shape(a), dtype=torch.float64, device=self.device)
                for a in range(self.levels)]

    def profile(self, enable=True):
        check(lib().sbm_amr_profile(self._ctx, int(bool(enable))))

    def profile_read(self):
        """{class: (total_ms, launches)} of the finest-level launches timed
        with HIP events since profile(True)."""
        from ._lib import PROF_CLASSES
        n = len(PROF_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(lib().sbm_amr_profile_read(self._ctx, ms, cnt))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(PROF_CLASSES)}

    # ---------------------------------------------------------- operators
    def ghost_fill(self, a, xc, xf):
        xc_t = self._dev(xc, self.node_shape(a - 1))
        xf_t = self._dev(xf, self.node_shape(a)).clone()
        check(lib().sbm_amr_ghost_fill(self._ctx, int(a), _P(xc_t.data_ptr()), _P(xf_t.data_ptr())))
        return xf_t

    def residual(self, u_levels):
        """(composite residual per level, its norm); ghosts of the given
        tensors are refilled in place."""
        u = [self._dev(x, self.node_shape(a)) for a, x in enumerate(u_levels)]
        r = self.new_levels()
        nrm = ctypes.c_double()
        check(lib().sbm_amr_residual(self._ctx, _ptr_array(u), _ptr_array(r), ctypes.byref(nrm)))
        return r, float(nrm.value), u

    def solve(self, u0=None, *, raise_on_fail=True):
        """Composite solve; returns (u per level, relative residual history,
        status)."""
        if self.problem is None:
            raise SbmError(-1, "set_problem first")
        u = self.new_levels() if u0 is None else [self._dev(x, self.node_shape(a)).clone()
                                                   for a, x in enumerate(u0)]
        cap = int(self._opts.max_cycles) + 1
        hist = (ctypes.c_double * cap)()
        n = ctypes.c_int()
        fin = ctypes.c_double()
        st = lib().sbm_amr_solve(self._ctx, _ptr_array(u), hist, cap, ctypes.byref(n),
                                 ctypes.byref(fin))
        if raise_on_fail:
            check(st, allow=(SBM_OK, SBM_NOT_CONVERGED))
        h = np.array(hist[: min(n.value + 1, cap)])
        return u, h, st
