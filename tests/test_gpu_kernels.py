"""Per-kernel parity of the HIP library against the FP64 oracle, through the
C ABI, on grids that span several thread blocks and end in ragged tails.

Bar: FP64 kernels agree with the oracle to <= 1e-13 relative (max norm);
the FP32 Apply to <= 1e-5 relative (one FP32 rounding per term on O(30)-term
sums of O(1) products)."""
import numpy as np
import pytest
import torch

import oracle
import sbm_inputs as si
from _util import random_problem, rel_l2, rel_max, say, solver_for, to_np

pytestmark = pytest.mark.gpu

GRIDS = [(40, 30), (37, 26), (20, 12, 16), (12, 18, 9)]


def _setup(ncell, seed=0, cubic=False):
    p = random_problem(ncell, seed=seed, cubic=cubic)
    say("kernel setup", ncell, seed, "cubic" if cubic else "")
    S = solver_for(p)
    psi = oracle.floor_psi(p.psi_raw, p.psi_floor)
    mask, uD = oracle.dirichlet(p.ncell, p.kind, p.val)
    rng = np.random.default_rng(seed + 100)
    u = rng.standard_normal((p.dim,) + p.node_shape)
    f = rng.standard_normal((p.dim,) + p.node_shape)
    return p, S, psi, mask, u, f


@pytest.mark.parametrize("ncell", GRIDS)
def test_apply(ncell):
    p, S, psi, mask, u, f = _setup(ncell)
    say("apply", ncell)
    got = to_np(S.apply(u))
    ref = oracle.apply(p.ncell, p.h, p.lam, p.mu, psi, u)
    assert rel_max(got, ref) < 1e-13
    say("apply_f32", ncell)
    got32 = to_np(S.level_apply_f32(0, torch.as_tensor(u, dtype=torch.float32)))
    assert rel_max(got32, ref) < 1e-5


@pytest.mark.parametrize("ncell", [(40, 32), (16, 24, 16)])
def test_hierarchy_psi_and_coarse_apply(ncell):
    p, S, psi, mask, u, f = _setup(ncell, seed=3)
    nc = p.ncell
    ps = psi
    for l in range(S.nlevels):
        say("level", l, nc)
        assert S.level_shape(l) == tuple(nc)
        assert rel_max(to_np(S.level_psi(l)), ps) < 1e-15
        hl = tuple(x * 2 ** l for x in p.h)
        ul = np.random.default_rng(l).standard_normal((p.dim,) + tuple(n + 1 for n in reversed(nc)))
        got = to_np(S.level_apply(l, ul))
        ref = oracle.apply(nc, hl, p.lam, p.mu, ps, ul)
        assert rel_max(got, ref) < 1e-13
        if l + 1 < S.nlevels:
            ps = oracle.coarsen_psi(nc, ps)
            nc = tuple(n // 2 for n in nc)


@pytest.mark.parametrize("ncell", GRIDS + [(8, 6, 10), (20, 16)])
def test_residual_and_smoothers(ncell):
    p, S, psi, mask, u, f = _setup(ncell, seed=1)
    u = np.where(mask == 1, oracle.dirichlet(p.ncell, p.kind, p.val)[1], u)
    say("residual", ncell)
    got = to_np(S.level_residual(0, u, f))
    ref = oracle.residual(p.ncell, p.h, p.lam, p.mu, psi, mask, u, f)
    assert rel_max(got, ref) < 1e-13
    assert (got[mask == 1] == 0).all()
    for omega in (0.8, 0.6):
        say("jacobi", ncell, omega)
        got = to_np(S.level_smooth(0, -1, omega, u, f))
        ref = oracle.jacobi(p.ncell, p.h, p.lam, p.mu, psi, mask, omega, u, f)
        assert rel_max(got, ref) < 1e-13
    for colour in (0, 1):
        say("rb half", ncell, colour)
        got = to_np(S.level_smooth(0, colour, 1.0, u, f))
        ref = oracle.rb_half(p.ncell, p.h, p.lam, p.mu, psi, mask, 1.0, colour, u, f)
        assert rel_max(got, ref) < 1e-13
        # the other colour is copied bit for bit
        idx = np.indices(p.node_shape).sum(0) % 2
        other = np.broadcast_to(idx != colour, got.shape)
        assert np.array_equal(got[other], u[other])


@pytest.mark.parametrize("cubic", [False, True])
@pytest.mark.parametrize("ncell", [(200, 30, 12), (230, 25, 9), (256, 33, 6), (256, 32, 10),
                                   (128, 30, 10), (100, 26, 7)])
def test_tiled_half_sweep(ncell, cubic):
    """Levels wider than 96 nodes in x take the LDS-tiled half-sweep: several
    64 x 8 tiles, a ragged last tile in x and y, z chunks; 257 and 129 nodes in
    x (and 33 in y) leave the last column (row) to the node-parallel face
    blocks.
    Cubic cells take the kernels' 4-coefficient form."""
    p, S, psi, mask, u, f = _setup(ncell, seed=11, cubic=cubic)
    u = np.where(mask == 1, oracle.dirichlet(p.ncell, p.kind, p.val)[1], u)
    for colour in (0, 1):
        say("tiled half sweep", ncell, colour)
        got = to_np(S.level_smooth(0, colour, 1.0, u, f))
        ref = oracle.rb_half(p.ncell, p.h, p.lam, p.mu, psi, mask, 1.0, colour, u, f)
        assert rel_max(got, ref) < 1e-13
        idx = np.indices(p.node_shape).sum(0) % 2
        other = np.broadcast_to(idx != colour, got.shape)
        assert np.array_equal(got[other], u[other])


@pytest.mark.parametrize("cubic", [False, True])
@pytest.mark.parametrize("ncell", [(200, 30, 12), (230, 25, 9), (256, 33, 6), (256, 20, 40),
                                   (256, 32, 7), (208, 32, 9)])
def test_fused_two_colour_sweep(ncell, cubic):
    """A whole Gauss-Seidel sweep in one launch (levels wider than 192 nodes):
    equal to the oracle's half-sweep of the first colour followed by the
    half-sweep of the second, for both colour orders, from a given iterate and
    from zero; several tiles, ragged last tiles in x and y, several z chunks
    (40 planes make ten); 257 x 33 nodes put the last node column and row into
    the edge tiles of the sweep from zero, 209 x 33 the last row with a ragged
    last tile in x.  The FP32 sweep is held to the FP32 bar against the
    FP64 oracle on the same (FP32-representable) inputs."""
    p, S, psi, mask, u, f = _setup(ncell, seed=13)
    u = np.where(mask == 1, oracle.dirichlet(p.ncell, p.kind, p.val)[1], u)
    half = lambda c, v: oracle.rb_half(p.ncell, p.h, p.lam, p.mu, psi, mask, 1.0, c, v, f)  # noqa: E731
    for c0 in (0, 1):
        say("fused sweep", ncell, c0)
        ref = half(1 - c0, half(c0, u))
        got = to_np(S.level_sweep(0, c0, 1.0, u, f))
        assert rel_max(got, ref) < 1e-13
        say("fused sweep from zero", ncell, c0)
        z = np.zeros_like(u)
        ref0 = half(1 - c0, half(c0, z))
        got0 = to_np(S.level_sweep(0, c0, 1.0, None, f))
        assert rel_max(got0, ref0) < 1e-13
    u32, f32 = u.astype(np.float32), f.astype(np.float32)
    u64, f64 = u32.astype(np.float64), f32.astype(np.float64)
    half64 = lambda c, v: oracle.rb_half(p.ncell, p.h, p.lam, p.mu, psi, mask, 1.0, c, v, f64)  # noqa: E731
    say("fused sweep fp32", ncell)
    ref = half64(1, half64(0, u64))
    got = to_np(S.level_sweep(0, 0, 1.0, u32, f32, fp32=True)).astype(np.float64)
    assert rel_l2(got, ref) < 1e-5


@pytest.mark.parametrize("cubic", [False, True])
@pytest.mark.parametrize("ncell", [(200, 30, 12), (256, 33, 6), (256, 32, 10)])
def test_tiled_residual_and_norm(ncell, cubic):
    """The tiled residual (r and its per-tile norm partials) at widths that
    take the tiled path, with anisotropic and cubic cells."""
    p, S, psi, mask, u, f = _setup(ncell, seed=12, cubic=cubic)
    u = np.where(mask == 1, oracle.dirichlet(p.ncell, p.kind, p.val)[1], u)
    say("tiled residual", ncell)
    got = to_np(S.level_residual(0, u, f))
    ref = oracle.residual(p.ncell, p.h, p.lam, p.mu, psi, mask, u, f)
    assert rel_max(got, ref) < 1e-13
    fA, _, _ = oracle.rhs(p.ncell, p.h, p.lam, p.mu, psi, p.kind, p.val, p.b)
    r_ref = oracle.residual(p.ncell, p.h, p.lam, p.mu, psi, mask, u, fA)
    r_got, nrm = S.residual(u)
    assert rel_max(to_np(r_got), r_ref) < 1e-13
    assert abs(nrm - np.linalg.norm(r_ref)) <= 1e-12 * np.linalg.norm(r_ref)


@pytest.mark.parametrize("ncell", [(40, 30), (36, 26), (20, 12, 16), (12, 18, 10)])
def test_transfers(ncell):
    p, S, psi, mask, u, f = _setup(ncell, seed=2)
    if S.nlevels < 2:
        pytest.skip("no coarser level")
    ncc = S.level_shape(1)
    maskc, _ = oracle.dirichlet(ncc, p.kind, p.val)
    say("restrict", ncell)
    got = to_np(S.level_restrict(0, f))
    ref = oracle.restrict(p.ncell, f, maskc)
    assert rel_max(got, ref) < 1e-14
    e = np.random.default_rng(7).standard_normal((p.dim,) + tuple(n + 1 for n in reversed(ncc)))
    e[maskc == 1] = 0.0
    say("prolong", ncell)
    got = to_np(S.level_prolong_add(0, e, u))
    ref = oracle.prolong_add(ncc, e, mask, u)
    assert rel_max(got, ref) < 1e-14


@pytest.mark.parametrize("ncell", [(200, 30, 12), (232, 26, 10), (256, 34, 6), (256, 32, 14)])
def test_tiled_restriction(ncell):
    """Full weighting from levels wider than 192 nodes runs as 64 x 4 coarse
    column tiles over chunks of coarse planes, plus a node-parallel pass over
    the last coarse column / row a 2^n + 1 level leaves: equal to the
    oracle's restriction (ragged last tiles, 129 coarse columns, coarse
    displacement DOF zeroed)."""
    p, S, psi, mask, u, f = _setup(ncell, seed=31)
    ncc = S.level_shape(1)
    maskc, _ = oracle.dirichlet(ncc, p.kind, p.val)
    say("tiled restriction", ncell)
    ref = oracle.restrict(p.ncell, f, maskc)
    got = to_np(S.level_restrict(0, f))
    assert rel_max(got, ref) < 1e-14
    assert np.all(got[maskc == 1] == 0.0)
    # the same numbers on every call (each coarse node is written by one
    # thread, from LDS planes no other thread writes meanwhile)
    for _ in range(3):
        assert np.array_equal(to_np(S.level_restrict(0, f)), got)


@pytest.mark.parametrize("ncell", [(16, 16), (24, 12, 12), (8, 8, 8), (35, 33)])
def test_bottom_cg(ncell):
    """The single-workgroup CG on the bottom grid reaches the dense solution
    (LDS-resident up to 1024 nodes; (35, 33) cannot be coarsened, so its
    1224-node bottom takes the global-memory variant)."""
    p, S, psi, mask, u, f = _setup(ncell, seed=4)
    L = S.nlevels - 1
    ncb = S.level_shape(L)
    psib = to_np(S.level_psi(L))
    hb = tuple(x * 2 ** L for x in p.h)
    maskb, _ = oracle.dirichlet(ncb, p.kind, p.val)
    fb = np.random.default_rng(5).standard_normal((p.dim,) + tuple(n + 1 for n in reversed(ncb)))
    fb[maskb == 1] = 0.0
    say("bottom", ncell, ncb)
    x, it = S.bottom_solve(fb)
    x = to_np(x)
    K = oracle.assemble(ncb, hb, p.lam, p.mu, psib)
    free = maskb.ravel() == 0
    ref = np.zeros(K.shape[0])
    A = K[np.ix_(free, free)]
    ref[free] = np.linalg.solve(A, fb.ravel()[free])
    cond = np.linalg.cond(A)
    assert rel_max(x.ravel(), ref) < max(1e-10, 1e-13 * cond)
    assert 0 < it <= 4 * free.sum()


@pytest.mark.parametrize("ncell", [(40, 30), (20, 12, 16)])
def test_rhs(ncell):
    p, S, psi, mask, u, f = _setup(ncell, seed=5)
    say("rhs", ncell)
    fA, fB = S.rhs()
    rA, rB, _ = oracle.rhs(p.ncell, p.h, p.lam, p.mu, psi, p.kind, p.val, p.b)
    assert rel_max(to_np(fA), rA) < 1e-14
    assert rel_max(to_np(fB), rB) < 1e-13


@pytest.mark.parametrize("ncell", [(40, 30), (20, 12, 16), (13, 9, 7)])
def test_sensitivity_and_compliance(ncell):
    p, S, psi, mask, u, f = _setup(ncell, seed=6)
    lam = np.where(mask == 1, 0.0, f)
    say("sensitivity", ncell)
    got = to_np(S.sensitivity(u, lam))
    ref = oracle.sensitivity(p.ncell, p.h, p.lam, p.mu, p.kind, p.val, u, lam)
    assert rel_max(got, ref) < 1e-12
    got2 = to_np(S.sensitivity(u, lam, lam_scale=0.5, design=p.psi_raw, chain=1))
    ref2 = np.where(p.psi_raw > p.psi_floor, 0.5 * ref, 0.0)
    assert rel_max(got2, ref2) < 1e-12
    rho = np.random.default_rng(1).uniform(0.0, 1.0, p.psi_raw.shape)
    got3 = to_np(S.sensitivity(u, lam, design=rho, chain=2))
    ref3 = oracle.sensitivity(p.ncell, p.h, p.lam, p.mu, p.kind, p.val, u, lam, rho=rho,
                              psi_floor=p.psi_floor)
    assert rel_max(got3, ref3) < 1e-12
    say("compliance", ncell)
    fA, _, _ = oracle.rhs(p.ncell, p.h, p.lam, p.mu, psi, p.kind, p.val, p.b)
    J = np.prod(p.h) * np.sum(fA[mask == 0] * u[mask == 0])
    assert abs(S.compliance(u) - J) < 1e-12 * np.prod(p.h) * np.abs(fA * u).sum()


def test_set_problem_errors():
    from paper_2212_02362_amd import SbmError
    p = random_problem((8, 8, 8), seed=9)
    S = solver_for(p)
    bad = p.psi_raw.copy()
    bad[1, 2, 3] = np.nan
    say("nonfinite psi")
    with pytest.raises(SbmError) as ei:
        S.set_problem(bad, p.lam, p.mu, p.psi_floor, p.kind, p.val, p.b)
    assert ei.value.status == -4
    say("zero diagonal")
    empty = p.psi_raw.copy()
    empty[:, :, :] = 0.0
    with pytest.raises(SbmError) as ei:
        S.set_problem(empty, p.lam, p.mu, 0.0, p.kind, p.val, p.b)
    assert ei.value.status == -6
    say("solve before problem")
    from paper_2212_02362_amd import Solver
    S2 = Solver(p.ncell, p.h)
    with pytest.raises(SbmError):
        S2.solve()
