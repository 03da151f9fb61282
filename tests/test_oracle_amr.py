"""Pins of the oracle's block-structured adaptive (BSAMR) composite solve:
reductions to uniform solves, exactness of the composite residual for
quadratic fields (quadratic ghost interpolation, padded fine residual,
restriction at the interface), brute-force tags and blocks, convergence and
the approach to the uniform fine solution as coverage grows."""
import numpy as np
import pytest

import oracle
import sbm_inputs as si

LAM, MU = si.lame(1.0, 0.3)


def _bc_c2():
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    kind[4, :] = oracle.DISPLACEMENT
    kind[5, :] = oracle.DISPLACEMENT
    val[5, 2] = 1e-3
    return kind, val


def _psi_levels(base, A, seed=0):
    p, psis = si.ellipsoidal_voids_amr(base=base, levels=A + 1, block=4, seed=seed)
    return p, psis


def test_single_level_equals_uniform_solve():
    p, psis = _psi_levels(8, 0)
    m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=4)
    u, hist, st = m.solve(rtol=1e-10, max_cycles=100)
    uo, ho, so = oracle.solve(p.ncell, p.h, p.lam, p.mu, psis[0], p.psi_floor, p.kind, p.val,
                              rtol=1e-10, max_cycles=100)
    assert st == 0 and so == 0 and len(hist) == len(ho)
    assert np.allclose(hist, ho, rtol=1e-8, atol=1e-14)
    assert np.linalg.norm(u[0] - uo) <= 1e-10 * np.linalg.norm(uo)


def test_full_coverage_equals_uniform_fine_solve():
    """A fine level covering the whole box: the composite cycle is a V-cycle
    of the fine grid, so its iterates equal the uniform solve's there."""
    p, psis = _psi_levels(8, 1)
    full = [np.ones((2, 2, 2), np.uint8)]
    m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=8,
                          blocks=full)
    blk, cls, _ = m.info(1)
    assert blk.all() and set(np.unique(cls)) == {1}
    u, hist, st = m.solve(rtol=1e-10, max_cycles=100)
    h1 = tuple(x / 2 for x in p.h)
    uo, ho, so = oracle.solve((16, 16, 16), h1, p.lam, p.mu, psis[1], p.psi_floor, p.kind, p.val,
                              rtol=1e-10, max_cycles=100)
    assert st == 0 and so == 0 and len(hist) == len(ho)
    assert np.allclose(hist, ho, rtol=1e-7, atol=1e-14)
    assert np.linalg.norm(u[1] - uo) <= 1e-9 * np.linalg.norm(uo)
    # the coarse level holds the injected fine values
    assert np.allclose(u[0], uo[:, ::2, ::2, ::2], rtol=0, atol=1e-15 * np.abs(uo).max())


@pytest.mark.parametrize("psi_kind", ["constant", "linear"])
def test_quadratic_field_has_zero_composite_residual(psi_kind):
    """u quadratic and psi constant or linear: with the continuum load at the
    nodes of every level, the composite residual vanishes at every composite
    unknown away from the box faces -- this needs the quadratic ghost
    interpolation (interface and outer layers), the padded fine residual and
    the injected coarse values."""
    base, A = 8, 2
    rng = np.random.default_rng(1)
    kind = np.zeros((6, 3), np.int32)
    val = np.zeros((6, 3))
    g = rng.uniform(-0.3, 0.3, 3) if psi_kind == "linear" else np.zeros(3)
    psis = []
    for a in range(A + 1):
        n = base << a
        X = si.cell_centres((n,) * 3, (1.0 / n,) * 3)
        psis.append(0.7 + g[0] * X[0] + g[1] * X[1] + g[2] * X[2])
    # partial coverage: level-1 blocks in one corner, level-2 blocks inside them
    b1 = np.zeros((4, 4, 4), np.uint8)
    b1[:2, 1:3, :3] = 1
    b2 = np.zeros((8, 8, 8), np.uint8)
    b2[1:3, 3:5, 1:5] = 1
    m = oracle.AmrProblem((base,) * 3, (1.0 / base,) * 3, LAM, MU, psis, 0.0, kind, val, block=4,
                          blocks=[b1, b2])
    classes = [m.info(a)[1] for a in (1, 2)]
    assert all((c == k).any() for c in classes for k in (1, 2, 3, 4))
    a0 = rng.standard_normal(3)
    B = rng.standard_normal((3, 3))
    Q = rng.standard_normal((3, 3, 3))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))
    I = np.eye(3)
    C = (LAM * np.einsum("ij,kl->ijkl", I, I)
         + MU * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))
    us, fs = [], []
    for a in range(A + 1):
        n = base << a
        Xn = si.node_coords((n,) * 3, (1.0 / n,) * 3)
        u = np.stack([a0[k] + sum(B[k, l] * Xn[l] for l in range(3))
                      + sum(Q[k, l, q] * Xn[l] * Xn[q] for l in range(3) for q in range(3))
                      for k in range(3)])
        psin = 0.7 + g[0] * Xn[0] + g[1] * Xn[1] + g[2] * Xn[2]
        f = np.zeros_like(u)
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    for l in range(3):
                        if C[i, j, k, l] == 0:
                            continue
                        grad = B[k, l] + 2 * sum(Q[k, l, q] * Xn[q] for q in range(3))
                        f[i] -= C[i, j, k, l] * (g[j] * grad + psin * 2 * Q[k, j, l])
        us.append(u)
        fs.append(f)
    r, nrm, _ = m.residual(us, fs)
    scale = max(np.abs(f).max() for f in fs)
    for a in range(A + 1):
        n = base << a
        inner = np.zeros(m.node_shape(a)[1:], bool)
        inner[2:-2, 2:-2, 2:-2] = True
        assert np.abs(r[a][:, inner]).max() < 1e-10 * scale, (a, np.abs(r[a][:, inner]).max())
    # hanging interface nodes (odd index along the interface) exist, so the
    # check above exercised the in-plane quadratic interpolation
    hang = np.argwhere(classes[1] == 2)
    assert ((hang % 2).sum(axis=1) > 0).any()


def test_tags_and_blocks_brute_force():
    p, psis = _psi_levels(8, 2, seed=3)
    m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=4)
    tags = []
    for a in range(2):
        n = 8 << a
        psi = np.maximum(psis[a], p.psi_floor)
        pp = np.pad(psi, 1, mode="edge")
        gs = 0.0
        for ax in range(3):
            sl_p = [slice(1, -1)] * 3
            sl_m = [slice(1, -1)] * 3
            sl_p[ax] = slice(2, None)
            sl_m[ax] = slice(0, -2)
            d = pp[tuple(sl_p)] - pp[tuple(sl_m)]
            gs = gs + (d / (2.0 / n)) ** 2
        t = gs * (1.0 / n) ** 2 > 0.05 ** 2
        assert np.array_equal(t.astype(np.uint8), oracle.amr_tags((n,) * 3, (1.0 / n,) * 3, psi, 0.05))
        tags.append(t)
    blocks = []
    for a in (1, 2):
        t = tags[a - 1]
        nb = (8 << a) // 4
        half = 2
        b = np.zeros((nb,) * 3, np.uint8)
        for k in range(nb):
            for j in range(nb):
                for i in range(nb):
                    sl = tuple(slice(max(0, q * half - 1), q * half + half + 1) for q in (k, j, i))
                    b[k, j, i] = t[sl].any()
        blocks.append(b)
    # nesting: parents and the parents' neighbours on the touching sides
    for (k, j, i) in np.argwhere(blocks[1]):
        for dk in (0, 1 if k % 2 else -1):
            for dj in (0, 1 if j % 2 else -1):
                for di in (0, 1 if i % 2 else -1):
                    q = (k // 2 + dk, j // 2 + dj, i // 2 + di)
                    if all(0 <= x < 4 for x in q):
                        blocks[0][q] = 1
    for a in (1, 2):
        assert np.array_equal(m.info(a)[0], blocks[a - 1])


def test_composite_converges_toward_uniform_fine_solution():
    """Finer coverage (lower threshold) brings the composite solution closer
    to the uniform solve on the finest grid."""
    p, psis = _psi_levels(8, 1, seed=2)
    h1 = tuple(x / 2 for x in p.h)
    uf, _, _ = oracle.solve((16, 16, 16), h1, p.lam, p.mu, psis[1], p.psi_floor, p.kind, p.val,
                            rtol=1e-11, max_cycles=200)
    errs, cover = [], []
    for thresh in (0.4, 0.05, None):
        full = None if thresh is not None else [np.ones((4, 4, 4), np.uint8)]
        m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val,
                              block=4, thresh=thresh if thresh is not None else 0.05, blocks=full)
        u, hist, st = m.solve(rtol=1e-11, max_cycles=200)
        assert st == 0 and np.all(np.diff(np.log(hist[1:])) < 0)
        blk, cls, _ = m.info(1)
        cover.append(blk.mean())
        # compare at level-0 node positions (level 0 holds injected fine values where covered)
        errs.append(np.linalg.norm(u[0] - uf[:, ::2, ::2, ::2]) / np.linalg.norm(uf))
    assert cover[0] < cover[1] <= cover[2] == 1.0
    assert errs[0] > errs[2] and errs[1] > errs[2] and errs[2] < 1e-9, (errs, cover)
