"""Pins of the oracle's Berger-Rigoutsos clustering of flagged blocks (the
regridding of the paper's adaptive grid, Sec. 2.2): the two limits of the
efficiency (0: one bounding box; 1: the boxes tile the flags exactly), two
separated clusters cut at the hole between them, an L cut at the inflection
of its signature, the box properties on random flag sets (covering, disjoint,
tight, efficient), and the nesting of a clustered adaptive hierarchy."""
import numpy as np
import pytest

import oracle
import sbm_inputs as si


def _box_mask(shape, lo, hi):
    m = np.zeros(shape, bool)
    sl = tuple(slice(lo[a], hi[a] + 1) for a in reversed(range(len(shape))))
    m[sl] = True
    return m


@pytest.mark.parametrize("shape", [(7, 9), (5, 6, 4)])
def test_efficiency_limits(shape):
    f = (np.random.default_rng(1).uniform(size=shape) < 0.25).astype(np.uint8)
    out, boxes = oracle.br_cluster(f, 0.0)
    idx = np.argwhere(f)
    lo, hi = idx.min(axis=0), idx.max(axis=0)
    bb = np.zeros(shape, np.uint8)
    bb[tuple(slice(l, h + 1) for l, h in zip(lo, hi))] = 1
    assert len(boxes) == 1 and np.array_equal(out, bb)
    out, boxes = oracle.br_cluster(f, 1.0)
    assert np.array_equal(out, f)
    for lo, hi in boxes:
        assert f[_box_mask(shape, lo, hi)].all()


def test_two_clusters_split_at_the_hole():
    f = np.zeros((8, 10), np.uint8)
    f[0:3, 1:3] = 1
    f[0, 1] = 0
    f[5:8, 6:10] = 1
    out, boxes = oracle.br_cluster(f, 0.5)
    assert sorted(boxes) == [((1, 0), (2, 2)), ((6, 5), (9, 7))]


def test_l_shape_split_at_the_inflection():
    f = np.ones((8, 8), np.uint8)
    f[4:, 4:] = 0                       # efficiency of the bounding box: 0.75
    out, boxes = oracle.br_cluster(f, 0.8)
    assert len(boxes) == 2 and np.array_equal(out, f)
    out, boxes = oracle.br_cluster(f, 0.7)
    assert len(boxes) == 1 and out.all()


@pytest.mark.parametrize("shape,seed", [((12, 15), 0), ((16, 16), 1), ((6, 7, 8), 2),
                                        ((8, 8, 8), 3)])
@pytest.mark.parametrize("eff", [0.5, 0.7, 0.9])
def test_box_properties(shape, seed, eff):
    rng = np.random.default_rng(seed)
    # clumpy flags: a few random boxes plus sparse noise
    f = (rng.uniform(size=shape) < 0.05).astype(np.uint8)
    for _ in range(3):
        lo = [rng.integers(0, n - 2) for n in reversed(shape)]
        hi = [l + rng.integers(1, 4) for l in lo]
        hi = [min(h, n - 1) for h, n in zip(hi, reversed(shape))]
        f[_box_mask(shape, lo, hi)] = 1
    out, boxes = oracle.br_cluster(f, eff)
    union = np.zeros(shape, int)
    for lo, hi in boxes:
        m = _box_mask(shape, lo, hi)
        union += m
        inside = f[m]
        assert inside.sum() >= eff * inside.size - 1e-9        # efficient
        idx = np.argwhere(m & (f == 1))
        assert tuple(idx.min(axis=0)) == tuple(reversed(lo))   # tight
        assert tuple(idx.max(axis=0)) == tuple(reversed(hi))
    assert union.max() == 1                                    # disjoint
    assert np.array_equal(union.astype(np.uint8), out)
    assert np.all(out[f == 1] == 1)                            # covering


@pytest.mark.parametrize("eff", [0.0, 0.7, 0.95])
def test_clustered_hierarchy_nests(eff):
    p, psis = si.ellipsoidal_voids_amr(base=8, levels=3, block=4, seed=0)
    m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=4,
                          cluster_eff=eff)
    m0 = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val, block=4)
    b = [m.info(a)[0] for a in (1, 2)]
    b0 = [m0.info(a)[0] for a in (1, 2)]
    if eff == 0.0:
        assert all(np.array_equal(x, y) for x, y in zip(b, b0))
    # clustering only adds blocks: the finest level covers the unclustered one
    assert np.all(b[1][b0[1] == 1] == 1)
    # nesting: every active level-2 block has its parent and the parent's
    # neighbours on the sides it touches active on level 1
    for z, y, x in np.argwhere(b[1]):
        bi = (x, y, z)
        pb = [c // 2 for c in bi]
        sg = [1 if c % 2 else -1 for c in bi]
        for o in range(8):
            q = [pb[a] + (sg[a] if (o >> a) & 1 else 0) for a in range(3)]
            if all(0 <= q[a] < b[0].shape[2 - a] for a in range(3)):
                assert b[0][q[2], q[1], q[0]] == 1
