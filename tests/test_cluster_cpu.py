"""The library's Berger-Rigoutsos clustering (host code of the adaptive
set-up, no device needed) against the oracle's, bit for bit, on random and
structured flag arrays in 2D and 3D, and its argument checks."""
import numpy as np
import pytest

import oracle


def _flags(shape, seed):
    rng = np.random.default_rng(seed)
    f = (rng.uniform(size=shape) < 0.04).astype(np.uint8)
    for _ in range(4):
        lo = [int(rng.integers(0, n)) for n in shape]
        hi = [min(l + int(rng.integers(1, 5)), n) for l, n in zip(lo, shape)]
        f[tuple(slice(l, h) for l, h in zip(lo, hi))] = 1
    return f


CASES = [((9, 13), s) for s in range(4)] + [((16, 16), 7), ((1, 12), 3), ((5, 7, 6), 1),
                                             ((8, 8, 8), 2), ((4, 16, 3), 5), ((12, 10, 14), 6)]


@pytest.mark.parametrize("shape,seed", CASES)
@pytest.mark.parametrize("eff", [0.0, 0.3, 0.7, 0.9, 1.0])
def test_library_clustering_matches_oracle(shape, seed, eff):
    from paper_2212_02362_amd.amr import cluster_blocks
    f = _flags(shape, seed)
    ref, _ = oracle.br_cluster(f, eff)
    got = cluster_blocks(f, eff)
    assert np.array_equal(got, ref)


def test_empty_and_full():
    from paper_2212_02362_amd.amr import cluster_blocks
    z = np.zeros((6, 5), np.uint8)
    assert not cluster_blocks(z, 0.7).any()
    o = np.ones((3, 4, 5), np.uint8)
    assert cluster_blocks(o, 1.0).all()


def test_cluster_argument_checks():
    from paper_2212_02362_amd import SbmError
    from paper_2212_02362_amd.amr import cluster_blocks
    with pytest.raises(SbmError):
        cluster_blocks(np.ones((3, 3), np.uint8), 1.5)
    with pytest.raises(ValueError):
        cluster_blocks(np.ones(4, np.uint8), 0.5)


def test_cluster_rejects_aliased_output():
    import ctypes
    from paper_2212_02362_amd._lib import lib
    f = np.ones((3, 4), np.uint8)
    nb = (ctypes.c_int64 * 3)(4, 3, 1)
    st = lib().sbm_amr_cluster(2, ctypes.cast(nb, ctypes.c_void_p), f.ctypes.data_as(ctypes.c_void_p),
                               0.5, f.ctypes.data_as(ctypes.c_void_p))
    assert st == -1
