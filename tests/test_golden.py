"""Checks against constants the paper prints (tests/golden/paper_constants.txt)."""
import os

import numpy as np

import oracle
import sbm_inputs as si

HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_constants.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v, *_ = line.split()
            out[k] = float(v)
    return out


def test_lame_pair_printed_in_paper():
    c = _load()
    lam, mu = si.lame(c["E"], c["nu"])
    assert round(lam, 2) == c["lambda"] and round(mu, 2) == c["mu"]


def test_stiffness_floors_printed_in_paper():
    """The topology-optimisation floor zeta^2 and the fracture floor eta are
    both 1e-4, the floor used for the density workload."""
    c = _load()
    assert np.isclose(c["zeta"] ** 2, 1e-4) and c["eta"] == 1e-4
    p = si.cantilever_density_3d(nx=8, ny=4, nz=4)
    assert p.psi_floor == c["eta"]


def test_constant_psi_diagonal_with_paper_moduli():
    """With the paper's moduli and psi = 1 the 3D interior diagonal is
    (2(lambda+2mu) + 4 mu)/h^2 (Navier-Lame, second order)."""
    c = _load()
    h = 0.5
    D = oracle.diag((4, 4, 4), (h, h, h), c["lambda"], c["mu"], np.ones((4, 4, 4)))
    expect = (2 * (c["lambda"] + 2 * c["mu"]) + 4 * c["mu"]) / h ** 2
    assert np.allclose(D[:, 2, 2, 2], expect, rtol=1e-14)
