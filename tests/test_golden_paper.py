"""Numbers the paper prints, kept as cited text fixtures under tests/golden/."""
from __future__ import annotations

import os

import numpy as np

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def test_table1_condition_numbers_fix_the_mass_convention():
    """kappa = lambda_max / (eps_min + (2 a m)^2) with lambda_max ~ 23 reproduces
    every kappa of Table 1 to the two digits printed; a mass term (a m)^2 would
    be off by 4x.  The oracle's operator carries exactly (2m)^2 when called with
    two_m = 2 a m."""
    for lat, am, eps, kappa in _rows("table1_condition.txt"):
        am, eps, kappa = float(am), float(eps), float(kappa)
        model = 23.0 / (eps + (2 * am) ** 2)
        wrong = 23.0 / (eps + am ** 2)
        assert abs(model - kappa) / kappa < 0.05, lat
        assert abs(wrong - kappa) / kappa > 1.0, lat
    dims = (2, 2, 2, 2)
    W = I.random_su3_field(dims, 0.5, 3)
    F, L = O.fold_links(W, W, I.C_FAT, I.C_LONG)
    am = 0.05
    d = O.dense_A(F, L, 2 * am) - O.dense_A(F, L, 0.0)
    assert np.abs(d - (2 * am) ** 2 * np.eye(d.shape[0])).max() < 1e-15
