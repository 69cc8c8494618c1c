"""Stored closed forms (paper, Section 5.3, eq. test-state) and the oracle's
hierarchy summary for the 32x32 workload (written by tests/golden/make_golden.py)."""
import json
import math
import os

import numpy as np

import inputs
from oracle import solve

G = os.path.join(os.path.dirname(__file__), "golden")


def test_test_state_coefficients():
    cf = json.load(open(os.path.join(G, "closed_forms.json")))
    m = inputs.mesh3d(4)
    v = 1 + 5 * (2 + 5 * 3)   # node (1/4, 2/4, 3/4)
    s = math.sin(math.pi / 4) * math.sin(math.pi / 2) * math.sin(3 * math.pi / 4)
    for beta, coef in cf["yd_coeff_3d"].items():
        assert abs(inputs.yd_manufactured(m, float(beta))[v] - coef * s) <= 1e-14 * coef
    assert abs(cf["u_amp_2d_for_unit_yd"]["0.01"] - 4.031401719316667) < 1e-12


def test_c1_hierarchy_regression():
    ref = json.load(open(os.path.join(G, "hierarchy_c1.json")))
    p = inputs.config("c1")
    h, A, M = solve.build_problem(p)
    assert [lev.n for lev in h.levels] == ref["n"]
    assert [int(lev.A.nnz) for lev in h.levels] == ref["nnzA"]
    assert h.levels[0].omega == ref["omega0"]
