"""Writes the stored expected values under tests/golden/.

Every value here is a closed form taken from the paper (cited per file) or is
computed by the CPU oracle; nothing is read from the GPU library.
Run:  python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def closed_forms():
    # Section 5.3, eq. test-state: y_d = (1/(3 pi^2) + 3 pi^2 beta) sin sin sin
    # has the optimal control u* = sin(pi x) sin(pi y) sin(pi z); the betas are
    # those of Tables 3 and 4.  The 2D analogue (y_d = sin sin) has
    # u* = c sin sin with c = 1/(2 pi^2 beta + 1/(2 pi^2)).
    out = {"source": "paper Section 5.3, eq. test-state (betas of Tables 3-4)",
           "yd_coeff_3d": {}, "u_amp_2d_for_unit_yd": {}}
    for beta in (1e-4, 1e-2, 1.0, 100.0, 1e-3):
        out["yd_coeff_3d"][repr(beta)] = 1.0 / (3 * math.pi ** 2) + 3 * math.pi ** 2 * beta
        out["u_amp_2d_for_unit_yd"][repr(beta)] = 1.0 / (2 * math.pi ** 2 * beta + 1.0 / (2 * math.pi ** 2))
    return out


def hierarchy_c1():
    import inputs
    from oracle import solve
    p = inputs.config("c1")
    h, A, M = solve.build_problem(p)
    return {"source": "oracle smoothed-aggregation hierarchy of the 32x32 workload",
            "n": [lev.n for lev in h.levels], "nnzA": [int(lev.A.nnz) for lev in h.levels],
            "nnzS": [int(lev.S.nnz) for lev in h.levels[:-1]],
            "omega0": h.levels[0].omega}


if __name__ == "__main__":
    with open(os.path.join(HERE, "closed_forms.json"), "w") as f:
        json.dump(closed_forms(), f, indent=1, sort_keys=True)
    with open(os.path.join(HERE, "hierarchy_c1.json"), "w") as f:
        json.dump(hierarchy_c1(), f, indent=1, sort_keys=True)
