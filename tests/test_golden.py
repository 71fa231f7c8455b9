"""The stored fixture tests/golden/sc3_generalized_G.txt (written by
tests/golden/make_golden.py from the oracle): the oracle still reproduces
it, and its values are the solutions of the shifted equations (dense solve
of (z_k S - H) x = e_j) to within the tolerance's bound."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from make_golden import compute, small_generalized     # noqa: E402
from synth import bsr_to_dense                           # noqa: E402

FIXTURE = os.path.join(HERE, "golden", "sc3_generalized_G.txt")


def load_fixture():
    rows = []
    with open(FIXTURE) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((t[0], int(t[1]), int(t[2]), int(t[3]), complex(float(t[4]), float(t[5])),
                         complex(float(t[6]), float(t[7])), int(t[8])))
    return rows


def test_fixture_is_the_solution_of_the_shifted_equations():
    p = small_generalized()
    Hd, Sd = bsr_to_dense(p.H), bsr_to_dense(p.S)
    lam_min = np.linalg.eigvalsh(Sd).min()
    worst = 0.0
    fx = load_fixture()
    assert len(fx) == 3 * p.nrhs * p.nshift * 8
    cache = {}
    for form, j, i, k, z, g, it in fx:
        assert np.isclose(z, p.shifts[k], rtol=0, atol=1e-15)
        if (j, k) not in cache:
            e = np.zeros(p.M)
            e[j] = 1.0
            cache[(j, k)] = np.linalg.solve(p.shifts[k] * Sd - Hd, e)
        x = cache[(j, k)]
        # ||x - x*|| <= ||(zS - H)^{-1}|| ||r||, with ||(zS - H)^{-1}|| <= 1 / (|Im z| lam_min(S))
        bound = 2 * p.tol / (abs(p.shifts[k].imag) * lam_min)
        assert abs(g - x[i]) <= bound, (form, j, i, k, abs(g - x[i]), bound)
        worst = max(worst, abs(g - x[i]))
    assert worst > 0.0


def test_oracle_reproduces_fixture():
    p = small_generalized()
    res = compute(p)
    stored = {}
    for form, j, i, k, z, g, it in load_fixture():
        stored[(form, j, i, k)] = (g, it)
    for form, per_rhs in res.items():
        for j, rows, r in per_rhs:
            for k in range(p.nshift):
                for o, i in enumerate(rows):
                    g, it = stored[(form, j, int(i), k)]
                    assert abs(r.x[o, k] - g) <= 1e-11 * max(1e-3, abs(g)), (form, j, i, k)
                    assert int(r.iters[k]) == it, (form, j, k)
