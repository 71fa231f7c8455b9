"""Writes the stored expected values under tests/golden/ from the oracle.

Run from the repository root:  python tests/golden/make_golden.py
It calls only the oracle (and the seeded input generator): no value here
comes from the GPU library.  The fixtures are plain text so that a change of
the oracle's arithmetic shows up as a diff.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import scocg, scocg_lanczos, sqmr          # noqa: E402
from synth import bsr_to_scipy, make_problem              # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def small_generalized():
    """The fixture's problem: simple cubic 3^3 with 4x4 blocks (M = 108),
    S = I + small symmetric bond blocks, 6 shifts, 2 RHS, tol 1e-12."""
    return make_problem(name="golden-sc3", lattice="sc", L=3, bdim=4, s_scale=0.03, K=6, eta=0.1, nrhs=2,
                        tol=1e-12, seed_key=(1402, 7285, 99))


def write(path, prob, results):
    with open(path, "w") as f:
        f.write("# G_ij(z_k) = x_j(z_k)[i] of (z_k S - H) x = e_j (the shifted equations of Sec. 3), written by\n")
        f.write("# tests/golden/make_golden.py from the oracle: simple cubic 3^3, 4x4 blocks, M = 108, S = I + N(0,0.03)\n")
        f.write("# bond blocks, seed key (1402, 7285, 99), 6 shifts, tol 1e-12.\n")
        f.write("# rows: per RHS the first 8 of its requested rows (its own atom, then a neighbour).\n")
        f.write("# columns: form rhs_j row_i shift_k Re(z_k) Im(z_k) Re(G) Im(G) iterations\n")
        for form, per_rhs in results.items():
            for j, rows, res in per_rhs:
                for k, z in enumerate(prob.shifts):
                    for o, i in enumerate(rows):
                        g = res.x[o, k]
                        f.write(f"{form} {j} {i} {k} {z.real:.17g} {z.imag:.17g} {g.real:.17g} {g.imag:.17g} "
                                f"{int(res.iters[k])}\n")


def compute(prob):
    Hs, Ss = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    out = {"cocg": [], "cocg_lanczos": [], "qmr": []}
    for j in range(prob.nrhs):
        b = np.zeros(prob.M)
        b[prob.rhs[j]] = 1.0
        rows = prob.outs(j)[:8]       # the RHS's own atom and its first neighbour
        full = scocg(Hs, Ss, prob.shifts, b.astype(np.complex128), prob.tol)
        full.x = full.x[rows]
        out["cocg"].append((int(prob.rhs[j]), rows, full))
        out["cocg_lanczos"].append((int(prob.rhs[j]), rows, scocg_lanczos(Hs, Ss, prob.shifts, b, prob.tol, rows=rows)))
        out["qmr"].append((int(prob.rhs[j]), rows, sqmr(Hs, Ss, prob.shifts, b, prob.tol, rows=rows)))
    return out


if __name__ == "__main__":
    p = small_generalized()
    write(os.path.join(HERE, "sc3_generalized_G.txt"), p, compute(p))
    print("wrote", os.path.join(HERE, "sc3_generalized_G.txt"))
