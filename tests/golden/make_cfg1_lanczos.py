"""Writes tests/golden/cfg1_lanczos_G.txt: the oracle's shifted-COCG iterates on
the real Lanczos basis (oracle.scocg_lanczos) for the first four RHS of
configuration 1 (simple cubic 16^3, 4x4 blocks, M = 16,384, S = I + bond
blocks N(0, 0.03)) on eight of its 128 shifts, to tol 1e-10, on the RHS's
requested rows.

Run from the repository root:  python tests/golden/make_cfg1_lanczos.py
It calls only the oracle and the seeded input generator (no value comes from
the GPU library).  The oracle needs a few minutes per RHS at this size, which
is why its results are stored rather than recomputed inside a GPU test; the
four RHS run in parallel processes.
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
NRHS = 4
TOL = 1e-10


def shift_subset(K):
    """Eight shifts spread over the energy mesh, both ends included."""
    return np.linspace(0, K - 1, 8).round().astype(int)


def solve(j):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    from oracle import scocg_lanczos
    from synth import bsr_to_scipy, make_config
    prob = make_config(1, nrhs=NRHS)
    H, S = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    ks = shift_subset(prob.nshift)
    b = np.zeros(prob.M)
    b[prob.rhs[j]] = 1.0
    rows = prob.outs(j)
    res = scocg_lanczos(H, S, prob.shifts[ks], b, TOL, rows=rows)
    return j, rows, ks, prob.shifts[ks], res.x, res.iters, res.status, res.n_outer


def main():
    with ProcessPoolExecutor(NRHS) as ex:
        out = list(ex.map(solve, range(NRHS)))
    path = os.path.join(HERE, "cfg1_lanczos_G.txt")
    with open(path, "w") as f:
        f.write("# G_ij(z_k) = x_j(z_k)[i] of (z_k S - H) x = e_j (the shifted equations of Sec. 3) on configuration 1\n")
        f.write("# (simple cubic 16^3, 4x4 blocks, M = 16384, S = I + N(0,0.03) bond blocks), written by\n")
        f.write(f"# tests/golden/make_cfg1_lanczos.py from oracle.scocg_lanczos at tol {TOL:g}: the first {NRHS} RHS,\n")
        f.write("# shifts k of the 128-point mesh listed below, every requested row of each RHS.\n")
        f.write("# columns: rhs_j row_i shift_k Re(z_k) Im(z_k) Re(G) Im(G) iterations status outer\n")
        for j, rows, ks, zs, x, iters, status, nout in out:
            for a, k in enumerate(ks):
                for o, i in enumerate(rows):
                    g = x[o, a]
                    f.write(f"{j} {int(i)} {int(k)} {zs[a].real:.17g} {zs[a].imag:.17g} {g.real:.17g} {g.imag:.17g} "
                            f"{int(iters[a])} {int(status[a])} {int(nout)}\n")
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
