"""GPU solve of matrices read from Matrix Market files, in scalar (1x1)
block form — the form for matrices whose atoms carry different numbers of
orbitals — against the oracle on the same matrices."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import scocg, scocg_projected
from synth import bsr_to_scipy, make_problem
from tests.parity import compare_rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _write(path, A):
    A = sp.tril(sp.coo_matrix(A)).tocoo()
    with open(path, "w") as f:
        f.write("%%MatrixMarket matrix coordinate real symmetric\n")
        f.write(f"{A.shape[0]} {A.shape[1]} {A.nnz}\n")
        for i, j, v in zip(A.row, A.col, A.data):
            f.write(f"{i + 1} {j + 1} {v:.17g}\n")


@pytest.mark.parametrize("full_x", [True, False])
def test_scalar_blocks_from_mtx(B, tmp_path, full_x):
    prob = make_problem(name="mtx-gen", lattice="sc", L=3, bdim=4, s_scale=0.03, K=8, eta=0.05, nrhs=3,
                        seed_key=(3, 1, 5))
    Hs, Ss = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    _write(tmp_path / "H.mtx", Hs)
    _write(tmp_path / "S.mtx", Ss)
    Hm = B.Matrix.from_mtx(tmp_path / "H.mtx", 1)
    Sm = B.Matrix.from_mtx(tmp_path / "S.mtx", 1)
    assert Hm.shape()[1] == 1
    P = B.Problem(Hm, Sm)
    plan = B.Plan(P, prob.shifts, prob.rhs, tol=prob.tol, full_x=full_x, out_ptr=prob.out_ptr,
                  out_rows=prob.out_rows)
    assert (plan.info["global"] & 2) == (0 if full_x else 2)
    r = plan.solve()
    worst = 0.0
    for j in range(prob.nrhs):
        b = np.zeros(prob.M, dtype=np.complex128)
        b[prob.rhs[j]] = 1.0
        rows = prob.outs(j)
        if full_x:
            res = scocg(Hs, Ss, prob.shifts, b, prob.tol)
            worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hs, Ss, prob.shifts, b,
                                           prob.tol, tag=f"rhs {j}"))
        else:
            res = scocg_projected(Hs, Ss, prob.shifts, b, rows, prob.tol)
            worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hs, Ss, prob.shifts, b,
                                           prob.tol, tag=f"proj rhs {j}", rows=rows, iter_frac=0.25))
    print(f"[mtx] scalar-block solve ({'full x' if full_x else 'projected'}): worst rel err {worst:.2e}", flush=True)
