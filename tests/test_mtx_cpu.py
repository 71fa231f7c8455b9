"""Matrix Market input (host code, no GPU): files written from the seeded
synthetic matrices are read back through the C ABI and compared entry by
entry with what scipy's reader makes of the same file (a library routine,
independent of the library under test) and with the source matrix."""
import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp

from synth import bsr_to_scipy, make_problem


@pytest.fixture(scope="module")
def B():
    from paper_1402_7285_amd import binding
    binding.load()
    return binding


def _prob():
    return make_problem(name="mtx", lattice="sc", L=3, bdim=4, s_scale=0.03, K=4, nrhs=2, seed_key=(3, 1, 4))


def _write(path, A, symmetric, comment="synthetic"):
    A = sp.coo_matrix(A)
    if symmetric:
        A = sp.tril(A).tocoo()
    with open(path, "w") as f:
        f.write(f"%%MatrixMarket matrix coordinate real {'symmetric' if symmetric else 'general'}\n")
        f.write(f"% {comment}\n%\n")
        f.write(f"{A.shape[0]} {A.shape[1]} {A.nnz}\n")
        for i, j, v in zip(A.row, A.col, A.data):
            f.write(f"{i + 1} {j + 1} {v:.17g}\n")


def _dense_of(m):
    e = m.export()
    return sp.bsr_matrix((e.vals, e.colidx, e.rowptr), shape=(e.n, e.n)).toarray()


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("bdim", [1, 4])
def test_read_back_equals_source(B, tmp_path, symmetric, bdim):
    p = _prob()
    for A in (p.H, p.S):
        As = bsr_to_scipy(A)
        f = tmp_path / "a.mtx"
        _write(f, As, symmetric)
        m = B.Matrix.from_mtx(f, bdim)
        nb, bd, nblk = m.shape()
        assert bd == bdim and nb * bd == A.n
        D = _dense_of(m)
        assert np.array_equal(D, As.toarray())
        assert np.array_equal(D, scipy.io.mmread(str(f)).toarray())


def test_duplicates_are_summed_and_comments_skipped(B, tmp_path):
    f = tmp_path / "d.mtx"
    f.write_text("%%MatrixMarket matrix coordinate real symmetric\n% c\n3 3 4\n1 1 2.0\n2 1 0.5\n2 1 0.25\n3 3 -1\n")
    D = _dense_of(B.Matrix.from_mtx(f, 1))
    want = np.array([[2.0, 0.75, 0.0], [0.75, 0.0, 0.0], [0.0, 0.0, -1.0]])
    assert np.array_equal(D, want)


@pytest.mark.parametrize("text,code", [
    ("%%MatrixMarket matrix array real general\n2 2\n1\n0\n0\n1\n", "SHAPE"),
    ("%%MatrixMarket matrix coordinate complex general\n1 1 1\n1 1 1 0\n", "SHAPE"),
    ("%%MatrixMarket matrix coordinate real general\n2 3 1\n1 1 1\n", "SHAPE"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 2\n1 1 1\n", "SHAPE"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 1\n3 1 1\n", "SHAPE"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 2\n1 2 1\n2 1 2\n", "NOT_SYMMETRIC"),
    ("not a matrix\n", "SHAPE"),
])
def test_bad_files_are_rejected(B, tmp_path, text, code):
    f = tmp_path / "bad.mtx"
    f.write_text(text)
    with pytest.raises(B.ScocgError) as ei:
        B.Matrix.from_mtx(f, 1)
    assert ei.value.code == getattr(B, "E_" + code)


def test_missing_file(B, tmp_path):
    with pytest.raises(B.ScocgError) as ei:
        B.Matrix.from_mtx(tmp_path / "none.mtx", 1)
    assert ei.value.code == B.E_ARG
