"""Host-only checks of the C ABI: the library loads, exports every function
that include/scocg.h declares, and validates matrices without a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1402_7285_amd import binding as B
from synth import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scocg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scocg_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert sorted(B.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in _declared():
        assert name in syms, name


def test_header_compiles_as_c():
    src = "#include \"scocg.h\"\nint main(void){scocg_options o; scocg_options_default(&o); return 0;}\n"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                        "-x", "c", "-"], input=src, text=True, stderr=subprocess.PIPE)
    assert r.returncode == 0, r.stderr


def test_options_default():
    o = B.scocg_options_default()
    assert o.tol == 1e-10 and o.maxiter == 0 and o.precision == B.FP64
    assert o.replace_every == 0 and o.inner_tol == 1e-13 and o.seed_index == -1 and o.audit == 1


def _bsr(p):
    return p.H.nbrows, p.H.bdim, p.H.rowptr, p.H.colidx, p.H.vals


def test_matrix_validation():
    p = make_problem(lattice="sc", L=3, bdim=4, nrhs=2)
    h = B.scocg_matrix_from_bsr(*_bsr(p))
    B.scocg_matrix_free(h)
    B.scocg_matrix_free(None)                 # NULL is accepted
    # not symmetric: perturb one off-diagonal block
    v = p.H.vals.copy()
    v[1, 0, 1] += 1e-12
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_bsr(p.H.nbrows, 4, p.H.rowptr, p.H.colidx, v)
    assert e.value.code == B.E_NOT_SYMMETRIC
    # column out of range
    c = p.H.colidx.copy()
    c[-1] = p.H.nbrows
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_bsr(p.H.nbrows, 4, p.H.rowptr, c, p.H.vals)
    assert e.value.code == B.E_SHAPE
    # unsorted columns
    c = p.H.colidx.copy()
    c[0], c[1] = c[1], c[0]
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_bsr(p.H.nbrows, 4, p.H.rowptr, c, p.H.vals)
    assert e.value.code == B.E_SHAPE
    # bad sizes
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_bsr(0, 4, p.H.rowptr, p.H.colidx, p.H.vals)
    assert e.value.code == B.E_ARG
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_bsr(p.H.nbrows, 17, p.H.rowptr, p.H.colidx, p.H.vals)
    assert e.value.code == B.E_ARG
    assert "bdim" in B.load().scocg_last_error().decode()


def test_matrix_from_csr_matches_bsr():
    import scipy.sparse as sp
    from synth import bsr_to_scipy
    p = make_problem(lattice="sc", L=3, bdim=4, nrhs=2)
    A = bsr_to_scipy(p.H)
    A.sort_indices()
    h = B.scocg_matrix_from_csr(A.shape[0], A.indptr.astype(np.int64), A.indices, A.data, 4)
    B.scocg_matrix_free(h)
    Au = sp.triu(A).tocsr()        # not symmetric
    with pytest.raises(B.ScocgError) as e:
        B.scocg_matrix_from_csr(A.shape[0], Au.indptr.astype(np.int64), Au.indices, Au.data, 4)
    assert e.value.code == B.E_NOT_SYMMETRIC


def test_new_entry_points_reject_bad_arguments_on_the_host():
    # argument checks that run before any device call
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_sync(None)
    assert ei.value.code == B.E_ARG
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_mlp_train(np.zeros((1, 16)), np.zeros(1))
    assert ei.value.code == B.E_ARG
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_mlp_train(np.zeros((4, 16)), np.array([0.0, 1.0, np.nan, 2.0]))
    assert ei.value.code == B.E_ARG
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_mlp_train(np.zeros((4, 16)), np.zeros(4), epochs=0)
    assert ei.value.code == B.E_ARG
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_mlp_train(np.zeros((4, 16)), np.zeros(4), val_frac=1.0)
    assert ei.value.code == B.E_ARG
    model = np.zeros(B.scocg_mlp_model_floats(), dtype=np.float32)      # sd = 0: not a trained model
    with pytest.raises(B.ScocgError) as ei:
        B.scocg_mlp_predict(model, np.zeros((3, 16)))
    assert ei.value.code == B.E_ARG
    assert B.scocg_mlp_model_floats() == B.scocg_mlp_nparams() + 32
    cfg = B.scocg_mlp_cfg_default()
    assert (cfg.epochs, cfg.batch, cfg.val_frac) == (200, 256, pytest.approx(0.2)) and cfg.init_weights is None
