"""Degenerate and symmetric cases on the GPU, in all three solver forms
(seed-switching COCG, COCG on the real Lanczos basis, shifted QMR):

* an RHS whose atom is decoupled from the rest (block-diagonal H and S):
  its Krylov space has dimension at most the block size, so every form ends
  within a few iterations with the exact solution (pinned to a dense solve);
* duplicate shifts give the same G;
* conjugate shifts give conjugate G (H and S are real), which also covers
  shifts below the real axis;
* scalar (1x1) blocks, against the oracle of each form.
"""
import numpy as np
import pytest

from oracle import local_system, scocg_lanczos, scocg_projected, sqmr
from synth import bsr_to_dense, bsr_to_scipy, make_problem
from synth.tb import Bsr
from tests.parity import compare_rhs

pytestmark = pytest.mark.gpu

METHODS = (0, 2, 1)       # seed-switching COCG, Lanczos-basis COCG, QMR


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _block_diagonal(nb=6, bd=4, seed=21):
    rng = np.random.default_rng(seed)
    Hv, Sv = [], []
    for _ in range(nb):
        a = rng.normal(size=(bd, bd))
        Hv.append((a + a.T) / 2)
        e = 0.05 * rng.normal(size=(bd, bd))
        Sv.append(np.eye(bd) + (e + e.T) / 2)
    rowptr = np.arange(nb + 1, dtype=np.int64)
    col = np.arange(nb, dtype=np.int32)
    H = Bsr(nb, bd, rowptr, col, np.stack(Hv))
    S = Bsr(nb, bd, rowptr.copy(), col.copy(), np.stack(Sv))
    return H, S


def _solve(B, H, S, shifts, rhs, out_ptr, out_rows, method, tol=1e-10):
    P = B.Problem(H, S)
    plan = B.Plan(P, shifts, rhs, out_ptr=out_ptr, out_rows=out_rows, tol=tol, method=method)
    return plan.solve()


@pytest.mark.parametrize("method", METHODS)
def test_decoupled_atom_ends_exactly(B, method):
    H, S = _block_diagonal()
    Hd, Sd = bsr_to_dense(H), bsr_to_dense(S)
    shifts = np.array([-2.0 + 0.05j, 0.3 + 0.01j, 1.7 + 0.2j, -0.4 - 0.1j])
    rhs = np.array([1, 9, 22], dtype=np.int32)
    rows = [np.arange(4 * (j // 4), 4 * (j // 4) + 4) for j in rhs]          # the RHS's own block
    out_ptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
    r = _solve(B, H, S, shifts, rhs, out_ptr, np.concatenate(rows).astype(np.int32), method)
    assert np.all(r["status"] == B.CONVERGED)
    assert r["iters"].max() <= 5, r["iters"]
    worst = 0.0
    for j, b in enumerate(rhs):
        e = np.zeros(Hd.shape[0])
        e[b] = 1.0
        for k, z in enumerate(shifts):
            x = np.linalg.solve(z * Sd - Hd, e)
            worst = max(worst, np.abs(r["G"][j][k] - x[rows[j]]).max() / np.abs(x[rows[j]]).max())
    print(f"[edge] decoupled atom, method {method}: max iterations {r['iters'].max()}, rel err {worst:.1e}",
          flush=True)
    assert worst < 1e-9


def _sc(nrhs=3, K=None, shifts=None, bdim=4, seed=(31, 7, 2)):
    p = make_problem(name="sc4-edge", lattice="sc", L=4, bdim=bdim, s_scale=0.03, K=K or 4, eta=0.05, nrhs=nrhs,
                     seed_key=seed)
    if shifts is not None:
        p.shifts = np.asarray(shifts, dtype=np.complex128)
    return p


@pytest.mark.parametrize("method", METHODS)
def test_duplicate_and_conjugate_shifts(B, method):
    z = np.array([-1.5 + 0.05j, 0.7 + 0.03j])
    shifts = np.array([z[0], z[1], z[0], np.conj(z[0]), np.conj(z[1])])
    p = _sc(shifts=shifts)
    r = _solve(B, p.H, p.S, p.shifts, p.rhs, p.out_ptr, p.out_rows, method)
    assert np.all(r["status"] == B.CONVERGED)
    for j in range(p.nrhs):
        G = r["G"][j]
        scale = np.abs(G).max()
        assert np.abs(G[2] - G[0]).max() <= 1e-12 * scale, "duplicate shift"
        assert r["iters"][j][2] == r["iters"][j][0]
        # the seed-switching form reaches z and conj z through a complex seed, so its two
        # answers agree to the solve's accuracy (the parity bar), not to rounding
        cbar = 1e-11 if method != 0 else 1e-8
        assert np.abs(G[3] - np.conj(G[0])).max() <= cbar * scale, "conjugate shift"
        assert np.abs(G[4] - np.conj(G[1])).max() <= cbar * scale, "conjugate shift"
        if method != 0:        # one real basis: the shift recurrences are the same operations
            assert np.array_equal(G[2], G[0])


@pytest.mark.parametrize("method", METHODS)
def test_scalar_blocks_against_oracle(B, method):
    p = make_problem(name="sc6-scalar", lattice="sc", L=6, bdim=1, s_scale=0.05, K=8, eta=0.05, nrhs=3,
                     seed_key=(4, 4, 4))
    r = _solve(B, p.H, p.S, p.shifts, p.rhs, p.out_ptr, p.out_rows, method, tol=p.tol)
    Hc, Sc = bsr_to_scipy(p.H), bsr_to_scipy(p.S)
    worst = 0.0
    for j in range(p.nrhs):
        Hl, Sl, loc, orb = local_system(p, j, Hc, Sc)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        pos = np.searchsorted(orb, p.outs(j))
        if method == 0:
            res = scocg_projected(Hl, Sl, p.shifts, b.astype(np.complex128), pos, p.tol)
        elif method == 2:
            res = scocg_lanczos(Hl, Sl, p.shifts, b, p.tol, rows=pos)
        else:
            res = sqmr(Hl, Sl, p.shifts, b, p.tol, rows=pos)
        worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hl, Sl, p.shifts,
                                       b.astype(np.complex128), p.tol, rows=pos, iter_frac=0.25, tag=f"rhs {j}"))
    print(f"[edge] scalar blocks, method {method}: worst rel err {worst:.1e}", flush=True)
