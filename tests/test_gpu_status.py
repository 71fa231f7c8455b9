"""The per-(RHS, shift) status paths of the GPU solvers, against the oracle on
the same inputs (the status of a pair is a unique result, so it must match):

* NONFINITE: a NaN in one on-site element of H.  It reaches every Krylov
  space that touches its atom; pairs still running then stop as NONFINITE
  (the paper's equations have no solution to report there).
* BREAKDOWN: a real shift equal to an eigenvalue of a diagonal H, with the
  RHS on that orbital: (z S - H) is singular on the one-dimensional Krylov
  space, the pivot of that shift is exactly zero; every other shift of the
  same RHS converges in one step with x = e_j / (z - h_j).
* MAXITER: an iteration cap below the convergence point: partial results
  equal to the oracle's iterates after the same number of steps.

Each runs through the one-workgroup Lanczos-basis solver, the team solver
and the seed-switching COCG solver."""
import numpy as np
import pytest

from oracle import local_system, scocg_lanczos, scocg_projected, sqmr
from synth import bsr_to_scipy, make_problem

pytestmark = pytest.mark.gpu

SOLVERS = {
    # (method name, options)
    "lanczos_one_workgroup": ("cocg-lanczos", dict(team_size=-1)),
    "lanczos_team": ("cocg-lanczos", dict(team_size=2, panel_width=1)),
    "qmr_team": ("qmr", dict(team_size=2, panel_width=1)),
    "seed_switching": ("cocg", dict()),
}


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _method(B, name):
    return {"cocg-lanczos": B.METHOD_COCG_LANCZOS, "qmr": B.METHOD_QMR, "cocg": B.METHOD_COCG}[name]


def _oracle(name, Hc, Sc, shifts, b, tol, rows, maxiter=None):
    if name == "cocg-lanczos":
        return scocg_lanczos(Hc, Sc, shifts, b, tol, rows=rows, maxiter=maxiter)
    if name == "qmr":
        return sqmr(Hc, Sc, shifts, b, tol, rows=rows, maxiter=maxiter)
    return scocg_projected(Hc, Sc, shifts, b.astype(np.complex128), rows, tol, maxiter=maxiter)


def _solve(B, prob, name, opts, **extra):
    P = B.Problem(prob.H, prob.S)
    plan = B.Plan(P, prob.shifts, prob.rhs, method=_method(B, name), tol=prob.tol, out_ptr=prob.out_ptr,
                  out_rows=prob.out_rows, **opts, **extra)
    return plan.solve()


@pytest.mark.parametrize("solver", sorted(SOLVERS))
def test_nonfinite_block(B, solver):
    name, opts = SOLVERS[solver]
    prob = make_problem(name="nan", lattice="sc", L=3, bdim=4, s_scale=0.03, K=6, eta=0.1, nrhs=3,
                        seed_key=(3, 1, 4))
    # NaN in the on-site block of the first RHS's atom (symmetric: a diagonal element)
    a = int(prob.rhs[0]) // 4
    e = int(np.nonzero(prob.H.colidx[prob.H.rowptr[a]:prob.H.rowptr[a + 1]] == a)[0][0]) + int(prob.H.rowptr[a])
    prob.H.vals[e, 1, 1] = np.nan
    r = _solve(B, prob, name, opts)
    Hc_all, Sc_all = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hc_all, Sc_all)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        res = _oracle(name, Hc, Sc, prob.shifts, b, prob.tol, np.searchsorted(orb, prob.outs(j)))
        assert np.array_equal(r["status"][j], res.status), (j, r["status"][j], res.status)
    assert np.all(r["status"][0] == B.NONFINITE)


@pytest.mark.parametrize("solver", sorted(SOLVERS))
def test_breakdown_on_an_eigenvalue(B, solver):
    name, opts = SOLVERS[solver]
    # diagonal H (scalar blocks, no hopping), S = I: the Krylov space of e_j is span(e_j)
    prob = make_problem(name="diag", lattice="sc", L=3, bdim=1, hop=(0.0, 0.0), K=4, eta=0.1, nrhs=2,
                        tol=1e-12, seed_key=(2, 7, 1))
    j0 = int(prob.rhs[0])
    row = np.arange(prob.H.rowptr[j0], prob.H.rowptr[j0 + 1])
    h = prob.H.vals[row[prob.H.colidx[row] == j0][0], 0, 0]
    # shift 0 sits exactly on h_j of RHS 0 (a real shift); the others are ordinary complex shifts
    prob.shifts = np.array([h + 0j, 0.3 + 0.1j, -0.7 + 0.05j, 1.1 + 0.2j])
    r = _solve(B, prob, name, opts)
    Hc_all = bsr_to_scipy(prob.H)
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hc_all, None)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        rows = np.searchsorted(orb, prob.outs(j))
        res = _oracle(name, Hc, None, prob.shifts, b, prob.tol, rows)
        assert np.array_equal(r["status"][j], res.status), (j, r["status"][j], res.status)
    if name != "cocg":
        # Lanczos basis: the pivot of shift 0 is exactly z - h = 0; the others are exact after one step
        assert r["status"][0][0] == B.BREAKDOWN
        hj = np.array([Hc_all[int(q), int(q)] for q in prob.rhs])
        for j in range(prob.nrhs):
            for k in range(prob.nshift):
                if r["status"][j][k] != B.CONVERGED:
                    continue
                own = list(prob.outs(j)).index(int(prob.rhs[j]))
                assert abs(r["G"][j][k][own] - 1.0 / (prob.shifts[k] - hj[j])) <= 1e-14 * abs(1.0 / (prob.shifts[k] - hj[j]))
                assert r["iters"][j][k] == 1


@pytest.mark.parametrize("solver", sorted(SOLVERS))
def test_maxiter_partial_results(B, solver):
    name, opts = SOLVERS[solver]
    prob = make_problem(name="cap", lattice="sc", L=3, bdim=4, s_scale=0.03, K=6, eta=0.05, nrhs=2,
                        tol=1e-12, seed_key=(8, 8, 2))
    r = _solve(B, prob, name, opts, maxiter=5)
    Hc_all, Sc_all = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    for j in range(prob.nrhs):
        assert np.all(r["status"][j] == B.MAXITER) and np.all(r["iters"][j] == -1)
        assert r["stats"][j][0] == 5
        Hc, Sc, loc, orb = local_system(prob, j, Hc_all, Sc_all)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        rows = np.searchsorted(orb, prob.outs(j))
        res = _oracle(name, Hc, Sc, prob.shifts, b, prob.tol, rows, maxiter=5)
        assert np.all(res.status == 1)
        # five steps are far from the chaotic regime: the iterates agree to rounding
        rel = np.abs(r["G"][j] - res.x.T).max() / np.abs(res.x).max()
        assert rel < 1e-11, (j, rel)
