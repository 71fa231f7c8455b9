"""Pins for the shifted QMR oracle (CPU).

* the S-Lanczos relation (z I - S^{-1}H) V_n = V_{n+1} Hbar_n and the
  S-orthonormality of the first Lanczos vectors;
* the incremental Givens QR gives the minimiser of the quasi-residual: after
  m steps, x_k equals V_m y with y from a dense least-squares solve of the
  (m+1) x m problem min ||beta_0 e_1 - Hbar_m(z_k) y|| (numpy lstsq);
* the stopping bound is an upper bound of the true residual, and converged
  results agree with the dense solution within the a-priori bound.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense_solve, sqmr
from synth import bsr_to_dense, bsr_to_scipy, make_problem


def _prob(S=True, K=6):
    return make_problem(name="qmr", lattice="sc", L=3, bdim=4, s_scale=0.03 if S else None, K=K, eta=0.1, nrhs=2,
                        seed_key=(9, 2, 6))


def _lanczos(prob, j, m):
    H, S = bsr_to_scipy(prob.H), (bsr_to_scipy(prob.S) if prob.S is not None else None)
    b = np.zeros(prob.M)
    b[prob.rhs[j]] = 1.0
    rec = []
    res = sqmr(H, S, prob.shifts, b, 1e-300, maxiter=m,
               record=lambda n, v, w, a, bn: rec.append((v.copy(), w.copy(), a, bn)))
    V = np.stack([r[0] for r in rec], 1)
    alpha = np.array([r[2] for r in rec])
    beta = np.array([r[3] for r in rec])
    return H, S, b, res, V, alpha, beta


@pytest.mark.parametrize("with_S", [True, False])
def test_lanczos_relation_and_orthonormality(with_S):
    prob = _prob(with_S)
    m = 12
    H, S, b, res, V, alpha, beta = _lanczos(prob, 0, m)
    Sd = np.eye(prob.M) if S is None else S.toarray()
    Hd = H.toarray()
    G = V.T @ Sd @ V
    assert np.abs(G - np.eye(m)).max() < 1e-8
    A = np.linalg.solve(Sd, Hd)                     # S^{-1} H
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    # columns 0..m-2 involve only v_0..v_{m-1}
    lhs = A @ V[:, :m - 1]
    rhs = V @ T[:, :m - 1]
    assert np.abs(lhs - rhs).max() < 1e-8 * np.abs(lhs).max()


@pytest.mark.parametrize("with_S", [True, False])
def test_iterate_minimises_quasi_residual(with_S):
    prob = _prob(with_S)
    m = 15
    H, S, b, res, V, alpha, beta = _lanczos(prob, 1, m)
    Sd = np.eye(prob.M) if S is None else S.toarray()
    beta0 = np.sqrt(b @ np.linalg.solve(Sd, b))
    T = np.zeros((m + 1, m))
    for n in range(m):
        T[n, n] = alpha[n]
        T[n + 1, n] = beta[n]
        if n + 1 < m:
            T[n, n + 1] = beta[n]
    for k, zk in enumerate(prob.shifts):
        Hb = zk * np.eye(m + 1, m) - T
        rhs = np.zeros(m + 1, dtype=np.complex128)
        rhs[0] = beta0
        y = np.linalg.lstsq(Hb, rhs, rcond=None)[0]
        x_ls = V @ y
        assert np.abs(res.x[:, k] - x_ls).max() < 1e-10 * np.abs(x_ls).max()
        qres = np.linalg.norm(rhs - Hb @ y)
        # the reported bound is quasi-residual times the Frobenius norm of W_{m+1}
        assert res.resid[k] >= qres * 0.999 / np.linalg.norm(b)


@pytest.mark.parametrize("with_S", [True, False])
def test_converged_results_and_bound(with_S):
    prob = _prob(with_S, K=8)
    H, S = bsr_to_scipy(prob.H), (bsr_to_scipy(prob.S) if prob.S is not None else None)
    Hd = bsr_to_dense(prob.H)
    Sd = np.eye(prob.M) if prob.S is None else bsr_to_dense(prob.S)
    lam_min = sla.eigh(Sd, eigvals_only=True)[0]
    tol = 1e-9
    for j in range(prob.nrhs):
        b = np.zeros(prob.M)
        b[prob.rhs[j]] = 1.0
        res = sqmr(H, S, prob.shifts, b, tol)
        assert np.all(res.status == 0)
        for k, zk in enumerate(prob.shifts):
            xs = dense_solve(Hd, Sd, zk, b)
            true_res = np.linalg.norm(b - (zk * Sd - Hd) @ res.x[:, k])
            assert true_res <= res.resid[k] * 1.0001 + 1e-14
            assert np.linalg.norm(res.x[:, k] - xs) <= 2 * tol / (abs(zk.imag) * lam_min)


def test_rows_subset_and_complex_rhs_rejected():
    prob = _prob(True)
    H, S = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    b = np.zeros(prob.M)
    b[prob.rhs[0]] = 1.0
    full = sqmr(H, S, prob.shifts, b, 1e-9)
    rows = prob.outs(0)
    part = sqmr(H, S, prob.shifts, b, 1e-9, rows=rows)
    assert np.array_equal(part.x, full.x[rows])
    with pytest.raises(ValueError):
        sqmr(H, S, prob.shifts, b * 1j, 1e-9)


# ---- COCG iterates on the real Lanczos basis

@pytest.mark.parametrize("with_S", [True, False])
def test_lanczos_cocg_equals_seed_switching_form_at_fixed_steps(with_S):
    """In exact arithmetic both forms produce the COCG (Galerkin) iterates;
    before rounding differences grow (a few tens of steps) they agree to
    rounding, iterate by iterate, with the residual norms too."""
    from oracle import scocg, scocg_lanczos
    prob = _prob(with_S, K=8)
    H, S = bsr_to_scipy(prob.H), (bsr_to_scipy(prob.S) if prob.S is not None else None)
    b = np.zeros(prob.M)
    b[prob.rhs[0]] = 1.0
    for m in (3, 8, 15):
        a = scocg_lanczos(H, S, prob.shifts, b, 1e-300, maxiter=m)
        c = scocg(H, S, prob.shifts, b.astype(np.complex128), 1e-300, maxiter=m)
        assert np.abs(a.x - c.x).max() <= 1e-9 * np.abs(c.x).max()
        assert np.allclose(a.resid, c.resid, rtol=1e-8)


def test_lanczos_cocg_is_the_galerkin_solution_and_its_residual_is_exact():
    from oracle import scocg_lanczos
    prob = _prob(True, K=6)
    m = 12
    H, S, b, res, V, alpha, beta = _lanczos(prob, 0, m + 1)
    Sd = S.toarray()
    beta0 = np.sqrt(b @ np.linalg.solve(Sd, b))
    T = np.diag(alpha[:m]) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    a = scocg_lanczos(H, S, prob.shifts, b, 1e-300, maxiter=m)
    Hd = H.toarray()
    for k, zk in enumerate(prob.shifts):
        y = np.linalg.solve(zk * np.eye(m) - T, beta0 * np.eye(m)[:, 0])
        xg = V[:, :m] @ y
        assert np.abs(a.x[:, k] - xg).max() <= 1e-10 * np.abs(xg).max()
        true_res = np.linalg.norm(b - (zk * Sd - Hd) @ a.x[:, k])
        assert abs(a.resid[k] - true_res) <= 1e-8 * true_res + 1e-13
