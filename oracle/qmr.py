"""Oracle for the generalized shifted QMR solve — TEST INFRASTRUCTURE ONLY.

The paper lists, beside gsCOCG, a generalized shifted quasi-minimal
residual method for the same equations (Sec. 3, item (ii)).  This is that
method written out for real symmetric H, real SPD S and a real right-hand
side b (here b = e_j), where the Krylov space shared by all shifts is real:

  S-Lanczos on S^{-1}H (inner products <u, v>_S = u^T S v), with w_i = S v_i:
    beta_0 = sqrt(b^T S^{-1} b),  v_0 = S^{-1} b / beta_0,  w_0 = b / beta_0
    u = H v_n;  alpha_n = v_n^T u;  t = u - alpha_n w_n - beta_n w_{n-1}
    q = S^{-1} t (inner CG);  beta_{n+1} = sqrt(q^T t)
    v_{n+1} = q / beta_{n+1};  w_{n+1} = t / beta_{n+1}
  so that (z I - S^{-1}H) V_n = V_{n+1} Hbar_n, Hbar_n = z Ibar - Tbar_n with the
  real tridiagonal Tbar_n (alpha on the diagonal, beta off it), and
  b - (zS - H) V_n y = W_{n+1} (beta_0 e_1 - Hbar_n y).

  For every shift z_k the iterate x_k = V_n y_k minimises the quasi-residual
  ||beta_0 e_1 - Hbar_n(z_k) y||_2: a QR factorisation of Hbar_n(z_k) by
  complex Givens rotations, one new column per iteration (the column has
  -beta_n, z_k - alpha_n, -beta_{n+1} in rows n-1, n, n+1), and the
  three-term direction recurrence d_n = (v_n - e d_{n-2} - f d_{n-1}) / R_nn,
  x_k += tau_n d_n.  The quasi-residual |g_{n+1}| bounds the true residual:
  ||b - (z_k S - H) x_k|| <= |g_{n+1}| (sum_{i<=n+1} ||w_i||^2)^{1/2}, and
  shift k stops when that bound is below tol ||b||.

The Lanczos process is shift-independent, so no seed shift and no seed
switching are involved; the shifts enter only through the 2x2 rotations.
Only the requested rows of x_k and d are kept (``rows``).
"""
from typing import Callable, Optional

import numpy as np

from .scocg import BREAKDOWN, CONVERGED, MAXITER, NONFINITE, ScocgResult, inner_cg


def givens(a, b):
    """(c, s, r) with c real >= 0, complex s, such that
    [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    aa, ab = abs(a), abs(b)
    if ab == 0.0:
        return 1.0, 0.0 + 0.0j, a
    if aa == 0.0:
        return 0.0, np.conj(b) / ab, ab + 0.0j
    nrm = np.hypot(aa, ab)
    ph = a / aa
    return aa / nrm, ph * np.conj(b) / nrm, ph * nrm


def sqmr(H, S, z, b, tol: float, rows=None, maxiter: Optional[int] = None, inner_tol: float = 1e-13,
         inner_maxiter: int = 1000, record: Optional[Callable] = None) -> ScocgResult:
    """Shifted QMR for (z_k S - H) x = b (S = None means I), real H, S, b.

    Returns x on ``rows`` ([len(rows), K]); ``record(n, v, w, alpha,
    beta_next)`` is called once per Lanczos step (for tests)."""
    b = np.asarray(b)
    if np.iscomplexobj(b):
        if np.any(b.imag != 0):
            raise ValueError("the real Lanczos form needs a real right-hand side")
        b = b.real
    b = b.astype(np.float64)
    z = np.asarray(z, dtype=np.complex128)
    M, K = b.size, z.size
    rows = np.arange(M) if rows is None else np.asarray(rows)
    maxiter = max(1000, 4 * M) if maxiter is None else maxiter
    nb = np.linalg.norm(b)
    inner_total = 0

    def s_solve(t):
        nonlocal inner_total
        if S is None:
            return t.copy()
        q, it = inner_cg(S, t, inner_tol, inner_maxiter)
        inner_total += it
        return q

    x = np.zeros((rows.size, K), dtype=np.complex128)
    iters = np.full(K, -1, dtype=np.int64)
    status = np.full(K, MAXITER, dtype=np.int8)
    resid = np.full(K, np.inf)
    if nb == 0.0:
        return ScocgResult(x, np.zeros(K, np.int64), np.zeros(K, np.int8), np.zeros(K), 0, 0, [])
    q0 = s_solve(b)
    beta0 = np.sqrt(b @ q0)
    v, w = q0 / beta0, b / beta0
    v_prev, w_prev = np.zeros(M), np.zeros(M)
    beta = 0.0
    sum_w2 = w @ w
    g = np.full(K, beta0, dtype=np.complex128)
    c1, s1 = np.ones(K), np.zeros(K, np.complex128)      # rotation of the previous column
    c2, s2 = np.ones(K), np.zeros(K, np.complex128)      # and of the one before
    d1 = np.zeros((rows.size, K), np.complex128)
    d2 = np.zeros((rows.size, K), np.complex128)
    done = np.zeros(K, dtype=bool)
    n_outer = 0
    for n in range(maxiter):
        n_outer = n + 1
        u = H @ v
        alpha = v @ u
        t = u - alpha * w - beta * w_prev
        q = s_solve(t)
        qt = q @ t
        if record is not None:
            record(n, v, w, alpha, np.sqrt(qt) if qt > 0 else 0.0)
        if not np.isfinite(qt):
            status[~done], done[:] = NONFINITE, True
            break
        if qt < 0.0:
            status[~done], done[:] = BREAKDOWN, True
            break
        beta_next = np.sqrt(qt)
        if beta_next > 0.0:
            sum_w2 += (t @ t) / qt
        bound_scale = np.sqrt(sum_w2)
        vr = v[rows]
        for k in range(K):
            if done[k]:
                continue
            # new column of Hbar(z_k): rows n-1, n, n+1
            a_prev, a_diag, a_next = -beta, z[k] - alpha, -beta_next
            e = s2[k] * a_prev                                  # rotation n-2 (row n-2 gets fill)
            f = c2[k] * a_prev
            f, gam = c1[k] * f + s1[k] * a_diag, -np.conj(s1[k]) * f + c1[k] * a_diag   # rotation n-1
            c, s, rnn = givens(gam, a_next)                      # rotation n
            if rnn == 0.0:
                status[k], done[k] = BREAKDOWN, True
                continue
            tau = c * g[k]
            g[k] = -np.conj(s) * g[k]
            dn = (vr - e * d2[:, k] - f * d1[:, k]) / rnn
            x[:, k] += tau * dn
            d2[:, k], d1[:, k] = d1[:, k], dn
            c2[k], s2[k], c1[k], s1[k] = c1[k], s1[k], c, s
            resid[k] = abs(g[k]) * bound_scale / nb
            if resid[k] < tol:
                status[k], done[k], iters[k] = CONVERGED, True, n + 1
        if done.all() or beta_next == 0.0:
            if beta_next == 0.0:       # invariant subspace: every iterate is exact
                for k in np.where(~done)[0]:
                    status[k], done[k], iters[k], resid[k] = CONVERGED, True, n + 1, 0.0
            break
        v_prev, w_prev = v, w
        v, w = q / beta_next, t / beta_next
        beta = beta_next
    return ScocgResult(x, iters, status, resid, n_outer, inner_total, [])


def scocg_lanczos(H, S, z, b, tol: float, rows=None, maxiter: Optional[int] = None, inner_tol: float = 1e-13,
                  inner_maxiter: int = 1000) -> ScocgResult:
    """The shifted COCG iterates of every shift, computed on the real
    S-Lanczos basis of the module docstring (real H, S, b).

    With a real basis the unconjugated bilinear form u^T S v of COCG is the
    S-inner product, so COCG's Galerkin condition V_n^T (b - (z_k S - H) x) = 0
    makes x_k = V_n y_k with (z_k I - T_n) y_k = beta_0 e_1: the same iterates
    as the seed-switching form in exact arithmetic.  Each shift factors its
    complex symmetric tridiagonal z_k I - T_n as L D L^T, one pivot per
    iteration (delta_n = z_k - alpha_n - beta_n^2 / delta_{n-1}), with
    p_n = v_n + (beta_n / delta_{n-1}) p_{n-1}, zeta_n = g_n / delta_n,
    g_n = (beta_n / delta_{n-1}) g_{n-1}, x_k += zeta_n p_n.  The residual is
    b - (z_k S - H) x_k = zeta_n t (t = beta_{n+1} w_{n+1}), so its norm
    |zeta_n| ||t|| is known exactly; shift k stops when it is below tol ||b||.
    """
    b = np.asarray(b)
    if np.iscomplexobj(b):
        if np.any(b.imag != 0):
            raise ValueError("the real Lanczos form needs a real right-hand side")
        b = b.real
    b = b.astype(np.float64)
    z = np.asarray(z, dtype=np.complex128)
    M, K = b.size, z.size
    rows = np.arange(M) if rows is None else np.asarray(rows)
    maxiter = max(1000, 4 * M) if maxiter is None else maxiter
    nb = np.linalg.norm(b)
    inner_total = 0

    def s_solve(t):
        nonlocal inner_total
        if S is None:
            return t.copy()
        q, it = inner_cg(S, t, inner_tol, inner_maxiter)
        inner_total += it
        return q

    x = np.zeros((rows.size, K), dtype=np.complex128)
    iters = np.full(K, -1, dtype=np.int64)
    status = np.full(K, MAXITER, dtype=np.int8)
    resid = np.full(K, np.inf)
    if nb == 0.0:
        return ScocgResult(x, np.zeros(K, np.int64), np.zeros(K, np.int8), np.zeros(K), 0, 0, [])
    q0 = s_solve(b)
    beta0 = np.sqrt(b @ q0)
    v, w = q0 / beta0, b / beta0
    w_prev = np.zeros(M)
    beta = 0.0
    delta = np.ones(K, dtype=np.complex128)       # previous pivot (unused at n = 0)
    g = np.full(K, beta0, dtype=np.complex128)
    p = np.zeros((rows.size, K), dtype=np.complex128)
    done = np.zeros(K, dtype=bool)
    n_outer = 0
    for n in range(maxiter):
        n_outer = n + 1
        u = H @ v
        alpha = v @ u
        t = u - alpha * w - beta * w_prev
        q = s_solve(t)
        qt = q @ t
        if not np.isfinite(qt):
            status[~done], done[:] = NONFINITE, True
            break
        if qt < 0.0:
            status[~done], done[:] = BREAKDOWN, True
            break
        beta_next = np.sqrt(qt)
        tnorm = np.linalg.norm(t)
        vr = v[rows]
        for k in range(K):
            if done[k]:
                continue
            c = 0.0 if n == 0 else beta / delta[k]
            dn = z[k] - alpha - (0.0 if n == 0 else beta * beta / delta[k])
            if dn == 0.0:
                status[k], done[k] = BREAKDOWN, True
                continue
            g[k] = beta0 if n == 0 else c * g[k]
            zeta = g[k] / dn
            p[:, k] = vr + c * p[:, k]
            x[:, k] += zeta * p[:, k]
            delta[k] = dn
            resid[k] = abs(zeta) * tnorm / nb
            if resid[k] < tol or beta_next == 0.0:
                status[k], done[k], iters[k] = CONVERGED, True, n + 1
        if done.all() or beta_next == 0.0:
            break
        w_prev = w
        v, w = q / beta_next, t / beta_next
        beta = beta_next
    return ScocgResult(x, iters, status, resid, n_outer, inner_total, [])
