"""Oracle: generalized shifted COCG with seed switching (FP64, NumPy).

TEST INFRASTRUCTURE ONLY — see the package docstring.

What is computed (Sec. 3, Eq. 2): for each complex energy z_k the solution
x(z_k) of the generalized shifted linear equation (z_k S - H) x = b, with H
real symmetric and S real symmetric positive definite (Sec. 2; S = I
reduces to the standard shifted problem, Sec. 3), and from it the
Green's-function elements G_ij(z_k) = e_i^T x_j(z_k) for b = e_j.  The
paper names the generalized shifted COCG method for this (Sec. 3, item (i))
but prints no algorithm; the steps below are derived from the mathematics.

Derivation (the recurrences the code relies on)
-----------------------------------------------
* With A'(z) = z I - S^{-1} H the equation reads A'(z) x = S^{-1} b.  S^{-1}H
  is self-adjoint in the unconjugated bilinear form <u, v>_S = u^T S v, so
  COCG (CG with the bilinear form u^T v in place of u^H v) applies in that
  form.  Writing rho = S r' for the residual of the original equation and
  r = S^{-1} rho, the coefficients become alpha = (rho^T r)/(p^T q) with
  q = (z S - H) p, and beta = (rho_new^T r_new)/(rho^T r): the only operator
  applications per iteration are one product with (z_s S - H) and one solve
  with S.
* The seed's residual polynomial R_n (R_n(0) = 1) obeys
  R_{n+1}(t) = (1 + beta_{n-1} alpha_n / alpha_{n-1} - alpha_n t) R_n(t)
               - (beta_{n-1} alpha_n / alpha_{n-1}) R_{n-1}(t).
  Since A'(z_k) = A'(z_s) + (z_k - z_s) I, the Krylov spaces of all shifts
  coincide and the shifted residuals are collinear: r^k_n = r_n / pi^k_n with
  pi^k_n = R_n(z_s - z_k), which gives the three-term recurrence for pi used
  below (pi_0 = pi_{-1} = 1, alpha_{-1} = 1, beta_{-1} = 0).
* The shifted coefficients follow as alpha^k = (pi_n/pi_{n+1}) alpha and
  beta^k = (pi_n/pi_{n+1})^2 beta (plain squares: the form is unconjugated),
  and the residual of shift k in the original equation is rho/pi^k, so its
  norm is ||rho|| / |pi^k|.
* Seed switching: when the seed converges while other shifts have not, the
  unconverged shift with the largest residual estimate becomes the seed.
  Its own COCG quantities are the old ones divided by its pi (rho, r by pi,
  gamma = rho^T r by pi^2, and alpha, beta of the step just taken by the
  shifted formulas above); every other shift's pi is re-expressed relative to
  the new seed by dividing by the new seed's pi at the same step.

Readings where the paper is silent (each also listed in the design notes):
x_0 = 0 for every shift; the initial seed is the shift with the smallest
|Im z|, then the real part closest to the median of the real parts, then the
lowest index; convergence is the strict test ||rho||/|pi^k| < tol ||b|| on
the recursive estimate; a converged shift is frozen and never becomes the
seed again; the switch happens at the end of the iteration in which the seed
converged; the inner solve with S is Hermitian CG from zero, stopped when
the recursive residual is <= inner_tol ||rho||.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

CONVERGED, MAXITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3


@dataclass
class ScocgResult:
    x: np.ndarray                 # [M, K] complex128
    iters: np.ndarray             # [K] int: iteration at which shift k converged (-1 if not)
    status: np.ndarray            # [K] int8
    resid: np.ndarray             # [K] recursive residual estimate ||rho||/|pi^k| / ||b||
    n_outer: int                  # iterations performed
    inner_iters: int              # total inner-CG iterations (0 if S = I)
    seeds: list = field(default_factory=list)   # [(iteration, seed index)], first entry (0, s0)


def initial_seed(z: np.ndarray) -> int:
    """Smallest |Im z|; then Re z closest to the median of all Re z; then lowest k.

    The median of an even count is the mean of the two middle values,
    computed as (a + b) / 2.
    """
    z = np.asarray(z, dtype=np.complex128)
    E = np.sort(z.real)
    K = len(E)
    med = E[K // 2] if K % 2 == 1 else (E[K // 2 - 1] + E[K // 2]) / 2.0
    best = 0
    for k in range(1, K):
        a = (abs(z[k].imag), abs(z[k].real - med))
        b = (abs(z[best].imag), abs(z[best].real - med))
        if a < b:
            best = k
    return best


def inner_cg(S, rho: np.ndarray, tol: float, maxiter: int):
    """Solve S r = rho for real SPD S and complex rho by Hermitian CG from 0.

    Stops when the recursive residual satisfies ||res|| <= tol ||rho||.
    Returns (r, iterations).
    """
    nr = np.linalg.norm(rho)
    r = np.zeros_like(rho)
    if nr == 0.0:
        return r, 0
    res = rho.copy()
    d = res.copy()
    rr = np.vdot(res, res).real
    for it in range(maxiter):
        if np.sqrt(rr) <= tol * nr:
            return r, it
        w = S @ d
        a = rr / np.vdot(d, w).real
        r = r + a * d
        res = res - a * w
        rrn = np.vdot(res, res).real
        d = res + (rrn / rr) * d
        rr = rrn
    return r, maxiter


def scocg(H, S, z, b, tol: float, maxiter: Optional[int] = None, inner_tol: float = 1e-13,
          inner_maxiter: int = 1000, seed: Optional[int] = None, s_solve: Optional[Callable] = None,
          record: Optional[Callable] = None) -> ScocgResult:
    """Shifted COCG for (z_k S - H) x = b, all k at once (S = None means I).

    ``seed`` forces the initial seed; ``s_solve`` replaces the inner CG by
    another solver of S r = rho (tests use a dense Cholesky solve);
    ``record(n, dict)`` is called after each iteration's update with the
    state (rho, pi, x, p, seed) for invariant checks.
    """
    z = np.asarray(z, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    M, K = b.shape[0], z.shape[0]
    if maxiter is None:
        maxiter = max(1000, 4 * M)
    inner_total = 0

    def apply_sinv(v):
        nonlocal inner_total
        if S is None:
            return v.copy()
        if s_solve is not None:
            return s_solve(v)
        out, it = inner_cg(S, v, inner_tol, inner_maxiter)
        inner_total += it
        return out

    nu0 = np.linalg.norm(b)
    x = np.zeros((M, K), dtype=np.complex128)
    iters = np.full(K, -1, dtype=np.int64)
    status = np.full(K, MAXITER, dtype=np.int8)
    resid = np.full(K, np.inf)
    if nu0 == 0.0:
        status[:] = CONVERGED
        iters[:] = 0
        resid[:] = 0.0
        return ScocgResult(x, iters, status, resid, 0, 0, [])

    rho = b.copy()
    r = apply_sinv(rho)
    gamma = rho @ r                       # unconjugated
    p = np.repeat(r[:, None], K, axis=1)
    pi = np.ones(K, dtype=np.complex128)
    pi_old = np.ones(K, dtype=np.complex128)
    done = np.zeros(K, dtype=bool)        # converged or broken: frozen
    s = initial_seed(z) if seed is None else int(seed)
    seeds = [(0, s)]
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    n_outer = 0

    for n in range(maxiter):
        n_outer = n + 1
        ps = p[:, s]
        q = z[s] * (ps if S is None else S @ ps) - H @ ps
        mu = ps @ q
        if not np.isfinite(mu) or mu == 0:
            status[~done] = NONFINITE if not np.isfinite(mu) else BREAKDOWN
            resid[~done] = np.linalg.norm(rho) / np.abs(pi[~done]) / nu0
            done[:] = True
            break
        alpha = gamma / mu
        rho = rho - alpha * q
        r = apply_sinv(rho)
        gamma_new = rho @ r
        nu = np.linalg.norm(rho)
        if not np.isfinite(nu) or not np.isfinite(gamma_new):
            status[~done] = NONFINITE
            done[:] = True
            break
        beta = gamma_new / gamma
        gamma = gamma_new

        act = np.flatnonzero(~done)
        pin = (1.0 + alpha * (z[act] - z[s])) * pi[act] + (beta_prev * alpha / alpha_prev) * (pi[act] - pi_old[act])
        bad = ~np.isfinite(pin) | (pin == 0)
        if np.any(bad):
            kb = act[bad]
            status[kb] = np.where(np.isfinite(pin[bad]), BREAKDOWN, NONFINITE)
            done[kb] = True
            act, pin = act[~bad], pin[~bad]
        ratio = pi[act] / pin
        ak = ratio * alpha
        bk = ratio * ratio * beta
        x[:, act] += ak[None, :] * p[:, act]
        p[:, act] = r[:, None] / pin[None, :] + bk[None, :] * p[:, act]
        pi_old[act] = pi[act]
        pi[act] = pin
        est = nu / np.abs(pin)
        resid[act] = est / nu0
        newly = act[est < tol * nu0]
        done[newly] = True
        status[newly] = CONVERGED
        iters[newly] = n + 1
        if record is not None:
            record(n, dict(rho=rho.copy(), r=r.copy(), pi=pi.copy(), x=x.copy(), p=p.copy(), seed=s,
                           alpha=alpha, beta=beta))
        if gamma == 0 and nu > 0 and not np.all(done):
            status[~done] = BREAKDOWN
            done[:] = True
            break
        if np.all(done):
            break
        if done[s]:
            cand = np.flatnonzero(~done)
            # largest residual estimate nu/|pi| == smallest |pi|; ties -> lowest k
            mags = np.abs(pi[cand])
            s_new = int(cand[np.argmin(mags)])
            cn, co = pi[s_new], pi_old[s_new]
            alpha = (co / cn) * alpha
            beta = (co / cn) ** 2 * beta
            rho = rho / cn
            r = r / cn
            gamma = gamma / (cn * cn)
            pi[cand] = pi[cand] / cn
            pi_old[cand] = pi_old[cand] / co
            s = s_new
            seeds.append((n + 1, s))
        alpha_prev, beta_prev = alpha, beta

    return ScocgResult(x, iters, status, resid, n_outer, inner_total, seeds)


def scocg_projected(H, S, z, b, rows, tol: float, maxiter: Optional[int] = None,
                    inner_tol: float = 1e-13, inner_maxiter: int = 1000, seed: Optional[int] = None,
                    s_solve: Optional[Callable] = None) -> ScocgResult:
    """Shifted COCG tracking only the rows ``rows`` of every x_k (projected G).

    The seed runs the three-term (Lanczos) form of COCG, which needs no
    search direction: with r = S^{-1} rho and q = (z_s S - H) r,
        mu_n  = r_n^T q_n - beta_{n-1} gamma_n / alpha_{n-1},  alpha_n = gamma_n / mu_n,
        c_n   = alpha_n beta_{n-1} / alpha_{n-1},
        rho_{n+1} = (1 + c_n) rho_n - alpha_n q_n - c_n rho_{n-1},
    obtained from the two-term form by eliminating p_n with
    (z_s S - H) p_{n-1} = (rho_{n-1} - rho_n) / alpha_{n-1} and the
    orthogonality of successive residuals.  Every shift (the seed included,
    with pi = 1) keeps x_k and p_k on ``rows`` only, updated with the same
    shifted coefficients as in ``scocg``; they read r on ``rows`` only.  A seed
    switch rescales the two latest residuals by the new seed's pi at the same
    steps, so no full vector of any other shift is ever needed.

    Returns a ScocgResult whose x is [len(rows), K].
    """
    z = np.asarray(z, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    rows = np.asarray(rows, dtype=np.int64)
    M, K = b.shape[0], z.shape[0]
    if maxiter is None:
        maxiter = max(1000, 4 * M)
    inner_total = 0

    def apply_sinv(v):
        nonlocal inner_total
        if S is None:
            return v.copy()
        if s_solve is not None:
            return s_solve(v)
        out, it = inner_cg(S, v, inner_tol, inner_maxiter)
        inner_total += it
        return out

    nu0 = np.linalg.norm(b)
    xI = np.zeros((rows.size, K), dtype=np.complex128)
    iters = np.full(K, -1, dtype=np.int64)
    status = np.full(K, MAXITER, dtype=np.int8)
    resid = np.full(K, np.inf)
    rho = b.copy()
    rho_old = np.zeros_like(rho)
    r = apply_sinv(rho)
    r_old = np.zeros_like(r)
    gamma = rho @ r
    pI = np.repeat(r[rows][:, None], K, axis=1)
    pi = np.ones(K, dtype=np.complex128)
    pi_old = np.ones(K, dtype=np.complex128)
    done = np.zeros(K, dtype=bool)
    s = initial_seed(z) if seed is None else int(seed)
    seeds = [(0, s)]
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    n_outer = 0
    for n in range(maxiter):
        n_outer = n + 1
        q = z[s] * (r if S is None else S @ r) - H @ r
        mu = r @ q - beta_prev * gamma / alpha_prev
        if not np.isfinite(mu) or mu == 0:
            status[~done] = NONFINITE if not np.isfinite(mu) else BREAKDOWN
            done[:] = True
            break
        alpha = gamma / mu
        c = alpha * beta_prev / alpha_prev
        rho_new = (1.0 + c) * rho - alpha * q - c * rho_old
        rho_old, rho = rho, rho_new
        r_new = apply_sinv(rho)
        r_old, r = r, r_new
        gamma_new = rho @ r
        nu = np.linalg.norm(rho)
        if not np.isfinite(nu) or not np.isfinite(gamma_new):
            status[~done] = NONFINITE
            done[:] = True
            break
        beta = gamma_new / gamma
        gamma = gamma_new
        act = np.flatnonzero(~done)
        pin = (1.0 + alpha * (z[act] - z[s])) * pi[act] + (beta_prev * alpha / alpha_prev) * (pi[act] - pi_old[act])
        bad = ~np.isfinite(pin) | (pin == 0)
        if np.any(bad):
            kb = act[bad]
            status[kb] = np.where(np.isfinite(pin[bad]), BREAKDOWN, NONFINITE)
            done[kb] = True
            act, pin = act[~bad], pin[~bad]
        ratio = pi[act] / pin
        ak = ratio * alpha
        bk = ratio * ratio * beta
        xI[:, act] += ak[None, :] * pI[:, act]
        pI[:, act] = r[rows][:, None] / pin[None, :] + bk[None, :] * pI[:, act]
        pi_old[act] = pi[act]
        pi[act] = pin
        est = nu / np.abs(pin)
        resid[act] = est / nu0
        newly = act[est < tol * nu0]
        done[newly] = True
        status[newly] = CONVERGED
        iters[newly] = n + 1
        if gamma == 0 and nu > 0 and not np.all(done):
            status[~done] = BREAKDOWN
            done[:] = True
            break
        if np.all(done):
            break
        if done[s]:
            cand = np.flatnonzero(~done)
            s_new = int(cand[np.argmin(np.abs(pi[cand]))])
            cn, co = pi[s_new], pi_old[s_new]
            alpha = (co / cn) * alpha
            beta = (co / cn) ** 2 * beta
            rho, rho_old = rho / cn, rho_old / co
            r, r_old = r / cn, r_old / co
            gamma = gamma / (cn * cn)
            pi[cand] = pi[cand] / cn
            pi_old[cand] = pi_old[cand] / co
            s = s_new
            seeds.append((n + 1, s))
        alpha_prev, beta_prev = alpha, beta
    return ScocgResult(xI, iters, status, resid, n_outer, inner_total, seeds)


# ----------------------------------------------------------------------------
# problems (global or cluster-restricted) — layout only
# ----------------------------------------------------------------------------

def _csr(A):
    from synth import bsr_to_scipy
    return bsr_to_scipy(A)


def local_system(prob, j: int, Hcsr=None, Scsr=None):
    """(H_c, S_c, local index of orbital rhs[j], orbital list) for RHS number j.

    Cluster mode takes the principal submatrices on the cluster's orbitals in
    ascending global order; global mode returns the full matrices.
    """
    bd = prob.bdim
    Hcsr = _csr(prob.H) if Hcsr is None else Hcsr
    if prob.S is not None and Scsr is None:
        Scsr = _csr(prob.S)
    jj = int(prob.rhs[j])
    if prob.cluster_ptr is None:
        orb = np.arange(prob.M)
        return Hcsr, Scsr, jj, orb
    atoms = prob.cluster(j).astype(np.int64)
    orb = (atoms[:, None] * bd + np.arange(bd)[None, :]).ravel()
    Hc = Hcsr[orb][:, orb].tocsr()
    Sc = Scsr[orb][:, orb].tocsr() if Scsr is not None else None
    loc = int(np.searchsorted(orb, jj))
    if loc >= orb.size or orb[loc] != jj:
        raise ValueError("RHS orbital not inside its own cluster")
    return Hc, Sc, loc, orb


def solve_rhs(prob, j: int, tol: Optional[float] = None, Hcsr=None, Scsr=None, full_x=False,
              projected=False, **kw):
    """Solve RHS number j for all shifts; returns (G [K, nout], result, orbitals).

    ``projected`` uses the three-term, rows-only form (``scocg_projected``)."""
    Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
    b = np.zeros(orb.size, dtype=np.complex128)
    b[loc] = 1.0
    outs = prob.outs(j)
    pos = np.searchsorted(orb, outs)
    if projected:
        res = scocg_projected(Hc, Sc, prob.shifts, b, pos, prob.tol if tol is None else tol, **kw)
        return res.x.T.copy(), res, orb
    res = scocg(Hc, Sc, prob.shifts, b, prob.tol if tol is None else tol, **kw)
    G = res.x[pos, :].T.copy()
    if not full_x:
        res.x = None
    return G, res, orb


def _worker(args):
    prob, idx, tol, kw = args
    Hcsr = _csr(prob.H)
    Scsr = _csr(prob.S) if prob.S is not None else None
    out = []
    for j in idx:
        G, res, _ = solve_rhs(prob, j, tol, Hcsr, Scsr, **kw)
        out.append((j, G, res))
    return out


def solve_problem(prob, idx=None, tol: Optional[float] = None, workers: int = 1, **kw):
    """Solve RHS numbers ``idx`` (default all); returns dict of stacked arrays.

    ``workers`` > 1 spreads RHS over processes (one BLAS thread each is the
    caller's business).
    """
    idx = list(range(prob.nrhs)) if idx is None else [int(i) for i in idx]
    if workers <= 1:
        results = _worker((prob, idx, tol, kw))
    else:
        import multiprocessing as mp
        chunks = [idx[w::workers] for w in range(workers)]
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            parts = pool.map(_worker, [(prob, c, tol, kw) for c in chunks if c])
        results = sorted([r for part in parts for r in part], key=lambda t: idx.index(t[0]))
    K = prob.nshift
    return dict(
        idx=np.array(idx),
        G=[r[1] for r in results],
        iters=np.stack([r[2].iters for r in results]) if results else np.zeros((0, K), np.int64),
        status=np.stack([r[2].status for r in results]) if results else np.zeros((0, K), np.int8),
        resid=np.stack([r[2].resid for r in results]) if results else np.zeros((0, K)),
        n_outer=np.array([r[2].n_outer for r in results]),
        inner_iters=np.array([r[2].inner_iters for r in results]),
        seeds=[r[2].seeds for r in results],
    )
