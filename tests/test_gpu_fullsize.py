"""GPU results at the full workload sizes, checked on sampled outputs.

The oracle's iteration is far too slow at these sizes (a configuration-1
RHS takes minutes on a CPU core), so the check uses what holds at any size:
the exact solution of (z_k S - H) x = e_j from a sparse LU factorisation
(the plain definition of the result) at sampled shifts, and the a-priori
bound ||x - x*|| <= ||A^-1||_2 ||b - A x|| with ||A^-1||_2 <= 1/(|Im z| lam_min(S))
(A = zS - H, H symmetric, S SPD) and lam_min(S) from a Lanczos estimate
less 1%.  The solver stops when its residual estimate is below tol; the
estimate and the true residual agree far below tol in FP64, so twice tol
is used as the residual.  The launch configuration is the one the benchmark
times (1024-thread workgroups, 256 resident), in both solver forms it times.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import CONVERGED, local_system
from synth import bsr_to_scipy, make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _lam_min_lower(Sc):
    """Lower bound on the smallest eigenvalue of the SPD S: the Lanczos
    estimate (scipy eigsh, relative accuracy far below 1e-6 on this well
    conditioned matrix) less 1%."""
    lam = float(sla.eigsh(Sc.tocsc(), k=1, which="SA", tol=1e-10, return_eigenvectors=False)[0])
    assert lam > 0.0
    return 0.99 * lam


def _plan(B, prob, **opt):
    P = B.Problem(prob.H, prob.S)
    kw = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        kw.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    return P, B.Plan(P, prob.shifts, prob.rhs, **kw, **opt)


def _check_sampled(prob, r, shifts_idx, tol, full_x=False, label=""):
    Hcsr = bsr_to_scipy(prob.H)
    Scsr = bsr_to_scipy(prob.S)
    worst_rel, worst_ratio = 0.0, 0.0
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        lam = _lam_min_lower(Sc)
        pos = np.searchsorted(orb, prob.outs(j))
        for k in shifts_idx:
            z = prob.shifts[k]
            b = np.zeros(orb.size, dtype=np.complex128)
            b[loc] = 1.0
            xs = sla.splu((z * Sc - Hc).tocsc()).solve(b)
            g = r["G"][j][k] if not full_x else r["G"][j][k][pos]
            err = np.linalg.norm(g - xs[pos])
            bound = 2.0 * tol / (abs(z.imag) * lam)
            assert err <= bound, f"{label} RHS {j} shift {k}: |G - G*| {err:.2e} > bound {bound:.2e}"
            worst_rel = max(worst_rel, err / np.linalg.norm(xs[pos]))
            worst_ratio = max(worst_ratio, err / bound)
    print(f"[fullsize] {label}: worst rel err of G rows {worst_rel:.2e}, worst err/bound {worst_ratio:.2e}",
          flush=True)
    return worst_rel


FORMS = {"seed-switching projected": 0, "Lanczos-basis": 2}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_cfg1_full_size_sampled(B, form):
    """Configuration 1 at full size (M = 16,384, 128 shifts), four RHS spread
    over the index set, the benchmark's launch shape (the Lanczos-basis form
    is the one the benchmark reports, the seed-switching form its companion);
    two sampled shifts (band centre and band edge) against sparse LU."""
    full = make_config(1)
    prob = full.subset([0, 85, 170, 255])
    tol = 1e-6
    P, plan = _plan(B, prob, tol=tol, threads=1024, slots=256, method=FORMS[form])
    # 1024 threads run unless that instance would spill registers to private memory (the seed-switching
    # kernel does at 1024; it then runs at 512)
    assert plan.info["threads"] == (1024 if FORMS[form] == 2 else 512), plan.info
    assert plan.info["global"] & (8 if FORMS[form] == 2 else 2)
    r = plan.solve()
    assert np.all(r["status"] == CONVERGED)
    assert np.all(r["resid"] <= tol)
    K = prob.nshift
    _check_sampled(prob, r, [K // 2, K - 1], tol, label=f"cfg1 {form} FP64")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_cfg2_full_size_smallest_clusters(B, form):
    """Configuration 2's matrices at full size (fcc 32^3, M = 1,179,648, 256
    shifts); the two RHS with the smallest clusters (M_j = 1,269) of the first
    64, every eighth shift and the last against sparse LU of the local
    system.  (The FP32 forms are checked against the oracle at small sizes:
    at this size their single-shift FP64 fallback, needed below their
    precision floor, runs for minutes.)"""
    full = make_config(2, nrhs=64)
    sizes = np.diff(full.cluster_ptr)
    pick = np.argsort(sizes, kind="stable")[:2]
    prob = full.subset(pick)
    tol = 1e-6
    P, plan = _plan(B, prob, tol=tol, method=FORMS[form])
    assert plan.info["global"] & (8 if FORMS[form] == 2 else 2)
    r = plan.solve()
    assert np.all(r["status"] == CONVERGED)
    assert np.all(r["resid"] <= tol)
    every = list(range(0, prob.nshift, 8)) + [prob.nshift - 1]
    _check_sampled(prob, r, every, tol, label=f"cfg2 {form} FP64")
