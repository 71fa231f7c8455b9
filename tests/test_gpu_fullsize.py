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
    # 1024 threads run unless that instance would spill registers to private memory (then 512 runs)
    assert plan.info["threads"] in (512, 1024), plan.info
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


def test_cfg2_full_size_largest_cluster_team(B):
    """Configuration 2's largest cluster among its first 64 RHS (r = 4a class,
    M_j = 9,495), solved by the team solver (the library's choice for
    clusters this large: 16 workgroups split the cluster's rows), every 32nd
    shift and the last against sparse LU of the local system.  One workgroup
    alone needs over two minutes for this RHS; the team bounds the launch by
    a sixteenth of that work plus its waits."""
    full = make_config(2, nrhs=64)
    sizes = np.diff(full.cluster_ptr)
    prob = full.subset([int(np.argmax(sizes))])
    tol = 1e-6
    P, plan = _plan(B, prob, tol=tol, method=2)
    assert plan.info["global"] & 64 and plan.info["team_size"] == 16, plan.info
    r = plan.solve()
    assert np.all(r["status"] == CONVERGED)
    assert np.all(r["resid"] <= tol)
    assert r["stats"][0][4] == 9 * int(sizes.max())
    every = list(range(0, prob.nshift, 32)) + [prob.nshift - 1]
    _check_sampled(prob, r, every, tol, label="cfg2 largest cluster, team of 16")
    print(f"[fullsize] cfg2 largest cluster: {int(r['stats'][0][0])} outer iterations", flush=True)


def test_cfg3_fp32_subset(B):
    """Configuration 3: configuration 2's inputs at tol 1e-6 in the FP32 form
    (FP32 blocks, complex FP32 vectors and updates, FP64 scalar recurrences,
    FP64 seed residual replacement every 20 iterations, FP64 audit of every
    pair and single-shift FP64 re-solve where the audit finds it above tol),
    on the smallest cluster of the first 64 RHS (M_j = 1,269) and every 16th
    of the 256 shifts, the whole x (the FP64 re-solves of the pairs the FP32
    process leaves above tol cost minutes per RHS at all 256 shifts).
    Reported: the maximum relative error of G_jj(z_k) and of x_j(z_k) against
    the exact FP64 solution (sparse LU of z_k S - H on the cluster, the plain
    definition of the result), before and after the audit; required: every
    pair converged with audited residual <= tol, and every x within the
    a-priori bound 2 tol / (|Im z| lam_min(S)) of the exact one."""
    full = make_config(3, nrhs=64)
    sizes = np.diff(full.cluster_ptr)
    prob = full.subset(np.argsort(sizes, kind="stable")[:1])
    shifts = prob.shifts[::16]
    tol = 1e-6
    P = B.Problem(prob.H, prob.S)
    Hcsr, Scsr = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    Hc, Sc, loc, orb = local_system(prob, 0, Hcsr, Scsr)
    lam = _lam_min_lower(Sc)
    b = np.zeros(orb.size, dtype=np.complex128)
    b[loc] = 1.0
    exact = [sla.splu((z * Sc - Hc).tocsc()).solve(b) for z in shifts]
    res = {}
    for audit in (0, 1):
        plan = B.Plan(P, shifts, prob.rhs, full_x=True, cluster_ptr=prob.cluster_ptr,
                      cluster_atoms=prob.cluster_atoms, tol=tol, precision=B.FP32, replace_every=20, method=0,
                      audit=audit)
        r = plan.solve()
        st = r["stats"][0]
        wx = max(np.linalg.norm(r["G"][0][k] - xs) / np.linalg.norm(xs) for k, xs in enumerate(exact))
        wg = max(abs(r["G"][0][k][loc] - xs[loc]) / abs(xs[loc]) for k, xs in enumerate(exact))
        tr = max(np.linalg.norm(b - (z * (Sc @ r["G"][0][k]) - Hc @ r["G"][0][k])) for k, z in enumerate(shifts))
        print(f"[fullsize] cfg3 FP32 (M_j {st[4]}, {shifts.size} shifts, audit {audit}): max rel err G_jj {wg:.2e}, "
              f"x {wx:.2e}; max true residual {tr:.2e}; outer {st[0]}, replacements {st[6]}, "
              f"FP64 re-solve iterations {st[7]}", flush=True)
        res[audit] = r
    r = res[1]
    assert np.all(r["status"] == CONVERGED), r["status"]
    assert np.all(r["resid"] <= tol * 1.0001)
    for k, (z, xs) in enumerate(zip(shifts, exact)):
        err = np.linalg.norm(r["G"][0][k] - xs)
        bound = 2.0 * tol / (abs(z.imag) * lam)
        assert err <= bound, (k, err, bound)
