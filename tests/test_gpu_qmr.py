"""GPU solvers on the real S-Lanczos basis: shifted QMR (method = QMR)
against the QMR oracle, and the COCG iterates on that basis (method =
COCG_LANCZOS) against both the oracle of that form and the seed-switching
COCG oracle (the same iterates in exact arithmetic); argument rules.

The parity rule is the projected COCG form's: per (RHS, shift) relative
difference <= 1e-8 with equal status, iteration counts within 25%, else
both inside the a-priori bound of the dense solution."""
import numpy as np
import pytest

from oracle import local_system, scocg_lanczos, scocg_projected, sqmr
from synth import bsr_to_scipy, make_config, make_problem
from tests.parity import compare_rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _plan(B, prob, method=None, **opt):
    P = B.Problem(prob.H, prob.S)
    kw = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        kw.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    opt.setdefault("tol", prob.tol)
    method = B.METHOD_QMR if method is None else method
    return P, B.Plan(P, prob.shifts, prob.rhs, method=method, **kw, **opt)


CASES = {
    "cfg0_S=I": lambda: make_config(0, nrhs=4),
    "sc4_generalized": lambda: make_problem(name="sc4-gen", lattice="sc", L=4, bdim=4, s_scale=0.03, K=16, eta=0.05,
                                            nrhs=4, seed_key=(5, 5, 5)),
    "fcc3_clusters": lambda: make_problem(name="fcc3-clusters", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5),
                                          s_scale=0.03, K=12, eta=0.05, nrhs=6, radius=(1.0, 1.6),
                                          seed_key=(6, 6, 6)),
    # 9x9 blocks on a global system with S: direction in LDS, S as I plus its off-diagonal blocks
    "fcc2_generalized": lambda: make_problem(name="fcc2-gen", lattice="fcc", L=2, bdim=9, hop=(0.0, 0.5),
                                             s_scale=0.03, K=8, eta=0.05, nrhs=3, seed_key=(3, 9, 3)),
    # 4x4 blocks in cluster mode: the block index of each entry comes from its map
    "sc5_clusters": lambda: make_problem(name="sc5-clusters", lattice="sc", L=5, bdim=4, s_scale=0.03, K=8,
                                         eta=0.05, nrhs=4, radius=(1.0, 1.8), seed_key=(9, 2, 7)),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("threads", [512, 1024])
def test_qmr_parity(B, case, threads):
    prob = CASES[case]()
    P, plan = _plan(B, prob, threads=threads)
    assert plan.info["global"] & 4
    assert bool(plan.info["global"] & 16) == (prob.S is not None)
    # a global system whose S has identity diagonal blocks: S = I + off-diagonal copy
    assert bool(plan.info["global"] & 32) == (prob.S is not None and prob.cluster_ptr is None)
    r = plan.solve()
    Hcsr = bsr_to_scipy(prob.H)
    Scsr = bsr_to_scipy(prob.S) if prob.S is not None else None
    worst, report = 0.0, []
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        pos = np.searchsorted(orb, prob.outs(j))
        res = sqmr(Hc, Sc, prob.shifts, b, prob.tol, rows=pos)
        worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hc, Sc, prob.shifts,
                                       b.astype(np.complex128), prob.tol, rows=pos, iter_frac=0.25, report=report,
                                       tag=f"rhs {j}"))
        assert abs(int(r["stats"][j][0]) - res.n_outer) <= max(3, 0.25 * res.n_outer)
        assert r["stats"][j][3] == 0          # no seed switches in the Lanczos form
    print(f"[qmr] {case} threads={threads}: worst rel err {worst:.2e}; shifts with other counts {len(report)}",
          flush=True)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("threads", [512, 1024])
def test_cocg_on_lanczos_basis_parity(B, case, threads):
    prob = CASES[case]()
    P, plan = _plan(B, prob, method=B.METHOD_COCG_LANCZOS, threads=threads)
    assert plan.info["global"] & 8
    # with S != I the inner CG's direction is kept in LDS (it fits at these sizes)
    assert bool(plan.info["global"] & 16) == (prob.S is not None)
    assert bool(plan.info["global"] & 32) == (prob.S is not None and prob.cluster_ptr is None)
    r = plan.solve()
    Hcsr = bsr_to_scipy(prob.H)
    Scsr = bsr_to_scipy(prob.S) if prob.S is not None else None
    worst = [0.0, 0.0]
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        pos = np.searchsorted(orb, prob.outs(j))
        for i, res in enumerate((scocg_lanczos(Hc, Sc, prob.shifts, b, prob.tol, rows=pos),
                                 scocg_projected(Hc, Sc, prob.shifts, b.astype(np.complex128), pos, prob.tol))):
            worst[i] = max(worst[i], compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hc, Sc, prob.shifts,
                                                 b.astype(np.complex128), prob.tol, rows=pos, iter_frac=0.25,
                                                 tag=f"rhs {j} oracle {i}"))
        assert r["stats"][j][3] == 0
    print(f"[cocg-lanczos] {case} threads={threads}: worst rel err vs its oracle {worst[0]:.2e}, "
          f"vs the seed-switching oracle {worst[1]:.2e}", flush=True)


def test_qmr_argument_rules(B):
    prob = make_config(0, nrhs=2)
    with pytest.raises(B.ScocgError) as ei:
        _plan(B, prob, full_x=True)
    assert ei.value.code == B.E_UNSUPPORTED
    with pytest.raises(B.ScocgError) as ei:
        _plan(B, prob, precision=B.FP32)
    assert ei.value.code == B.E_UNSUPPORTED
    with pytest.raises(B.ScocgError) as ei:
        P = B.Problem(prob.H, prob.S)
        B.Plan(P, prob.shifts, prob.rhs, method=7, out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    assert ei.value.code == B.E_ARG


def _ragged_S_problem():
    """sc 5^3 with 4x4 blocks whose S lacks the bond blocks of every atom pair
    with (a + b) % 10 == 0 (both orientations, so S stays symmetric; it stays
    SPD, its off-diagonal part being small): block rows of S then hold 3 to 6
    off-diagonal blocks, so the plan's ELL copy pads the shorter rows with
    their own column and a zero block."""
    prob = make_problem(name="sc5-ragged-S", lattice="sc", L=5, bdim=4, s_scale=0.03, K=12, eta=0.05, nrhs=4,
                        seed_key=(5, 3, 5))
    S = prob.S
    lens = []
    for a in range(S.nbrows):
        n = 0
        for e in range(S.rowptr[a], S.rowptr[a + 1]):
            b = int(S.colidx[e])
            if b != a and (a + b) % 10 == 0:
                S.vals[e] = 0.0
            elif b != a:
                n += 1
        lens.append(n)
    return prob, np.array(lens)


@pytest.mark.parametrize("threads", [512, 1024])
def test_ell_padding_parity(B, threads):
    """The one-workgroup Lanczos-basis kernel on S's off-diagonal blocks in
    ELL form with padded rows (both instances the benchmark chooses between:
    the register form at 512 threads, the memory form at 1024), against the
    oracle of that form."""
    prob, lens = _ragged_S_problem()
    assert lens.min() < lens.max() and 4 * lens.sum() >= 3 * lens.max() * lens.size   # padded, under a quarter
    P, plan = _plan(B, prob, method=B.METHOD_COCG_LANCZOS, threads=threads, team_size=-1)
    info = plan.info
    assert info["threads"] == threads and info["global"] & 32 and info["global"] & 512, info
    assert bool(info["global"] & 256) == (threads == 512), info
    r = plan.solve()
    Hcsr, Scsr = bsr_to_scipy(prob.H), bsr_to_scipy(prob.S)
    worst = 0.0
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        pos = np.searchsorted(orb, prob.outs(j))
        res = scocg_lanczos(Hc, Sc, prob.shifts, b, prob.tol, rows=pos)
        worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hc, Sc, prob.shifts,
                                       b.astype(np.complex128), prob.tol, rows=pos, iter_frac=0.25, tag=f"rhs {j}"))
    print(f"[ell] ragged S, threads={threads}: rows of {lens.min()}-{lens.max()} blocks, worst rel err {worst:.2e}",
          flush=True)
