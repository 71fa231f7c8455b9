"""The team (panel) solver of the real Lanczos-basis methods against their
oracles: G workgroups share one panel of W right-hand sides (rows split
among the workgroups; with 4x4 blocks and W = 4 or 8 the block products run
on FP64 matrix cores), for the COCG iterates (method COCG_LANCZOS, against
both its own oracle and the seed-switching COCG oracle) and for shifted QMR.

Cases cover every kernel variant: S = I; S with the inner CG's direction in
LDS, with and without S applied as I plus its off-diagonal blocks; the
direction in HBM; 4x4 and 9x9 blocks; global systems and order-N clusters;
a ragged last panel (RHS count not a multiple of W).  The parity rule is
that of the other Lanczos-basis tests (tests/parity.py): per (RHS, shift)
relative difference <= 1e-8 with equal status, iteration counts within 25%,
else both inside the a-priori bound of the dense solution."""
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


def _plan(B, prob, method, **opt):
    P = B.Problem(prob.H, prob.S)
    kw = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        kw.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    opt.setdefault("tol", prob.tol)
    return P, B.Plan(P, prob.shifts, prob.rhs, method=method, **kw, **opt)


def _check(B, prob, plan, method, tag):
    r = plan.solve()
    Hcsr = bsr_to_scipy(prob.H)
    Scsr = bsr_to_scipy(prob.S) if prob.S is not None else None
    worst = 0.0
    for j in range(prob.nrhs):
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        b = np.zeros(orb.size)
        b[loc] = 1.0
        pos = np.searchsorted(orb, prob.outs(j))
        if method == B.METHOD_QMR:
            refs = [sqmr(Hc, Sc, prob.shifts, b, prob.tol, rows=pos)]
        else:
            refs = [scocg_lanczos(Hc, Sc, prob.shifts, b, prob.tol, rows=pos),
                    scocg_projected(Hc, Sc, prob.shifts, b.astype(np.complex128), pos, prob.tol)]
        for i, res in enumerate(refs):
            worst = max(worst, compare_rhs(r["G"][j], r["iters"][j], r["status"][j], res, Hc, Sc, prob.shifts,
                                           b.astype(np.complex128), prob.tol, rows=pos, iter_frac=0.25,
                                           tag=f"{tag} rhs {j} oracle {i}"))
        n_or = refs[0].n_outer
        assert abs(int(r["stats"][j][0]) - n_or) <= max(3, 0.25 * n_or), (j, r["stats"][j][0], n_or)
        assert r["stats"][j][4] == orb.size, (j, r["stats"].tolist())
    # the per-RHS shift-update counters add up over the team's workgroups
    assert np.all(r["stats"][:, 1] >= r["stats"][:, 0])
    assert np.all(r["stats"][:, 1] <= r["stats"][:, 0] * prob.nshift)
    print(f"[team] {tag}: worst rel err {worst:.2e}; outer iterations {r['stats'][:, 0].tolist()}", flush=True)
    return r


def _sc4(nrhs=12):
    return make_problem(name="sc4-gen", lattice="sc", L=4, bdim=4, s_scale=0.03, K=16, eta=0.05, nrhs=nrhs,
                        seed_key=(5, 5, 5))


# (problem, W, G, threads, expected variant flags)
CASES = {
    # panels on matrix cores: S = I + off-diagonal blocks, direction in LDS; 12 RHS = one full and one half panel
    "sc4_W8_G2": (_sc4, 8, 2, 1024),
    "sc4_W8_G4_512": (_sc4, 8, 4, 512),
    "sc4_W4_G2": (_sc4, 4, 2, 512),
    "sc4_W4_G1": (_sc4, 4, 1, 1024),
    # S = I (no inner CG)
    "cfg0_W8_G2": (lambda: make_config(0, nrhs=8), 8, 2, 1024),
    # one RHS per team, rows split: 4x4 blocks (DPP quad path), 9x9 clusters, 9x9 global
    "sc4_W1_G4": (lambda: _sc4(6), 1, 4, 512),
    "fcc3_clusters_G2": (lambda: make_problem(name="fcc3-clusters", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5),
                                              s_scale=0.03, K=12, eta=0.05, nrhs=6, radius=(1.0, 1.6),
                                              seed_key=(6, 6, 6)), 1, 2, 512),
    "sc5_clusters_G4": (lambda: make_problem(name="sc5-clusters", lattice="sc", L=5, bdim=4, s_scale=0.03, K=8,
                                             eta=0.05, nrhs=4, radius=(1.0, 1.8), seed_key=(9, 2, 7)), 1, 4, 1024),
    "fcc2_generalized_G2": (lambda: make_problem(name="fcc2-gen", lattice="fcc", L=2, bdim=9, hop=(0.0, 0.5),
                                                 s_scale=0.03, K=8, eta=0.05, nrhs=3, seed_key=(3, 9, 3)),
                            1, 2, 512),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("regs", [1, 0])
def test_team_cocg_lanczos_parity(B, case, regs):
    mk, W, G, nt = CASES[case]
    prob = mk()
    P, plan = _plan(B, prob, B.METHOD_COCG_LANCZOS, team_size=G, panel_width=W, threads=nt, team_registers=regs)
    info = plan.info
    # the inner CG's vectors in registers: only if asked, with S != I, 4x4 blocks and panels of 4 or 8, and
    # only for instances that keep every value in registers (512 threads, W = 4 here)
    rv = bool(info["global"] & 256)
    if not (regs and prob.S is not None and W % 4 == 0 and prob.bdim == 4):
        assert not rv, info
    if regs and case == "sc4_W4_G2":
        assert rv and info["threads"] == 512, info
    assert info["global"] & 64, info                      # the team solver runs
    assert info["team_size"] == G and info["panel_width"] == W
    # the requested workgroup size runs unless its instance would spill registers (then the other one)
    assert info["threads"] in (512, 1024)
    assert bool(info["global"] & 128) == (W % 4 == 0 and prob.bdim == 4)    # matrix cores
    if prob.S is not None:
        assert info["global"] & 16                          # the CG direction fits in LDS here
        assert bool(info["global"] & 32) == (prob.cluster_ptr is None)
    _check(B, prob, plan, B.METHOD_COCG_LANCZOS, f"cocg-lanczos {case}")


@pytest.mark.parametrize("case", ["sc4_W8_G2", "sc4_W4_G2", "cfg0_W8_G2", "fcc3_clusters_G2", "sc5_clusters_G4"])
@pytest.mark.parametrize("regs", [1, 0])
def test_team_qmr_parity(B, case, regs):
    mk, W, G, nt = CASES[case]
    prob = mk()
    P, plan = _plan(B, prob, B.METHOD_QMR, team_size=G, panel_width=W, threads=nt, team_registers=regs)
    assert plan.info["global"] & 64
    _check(B, prob, plan, B.METHOD_QMR, f"qmr {case}")


def test_team_direction_in_hbm(B):
    """A panel whose CG direction does not fit in LDS (M W doubles on one
    workgroup): the variant that keeps it in HBM."""
    prob = make_problem(name="sc12-gen", lattice="sc", L=12, bdim=4, s_scale=0.03, K=6, eta=0.5, nrhs=4,
                        seed_key=(12, 4, 12))
    P, plan = _plan(B, prob, B.METHOD_COCG_LANCZOS, team_size=1, panel_width=4, threads=512)
    assert plan.info["global"] & 64 and not plan.info["global"] & 16, plan.info
    _check(B, prob, plan, B.METHOD_COCG_LANCZOS, "cocg-lanczos sc12 W4 G1 direction in HBM")


def test_team_argument_rules(B):
    prob = _sc4(4)
    for bad in (dict(panel_width=3), dict(panel_width=16), dict(team_size=33)):
        with pytest.raises(B.ScocgError) as ei:
            _plan(B, prob, B.METHOD_COCG_LANCZOS, **bad)
        assert ei.value.code == B.E_ARG, bad
    with pytest.raises(B.ScocgError) as ei:
        _plan(B, prob, B.METHOD_COCG_LANCZOS, team_size=2, threads=256)
    assert ei.value.code == B.E_ARG
    # panels of several RHS need the whole system and 4x4 blocks
    cl = make_problem(name="sc5-clusters", lattice="sc", L=5, bdim=4, s_scale=0.03, K=8, eta=0.05, nrhs=4,
                      radius=(1.0, 1.8), seed_key=(9, 2, 7))
    with pytest.raises(B.ScocgError) as ei:
        _plan(B, cl, B.METHOD_COCG_LANCZOS, panel_width=4)
    assert ei.value.code == B.E_UNSUPPORTED
    # team_size -1: the one-workgroup solver
    P, plan = _plan(B, prob, B.METHOD_COCG_LANCZOS, team_size=-1)
    assert not plan.info["global"] & 64 and plan.info["team_size"] == 1


@pytest.mark.parametrize("case", ["fcc3", "sc5"])
def test_team_many_panels_per_team_repeatable(B, case):
    """Two teams take sixteen order-N clusters of different sizes from the
    work queue, so every team solves panel after panel on the same workspace
    (each panel's first products read the neighbours' rows of b, which must
    be this panel's, not the last one's).  Against the oracles, and three
    runs bitwise the same: the team's sums are in a fixed order, so any
    difference between runs is a read of another workgroup's data before it
    was written."""
    if case == "fcc3":
        prob = make_problem(name="fcc3-clusters", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5), s_scale=0.03, K=12,
                            eta=0.05, nrhs=16, radius=(1.0, 1.6), seed_key=(6, 6, 6))
        G = 2
    else:
        prob = make_problem(name="sc5-clusters", lattice="sc", L=5, bdim=4, s_scale=0.03, K=8, eta=0.05, nrhs=16,
                            radius=(1.0, 1.8), seed_key=(9, 2, 7))
        G = 4
    P, plan = _plan(B, prob, B.METHOD_COCG_LANCZOS, team_size=G, panel_width=1, threads=512, slots=2 * G)
    assert plan.info["global"] & 64 and plan.info["team_size"] == G, plan.info
    assert plan.info["slots"] == 2 * G, plan.info
    r0 = _check(B, prob, plan, B.METHOD_COCG_LANCZOS, f"cocg-lanczos {case} 2 teams x 8 panels")
    for rep in range(2):
        r = plan.solve()
        for j in range(prob.nrhs):
            assert np.array_equal(r["G"][j], r0["G"][j]), (rep, j)
        assert np.array_equal(r["status"], r0["status"]) and np.array_equal(r["iters"], r0["iters"]), rep
        assert np.array_equal(r["stats"], r0["stats"]), rep
