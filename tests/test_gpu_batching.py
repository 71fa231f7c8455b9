"""Batched execution: HIP-graph replay, queue order, autotuned launch shape.

The solver is deterministic (fixed-order reductions, one workgroup per RHS),
so a replayed graph and any RHS order must reproduce the eager run bit for
bit; an autotuned launch shape must give the same answer within the FP64
parity bar.
"""
import numpy as np
import pytest

from synth import make_config, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _cluster(nrhs=12, K=16, seed=(11, 12, 13)):
    return make_problem(name="fcc3", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5), s_scale=0.03, K=K, eta=0.05,
                        nrhs=nrhs, radius=(1.0, 1.6), seed_key=seed)


def _plan(B, prob, **kw):
    P = B.Problem(prob.H, prob.S)
    extra = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        extra.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    extra.update(kw)
    extra.setdefault("tol", prob.tol)
    return P, B.Plan(P, prob.shifts, prob.rhs, **extra)


@pytest.mark.parametrize("form", ["projected", "full", "lanczos", "qmr"])
def test_graph_replay_matches_eager(B, form):
    import torch
    prob = _cluster()
    opt = {"projected": dict(projected=1), "full": dict(projected=0),
           "lanczos": dict(method=B.METHOD_COCG_LANCZOS), "qmr": dict(method=B.METHOD_QMR)}[form]
    P, plan = _plan(B, prob, **opt)
    eager = plan.solve()
    s = torch.cuda.Stream()
    bufs = plan.alloc_outputs()
    with torch.cuda.stream(s):
        plan.capture(bufs, s)
    torch.cuda.synchronize()
    x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        for b in bufs.values():
            b.zero_()
        torch.cuda.synchronize()
        plan.replay(s)
        s.synchronize()
        y = (x * 2.0).sum()                         # eager work between replays
        torch.cuda.synchronize()
        out = bufs["out"].cpu().numpy()
        for r in range(prob.nrhs):
            a, b_ = plan.out_offsets[r] * prob.nshift, plan.out_offsets[r + 1] * prob.nshift
            assert np.array_equal(out[a:b_].reshape(prob.nshift, -1), eager["G"][r]), (rep, r)
        assert np.array_equal(bufs["iters"].cpu().numpy(), eager["iters"])
        assert np.array_equal(bufs["status"].cpu().numpy(), eager["status"])
        del y


@pytest.mark.parametrize("method", [0, 2])
def test_queue_order_changes_nothing(B, method):
    prob = _cluster(nrhs=16)
    P, plan = _plan(B, prob, method=method)
    ref = plan.solve()
    rng = np.random.default_rng(3)
    for order in (np.arange(prob.nrhs)[::-1], rng.permutation(prob.nrhs)):
        P2, plan2 = _plan(B, prob, method=method, order=order.astype(np.int32))
        r = plan2.solve()
        for j in range(prob.nrhs):
            assert np.array_equal(r["G"][j], ref["G"][j])
        assert np.array_equal(r["iters"], ref["iters"])


def test_fewer_slots_than_rhs(B):
    """More RHS than resident workgroups: the queue hands RHS out in turn."""
    prob = _cluster(nrhs=20)
    P, plan = _plan(B, prob, slots=3)
    assert plan.info["slots"] == 3
    r = plan.solve()
    P2, plan2 = _plan(B, prob)
    ref = plan2.solve()
    for j in range(prob.nrhs):
        assert np.array_equal(r["G"][j], ref["G"][j])


def test_autotune(B, tmp_path):
    prob = make_config(1, nrhs=32)
    P = B.Problem(prob.H, prob.S)
    cache = tmp_path / "tune.json"
    res = B.autotune(P, prob.shifts, prob.rhs, probe_iters=50, cache_path=str(cache),
                     out_ptr=prob.out_ptr, out_rows=prob.out_rows, tol=1e-6)
    print("[autotune]", res, flush=True)
    assert res["threads"] in (256, 512, 1024) and 1 <= res["slots"] <= prob.nrhs
    again = B.autotune(P, prob.shifts, prob.rhs, probe_iters=50, cache_path=str(cache),
                       out_ptr=prob.out_ptr, out_rows=prob.out_rows, tol=1e-6)
    assert again == res                               # served from the cache
    small = make_config(0)
    P0 = B.Problem(small.H, None)
    t = B.autotune(P0, small.shifts, small.rhs, probe_iters=100, full_x=True, tol=small.tol)
    kw = dict(full_x=True, tol=small.tol)
    a = B.Plan(P0, small.shifts, small.rhs, **kw).solve()
    b = B.Plan(P0, small.shifts, small.rhs, threads=t["threads"], slots=t["slots"], **kw).solve()
    for j in range(small.nrhs):
        rel = np.linalg.norm(a["G"][j] - b["G"][j], axis=1) / np.linalg.norm(a["G"][j], axis=1)
        assert rel.max() < 1e-8
