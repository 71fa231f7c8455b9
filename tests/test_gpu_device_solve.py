"""Device-buffer solve (scocg_solve_device, then scocg_sync): the same
results as the plan API, bit for bit, enqueued on a caller's stream into
caller-owned device buffers; several pending solves; partial convergence
reported by the sync; the empty RHS set."""
import numpy as np
import pytest

from synth import make_config, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


CASES = {
    "cfg0_S=I": lambda: make_config(0, nrhs=4),
    "sc3_generalized": lambda: make_problem(name="sc3-gen", lattice="sc", L=3, bdim=4, s_scale=0.03, K=8, eta=0.05,
                                            nrhs=3, seed_key=(8, 1, 3)),
}


def _device_solve(B, P, prob, stream, **opt):
    import torch
    o = B.scocg_options_default(tol=prob.tol, **opt)
    spec = B.make_spec(None, None, prob.out_ptr, prob.out_rows)
    R, K = prob.nrhs, prob.nshift
    bufs = dict(out=torch.full((int(prob.out_ptr[-1]) * K,), np.nan, dtype=torch.complex128, device="cuda"),
                iters=torch.full((R, K), -7, dtype=torch.int32, device="cuda"),
                status=torch.full((R, K), -7, dtype=torch.int8, device="cuda"),
                resid=torch.full((R, K), np.nan, dtype=torch.float64, device="cuda"))
    B.scocg_solve_device(P.h, o, prob.shifts, prob.rhs, spec, bufs["out"], bufs["iters"], bufs["status"],
                         bufs["resid"], stream)
    return bufs


@pytest.mark.parametrize("method", [0, 2])
@pytest.mark.parametrize("case", sorted(CASES))
def test_device_solve_equals_plan_run(B, case, method):
    import torch
    prob = CASES[case]()
    P = B.Problem(prob.H, prob.S)
    ref = B.Plan(P, prob.shifts, prob.rhs, out_ptr=prob.out_ptr, out_rows=prob.out_rows, tol=prob.tol,
                 method=method).solve()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = _device_solve(B, P, prob, s1, method=method)
    b = _device_solve(B, P, prob, s2, method=method)       # two solves pending at once
    assert B.scocg_sync(P.h) == B.OK
    for bufs in (a, b):
        out = bufs["out"].cpu().numpy()
        off = 0
        for j in range(prob.nrhs):
            n = int(prob.out_ptr[j + 1] - prob.out_ptr[j])
            g = out[off:off + n * prob.nshift].reshape(prob.nshift, n)
            off += n * prob.nshift
            assert np.array_equal(g, ref["G"][j]), (case, method, j)
        assert np.array_equal(bufs["iters"].cpu().numpy(), ref["iters"])
        assert np.array_equal(bufs["status"].cpu().numpy(), ref["status"])
        assert np.array_equal(bufs["resid"].cpu().numpy(), ref["resid"])
    assert B.scocg_sync(P.h) == B.OK                          # nothing pending: immediate OK
    print(f"[device-solve] {case} method {method}: equal to the plan run", flush=True)


def test_sync_reports_partial_convergence(B):
    import torch
    prob = CASES["sc3_generalized"]()
    P = B.Problem(prob.H, prob.S)
    bufs = _device_solve(B, P, prob, torch.cuda.Stream(), maxiter=2)
    assert B.scocg_sync(P.h) == B.W_PARTIAL
    st = bufs["status"].cpu().numpy()
    assert np.all(st == B.MAXITER)
    assert np.all(bufs["iters"].cpu().numpy() == -1)


def test_empty_rhs_and_free_with_pending(B):
    import torch
    prob = CASES["cfg0_S=I"]()
    P = B.Problem(prob.H, prob.S)
    o = B.scocg_options_default(tol=prob.tol)
    spec = B.make_spec(None, None, np.zeros(1, np.int64), np.zeros(0, np.int32))
    dummy = torch.zeros(1, dtype=torch.complex128, device="cuda")
    assert B.scocg_solve_device(P.h, o, prob.shifts, np.zeros(0, np.int32), spec, dummy) == B.OK
    assert B.scocg_sync(P.h) == B.OK
    s = torch.cuda.Stream()
    bufs = _device_solve(B, P, prob, s)
    del P                                                      # problem_free finishes the pending solve first
    torch.cuda.synchronize()
    assert np.all(bufs["status"].cpu().numpy() == B.CONVERGED)
