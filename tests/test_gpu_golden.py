"""The GPU library, in each solver form, against the stored fixture
tests/golden/sc3_generalized_G.txt (the oracle's values of the same form,
pinned to a dense solve by tests/test_golden.py): per (RHS, shift) relative
difference of the stored rows at most 1e-8, iteration counts within 25%."""
import numpy as np
import pytest

from tests.test_golden import load_fixture, small_generalized

pytestmark = pytest.mark.gpu

FORMS = {"cocg": 0, "cocg_lanczos": 2, "qmr": 1}


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


@pytest.mark.parametrize("form", sorted(FORMS))
def test_gpu_matches_stored_fixture(B, form):
    p = small_generalized()
    stored = {}
    for f, j, i, k, z, g, it in load_fixture():
        if f == form:
            stored.setdefault(j, {})[(i, k)] = (g, it)
    rows = [np.array(sorted({i for (i, _) in stored[int(j)]}), dtype=np.int32) for j in p.rhs]
    out_ptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
    P = B.Problem(p.H, p.S)
    plan = B.Plan(P, p.shifts, p.rhs, out_ptr=out_ptr, out_rows=np.concatenate(rows), tol=p.tol,
                  method=FORMS[form])
    r = plan.solve()
    assert np.all(r["status"] == B.CONVERGED)
    worst = 0.0
    for jj, j in enumerate(p.rhs):
        for k in range(p.nshift):
            ref = np.array([stored[int(j)][(int(i), k)][0] for i in rows[jj]])
            it = stored[int(j)][(int(rows[jj][0]), k)][1]
            err = np.abs(r["G"][jj][k] - ref).max() / np.abs(ref).max()
            worst = max(worst, err)
            assert err <= 1e-8, (form, int(j), k, err)
            assert abs(int(r["iters"][jj][k]) - it) <= max(2, 0.25 * it), (form, int(j), k)
    print(f"[golden] {form}: worst rel err {worst:.1e}", flush=True)
