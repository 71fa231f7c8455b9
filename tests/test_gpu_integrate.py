"""GPU energy integration of G (density matrix rows, local DOS) against the
oracle: on the GPU's own G (same inputs, so only the summation rounding
differs) and end to end against the oracle's quadrature of the exact G."""
import numpy as np
import pytest

from oracle import dense_solve, integrate as I, local_system
from synth import bsr_to_dense, bsr_to_scipy, make_config, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _run(B, prob, **kw):
    P = B.Problem(prob.H, prob.S)
    spec = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        spec.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    spec.update(kw)
    plan = B.Plan(P, prob.shifts, prob.rhs, tol=prob.tol, **spec)
    bufs = plan.alloc_outputs()
    plan.run(bufs)
    return P, plan, bufs


def _g_blocks(plan, bufs, K):
    out = bufs["out"].cpu().numpy()
    off = plan.out_offsets
    return [out[off[j] * K: off[j + 1] * K].reshape(K, -1) for j in range(plan.nrhs)]


@pytest.mark.parametrize("case", ["cfg0", "clusters"])
@pytest.mark.parametrize("kT", [0.0, 0.3])
def test_integrate_matches_oracle(B, case, kT):
    if case == "cfg0":
        prob = make_config(0)
    else:
        prob = make_problem(name="fcc3-clusters", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5), s_scale=0.03,
                            K=12, eta=0.05, nrhs=6, radius=(1.0, 1.6), seed_key=(6, 6, 6))
    K = prob.nshift
    w = I.trapezoid_weights(prob.shifts.real)
    mu = 0.25
    P, plan, bufs = _run(B, prob)
    rho, ldos = plan.integrate(bufs, w, mu, kT)
    rho, ldos = rho.cpu().numpy(), ldos.cpu().numpy()
    Gs = _g_blocks(plan, bufs, K)
    off = plan.out_offsets
    Hcsr = bsr_to_scipy(prob.H)
    Scsr = bsr_to_scipy(prob.S) if prob.S is not None else None
    worst_e2e = 0.0
    for j in range(prob.nrhs):
        want = I.density_matrix(Gs[j], prob.shifts, w, mu, kT)
        got = rho[off[j]:off[j + 1]]
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())
        Hc, Sc, loc, orb = local_system(prob, j, Hcsr, Scsr)
        pos = np.searchsorted(orb, prob.outs(j))
        d = int(np.where(pos == loc)[0][0])
        assert np.allclose(ldos[j], I.ldos(Gs[j][:, d]), rtol=1e-14, atol=0)
        # end to end: the oracle's quadrature of the exact G
        b = np.zeros(orb.size, dtype=np.complex128)
        b[loc] = 1.0
        Gx = np.stack([dense_solve(Hc, Sc, z, b)[pos] for z in prob.shifts])
        ref = I.density_matrix(Gx, prob.shifts, w, mu, kT)
        worst_e2e = max(worst_e2e, np.abs(got - ref).max() / np.abs(ref).max())
    print(f"[integrate] {case} kT={kT}: worst rel diff to the exact-G quadrature {worst_e2e:.2e}", flush=True)
    assert worst_e2e < 1e-6


def test_integrate_full_x_and_missing_diagonal(B):
    prob = make_config(0, nrhs=3)
    K = prob.nshift
    w = I.trapezoid_weights(prob.shifts.real)
    # full x: every row, the diagonal is row rhs[j]
    P, plan, bufs = _run(B, prob, full_x=True)
    rho, ldos = plan.integrate(bufs, w, 0.0, 0.1)
    rho, ldos = rho.cpu().numpy(), ldos.cpu().numpy()
    Gs = _g_blocks(plan, bufs, K)
    for j in range(prob.nrhs):
        assert Gs[j].shape == (K, prob.M)
        assert np.allclose(rho[j * prob.M:(j + 1) * prob.M], I.density_matrix(Gs[j], prob.shifts, w, 0.0, 0.1),
                           rtol=1e-12, atol=1e-15)
        assert np.allclose(ldos[j], I.ldos(Gs[j][:, prob.rhs[j]]), rtol=1e-14, atol=0)
    # requested rows without the RHS's own orbital: no local DOS (NaN), rho still defined
    rows = [np.setdiff1d(prob.outs(j), [prob.rhs[j]]) for j in range(prob.nrhs)]
    out_ptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
    P2, plan2, bufs2 = _run(B, prob, out_ptr=out_ptr, out_rows=np.concatenate(rows).astype(np.int32))
    rho2, ldos2 = plan2.integrate(bufs2, w, 0.0, 0.1)
    assert np.all(np.isnan(ldos2.cpu().numpy()))
    assert np.all(np.isfinite(rho2.cpu().numpy()))
    # arguments
    with pytest.raises(B.ScocgError):
        plan.integrate(bufs, w, 0.0, -1.0)


@pytest.mark.parametrize("case", ["cfg0", "clusters", "clusters_full_x"])
def test_cohp_matches_oracle(B, case):
    """GPU COHP = H_{row, j} rho per output row, against the oracle's product
    on the GPU's own rho (only the H lookup and the layout can differ, so
    the match is exact); the rows' global orbitals follow the output mode."""
    if case == "cfg0":
        prob = make_config(0)
        kw = {}
    else:
        prob = make_problem(name="fcc3-clusters", lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5), s_scale=0.03,
                            K=12, eta=0.05, nrhs=6, radius=(1.0, 1.6), seed_key=(6, 6, 6))
        kw = dict(full_x=True) if case.endswith("full_x") else {}
    w = I.trapezoid_weights(prob.shifts.real)
    P, plan, bufs = _run(B, prob, **kw)
    rho_d, _ = plan.integrate(bufs, w, 0.1, 0.2)
    cohp = plan.cohp(rho_d).cpu().numpy()
    rho = rho_d.cpu().numpy()
    off = plan.out_offsets
    Hd = bsr_to_scipy(prob.H).tocsc()
    bd = prob.H.bdim
    nonzero = 0
    for j in range(prob.nrhs):
        if case == "clusters_full_x":
            at = prob.cluster_atoms[prob.cluster_ptr[j]:prob.cluster_ptr[j + 1]]
            rows = (at[:, None] * bd + np.arange(bd)[None, :]).ravel()
        else:
            rows = prob.outs(j)
        h = Hd[:, int(prob.rhs[j])].toarray().ravel()[rows]
        want = I.cohp(h, rho[off[j]:off[j + 1]])
        got = cohp[off[j]:off[j + 1]]
        assert got.shape == want.shape
        assert np.array_equal(got, want), (case, j, np.abs(got - want).max())
        nonzero += int(np.count_nonzero(got))
    assert nonzero > 0
    print(f"[cohp] {case}: {cohp.size} rows, {nonzero} nonzero pair populations, equal to the oracle", flush=True)


def test_cohp_sum_rule_full_x(B):
    """Summed over every row of a FULL_X output, the COHP of RHS j is
    (H rho)_jj, which the eigen-expansion gives without G."""
    prob = make_config(0, nrhs=3)
    w = I.trapezoid_weights(prob.shifts.real)
    mu, kT = 0.2, 0.3
    P, plan, bufs = _run(B, prob, full_x=True)
    rho_d, _ = plan.integrate(bufs, w, mu, kT)
    cohp = plan.cohp(rho_d).cpu().numpy()
    Hd = bsr_to_dense(prob.H)
    eps, Y = np.linalg.eigh(Hd)                  # S = I here
    E, eta = prob.shifts.real, prob.shifts.imag[0]
    L = (eta / np.pi) / ((E[:, None] - eps[None, :]) ** 2 + eta ** 2)
    c = (w * I.fermi(E, mu, kT)) @ L
    off = plan.out_offsets
    for j in range(prob.nrhs):
        jj = int(prob.rhs[j])
        band_jj = np.sum(c * eps * Y[jj, :] ** 2)
        got = cohp[off[j]:off[j + 1]].sum()
        assert abs(got - band_jj) <= 1e-6 * max(1.0, abs(band_jj)), (j, got, band_jj)
