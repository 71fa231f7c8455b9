"""Pins for the energy-integration oracle (CPU).

The oracle's quadrature is checked against the eigen-expansion of G: with
H y_n = eps_n S y_n (Y^T S Y = I), -(1/pi) Im G_ij(E + i eta) is
sum_n y_in y_jn L(E - eps_n) with the Lorentzian L(x) = (eta/pi)/(x^2 + eta^2),
so the quadrature sum has a closed form that never forms G.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense_solve, integrate as I
from synth import bsr_to_dense, make_problem


def _small(S=True):
    return make_problem(name="int", lattice="sc", L=3, bdim=4, s_scale=0.03 if S else None, K=64, eta=0.1,
                        nrhs=3, seed_key=(7, 1, 3))


def test_fermi_and_weights():
    assert np.allclose(I.fermi([-1.0, 0.0, 1.0], 0.0, 0.0), [1.0, 0.5, 0.0])
    f = I.fermi([0.3], 0.3, 0.1)
    assert np.isclose(f[0], 0.5)
    assert np.isclose(I.fermi([1e3], 0.0, 0.1)[0], 0.0) and np.isclose(I.fermi([-1e3], 0.0, 0.1)[0], 1.0)
    E = np.linspace(-2.0, 3.0, 11)
    w = I.trapezoid_weights(E)
    assert np.isclose(w.sum(), 5.0)
    assert np.isclose(np.sum(w * E ** 1), 0.5 * (9.0 - 4.0))          # trapezoid is exact on linear functions


@pytest.mark.parametrize("with_S", [False, True])
@pytest.mark.parametrize("kT", [0.0, 0.25])
def test_density_matrix_matches_eigen_expansion(with_S, kT):
    p = _small(with_S)
    Hd = bsr_to_dense(p.H)
    Sd = np.eye(p.M) if p.S is None else bsr_to_dense(p.S)
    eps, Y = sla.eigh(Hd, Sd)
    E = p.shifts.real
    eta = p.shifts.imag[0]
    w = I.trapezoid_weights(E)
    mu = 0.4
    f = I.fermi(E, mu, kT)
    for j in p.rhs:
        b = np.zeros(p.M)
        b[j] = 1.0
        G = np.stack([dense_solve(Hd, Sd, z, b) for z in p.shifts])          # [K, M]: G_ij for every i
        rho = I.density_matrix(G, p.shifts, w, mu, kT)
        L = (eta / np.pi) / ((E[:, None] - eps[None, :]) ** 2 + eta ** 2)    # [K, N]
        c = (w * f) @ L                                                       # per eigenpair
        want = (Y * (Y[j, :] * c)[None, :]).sum(axis=1)
        assert np.allclose(rho, want, rtol=1e-10, atol=1e-12)
        nj = I.ldos(G[:, j])
        assert np.allclose(nj, L @ (Y[j, :] ** 2), rtol=1e-10, atol=1e-12)


def test_density_matrix_tends_to_occupied_projector():
    """Small eta on a fine mesh: rho -> sum_n f(eps_n) y_n y_n^T (S-orthonormal y)."""
    p = make_problem(name="int2", lattice="sc", L=3, bdim=4, s_scale=0.03, K=4001, eta=0.02, nrhs=2,
                     seed_key=(7, 1, 4))
    Hd, Sd = bsr_to_dense(p.H), bsr_to_dense(p.S)
    eps, Y = sla.eigh(Hd, Sd)
    # a mesh covering the whole spectrum well beyond eta
    E = np.linspace(eps.min() - 4.0, eps.max() + 4.0, 4001)
    z = E + 1j * 0.02
    w = I.trapezoid_weights(E)
    mu = 0.5 * (eps[p.M // 2 - 1] + eps[p.M // 2])
    j = int(p.rhs[0])
    b = np.zeros(p.M)
    b[j] = 1.0
    Hs = bsr_to_dense(p.H)
    G = np.stack([np.linalg.solve(zz * Sd - Hs, b) for zz in z])
    rho = I.density_matrix(G, z, w, mu, 0.0)
    want = (Y * (Y[j, :] * (eps < mu))[None, :]).sum(axis=1)
    # Lorentzian tails of half-width eta cost O(eta / gap) and O(eta / 4) at the mesh ends
    assert np.abs(rho - want).max() < 0.05


@pytest.mark.parametrize("kT", [0.0, 0.25])
def test_cohp_sum_rule_and_bonds_against_eigen_expansion(kT):
    """Sum over every row i of H_ij rho_ij is (H rho)_jj = sum_n c_n eps_n
    (S y_n)_j y_jn (from H y_n = eps_n S y_n), and the sum over one atom's
    orbitals is sum_{i in b} H_ij sum_n c_n y_in y_jn, both without forming
    G; c_n is the quadrature of f times the Lorentzian of eigenvalue n."""
    p = _small(True)
    Hd, Sd = bsr_to_dense(p.H), bsr_to_dense(p.S)
    eps, Y = sla.eigh(Hd, Sd)
    E = p.shifts.real
    eta = p.shifts.imag[0]
    w = I.trapezoid_weights(E)
    mu = -0.3
    f = I.fermi(E, mu, kT)
    L = (eta / np.pi) / ((E[:, None] - eps[None, :]) ** 2 + eta ** 2)
    c = (w * f) @ L
    SY = Sd @ Y
    bd = p.H.bdim
    for j in p.rhs:
        b = np.zeros(p.M)
        b[j] = 1.0
        G = np.stack([dense_solve(Hd, Sd, z, b) for z in p.shifts])
        rho = I.density_matrix(G, p.shifts, w, mu, kT)
        pop = I.cohp(Hd[:, j], rho)
        band_jj = np.sum(c * eps * SY[j, :] * Y[j, :])
        assert np.isclose(pop.sum(), band_jj, rtol=1e-9, atol=1e-12)
        # the bond between orbital j and each neighbouring atom
        for a in {int(i) // bd for i in np.nonzero(Hd[:, j])[0]}:
            rows = np.arange(a * bd, (a + 1) * bd)
            want = np.sum(Hd[rows, j] * (Y[rows, :] @ (c * Y[j, :])))
            assert np.isclose(pop[rows].sum(), want, rtol=1e-9, atol=1e-12)
