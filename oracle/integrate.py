"""Oracle for the energy integration of G — TEST INFRASTRUCTURE ONLY.

Once G_ij(z_k) is known on the energy mesh z_k = E_k + i eta, the quantities
the paper uses G for follow by integrating over energy (Sec. 2-3: the
Green's function as the analysis object; the density of states and the
density matrix of the electronic structure):

  local density of states  n_j(E_k) = -(1/pi) Im G_jj(E_k + i eta)
  density matrix           rho_ij   = -(1/pi) sum_k w_k f(E_k) Im G_ij(E_k + i eta)

with quadrature weights w_k on the real-axis mesh and the Fermi function
f(E) = 1 / (1 + exp((E - mu) / kT)) (a step, 1/2 at E = mu, for kT = 0).
In the S-orthonormal eigenbasis (H y_n = eps_n S y_n), G_ij(z) =
sum_n y_in y_jn / (z - eps_n), so -(1/pi) Im G is a sum of Lorentzians of
half-width eta and rho_ij tends to sum_n f(eps_n) y_in y_jn as eta -> 0 on
a fine mesh.  The sums below are written out in that order; no blocking.

The paper's bond analysis (Sec. 2, a COHP extension based on G) splits the
band energy tr(rho H) = sum_ij H_ji rho_ij into pair terms: the integrated
crystal-orbital Hamilton population of the pair (i, j) is H_ij rho_ij
(H symmetric), and its sum over the orbitals i of an atom b is the
population of the bond between orbital j and atom b.
"""
import numpy as np


def fermi(E, mu, kT):
    """Fermi-Dirac occupation; kT = 0 gives the step with 1/2 at E = mu."""
    E = np.asarray(E, dtype=np.float64)
    if kT == 0.0:
        return np.where(E < mu, 1.0, np.where(E > mu, 0.0, 0.5))
    return 0.5 * (1.0 - np.tanh(0.5 * (E - mu) / kT))     # = 1/(1 + exp((E - mu)/kT)), no overflow


def trapezoid_weights(E):
    """Trapezoid weights of an ascending real mesh E_0 < ... < E_{K-1}."""
    E = np.asarray(E, dtype=np.float64)
    w = np.zeros_like(E)
    if E.size > 1:
        d = np.diff(E)
        w[:-1] += 0.5 * d
        w[1:] += 0.5 * d
    return w


def ldos(G_diag, shifts=None):
    """-(1/pi) Im G_jj at every mesh point (G_diag: [K] complex)."""
    return -np.imag(np.asarray(G_diag)) / np.pi


def density_matrix(G, shifts, weights, mu, kT):
    """rho_i for the rows of G ([K, n] complex, row k at z_k = shifts[k])."""
    G = np.asarray(G)
    f = fermi(np.real(shifts), mu, kT)
    acc = np.zeros(G.shape[1], dtype=np.float64)
    for k in range(G.shape[0]):
        acc += weights[k] * f[k] * np.imag(G[k])
    return -acc / np.pi


def cohp(h_col, rho):
    """Integrated COHP H_ij rho_ij of the listed rows i of one RHS j
    (h_col[i] = H_ij, rho[i] = rho_ij as density_matrix returns it)."""
    return np.asarray(h_col, dtype=np.float64) * np.asarray(rho, dtype=np.float64)
