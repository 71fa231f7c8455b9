"""Generator checks: the stand-in matrices have the properties the paper
states for the LCAO Hamiltonian and overlap (Sec. 2: real symmetric, overlap
positive definite; Sec. 8: unit overlap diagonal, off-diagonal overlap
elements of magnitude below one) and the draws are reproducible."""
import numpy as np
import pytest

from synth import (bsr_to_dense, cluster_offsets_fcc, cluster_offsets_sc, lattice_fcc,
                   lattice_sc, make_config, make_problem)


def test_sc_neighbours():
    nb, coords, s2 = lattice_sc(5)
    assert nb.shape == (125, 6)
    for a in range(125):
        d = (coords[nb[a]] - coords[a] + 2) % 5 - 2
        assert sorted((d * d).sum(1).tolist()) == [1] * 6
        assert len(set(nb[a].tolist())) == 6


def test_fcc_neighbours():
    nb, coords, s2 = lattice_fcc(3)
    assert nb.shape == (108, 12)
    for a in range(108):
        d = (coords[nb[a]] - coords[a] + 3) % 6 - 3
        assert sorted((d * d).sum(1).tolist()) == [2] * 12   # |d|^2 = 2 half-units^2 = a^2/2
        assert len(set(nb[a].tolist())) == 12
        for b in nb[a]:
            assert a in nb[b]


def test_fcc_cluster_counts_brute_force():
    """Offsets within r (units of a) against a brute-force count over fcc sites."""
    for r in (0.75, 1.0, 2.0, 2.5, 4.0):
        offs = cluster_offsets_fcc(r)
        R = int(np.ceil(r)) + 1
        cnt = 0
        for cx in range(-R, R + 1):
            for cy in range(-R, R + 1):
                for cz in range(-R, R + 1):
                    for b in ((0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)):
                        p = np.array([cx, cy, cz]) + np.array(b)
                        if (p * p).sum() <= r * r:
                            cnt += 1
        assert len(offs) == cnt
    assert len(cluster_offsets_fcc(2.0)) == 141
    assert len(cluster_offsets_fcc(4.0)) == 1061
    assert len(cluster_offsets_sc(1.0)) == 7


@pytest.mark.parametrize("lattice,L,bd,s", [("sc", 4, 4, None), ("sc", 3, 4, 0.03), ("fcc", 2, 9, 0.03)])
def test_matrix_properties(lattice, L, bd, s):
    p = make_problem(lattice=lattice, L=L, bdim=bd, s_scale=s, hop=(-1.0, 0.5), nrhs=4)
    H = bsr_to_dense(p.H)
    assert np.array_equal(H, H.T)
    z = 6 if lattice == "sc" else 12
    assert p.H.nblk == p.natoms * (z + 1)
    if s is not None:
        S = bsr_to_dense(p.S)
        assert np.array_equal(S, S.T)
        assert np.all(np.diag(S) == 1.0)
        off = S - np.diag(np.diag(S))
        assert np.abs(off).max() < 1.0
        assert np.linalg.eigvalsh(S)[0] > 0.1


def test_cfg1_overlap_spd_and_shapes():
    p = make_config(1)
    assert p.M == 16384 and p.nshift == 128 and p.nrhs == 256
    assert p.H.nblk == 4096 * 7
    # lambda_min(S) by a few Lanczos steps of S - c I (sparse, cheap)
    import scipy.sparse.linalg as spl
    from synth import bsr_to_scipy
    S = bsr_to_scipy(p.S)
    lmin = spl.eigsh(S, k=1, which="SA", tol=1e-6, return_eigenvectors=False)[0]
    assert lmin > 0.1
    assert np.allclose(p.shifts.imag, 0.02)
    E = p.shifts.real
    assert E[0] == -8.0 and E[-1] == 8.0 and np.allclose(np.diff(E), 16 / 127)


def test_reproducible_and_cfg4_disjoint():
    a = make_config(0)
    b = make_config(0)
    assert np.array_equal(a.H.vals, b.H.vals) and np.array_equal(a.rhs, b.rhs)
    p2 = make_problem(lattice="fcc", L=3, bdim=9, hop=(0.0, 0.5), s_scale=0.03, nrhs=20,
                      radius=(1.0, 1.5), seed_key=(1, 2, 3))
    sizes = np.diff(p2.cluster_ptr)
    assert sizes.min() >= 13
    for j in range(p2.nrhs):
        atoms = p2.cluster(j)
        assert np.all(np.diff(atoms) > 0)
        assert int(p2.rhs[j]) // 9 in atoms
        assert set((p2.outs(j) // 9).tolist()) <= set(atoms.tolist())
