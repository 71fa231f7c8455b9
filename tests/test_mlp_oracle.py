"""Pins for the MLP and feature oracles (CPU)."""
import numpy as np
import pytest

from oracle import features as F
from oracle import mlp
from synth import bsr_to_dense, make_problem, mlp_init_weights, rngs_for


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16))
    t = rng.normal(size=n)
    w = mlp_init_weights(rngs_for((1, 2, 3))["mlp_init"])
    return w, X, t


def test_param_count_and_pack():
    w, X, t = _data()
    assert mlp.NPARAM == 5313 == w.size
    assert np.array_equal(mlp.pack(mlp.unpack(w)), w)


def test_gradient_central_differences():
    w, X, t = _data()
    w = w + 0.05 * np.random.default_rng(1).normal(size=w.size)      # break symmetric zero biases
    L, g = mlp.loss_and_grad(w, X, t)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(w.size, 60, replace=False), [w.size - 1, 1024, 5248]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss_and_grad(wp, X, t)[0] - mlp.loss_and_grad(wm, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_forward_matches_explicit_loops():
    w, X, t = _data(n=3)
    p = mlp.unpack(w)
    y, _ = mlp.forward(w, X)
    for s in range(3):
        h1 = [max(0.0, sum(p["W1"][j, i] * X[s, i] for i in range(16)) + p["b1"][j]) for j in range(64)]
        h2 = [max(0.0, sum(p["W2"][j, k] * h1[k] for k in range(64)) + p["b2"][j]) for j in range(64)]
        ys = sum(p["W3"][j] * h2[j] for j in range(64)) + p["b3"]
        assert abs(ys - y[s]) < 1e-12


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.1, 1e-3])
    w1, m, v = mlp.adam_step(w, np.zeros(3), np.zeros(3), g, lr=1e-2, step=1)
    assert np.allclose(w1, w - 1e-2 * np.sign(g), atol=1e-7)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(256, 16))
    t = np.tanh(X[:, 0]) + 0.5 * X[:, 1]
    w = mlp_init_weights(rngs_for((9, 9, 9))["mlp_init"])
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    L0 = mlp.loss_and_grad(w, X, t)[0]
    for step in range(1, 301):
        L, g = mlp.loss_and_grad(w, X, t)
        w, m, v = mlp.adam_step(w, m, v, g, 1e-3, step)
    assert mlp.loss_and_grad(w, X, t)[0] < 0.1 * L0


def test_features_against_dense_definitions():
    p = make_problem(lattice="fcc", L=4, bdim=9, hop=(0.0, 0.5), s_scale=0.03, K=4, nrhs=6, radius=(1.2, 1.6),
                     seed_key=(5, 6, 7))
    Hd = bsr_to_dense(p.H)
    Sd = bsr_to_dense(p.S)
    for j in range(p.nrhs):
        f = F.rhs_features(p, j)
        atoms = p.cluster(j)
        orb = (atoms[:, None] * 9 + np.arange(9)[None, :]).ravel()
        jj = int(p.rhs[j])
        c, o = jj // 9, jj % 9
        assert f[0] == atoms.size
        assert f[2] == 12                                 # every fcc neighbour lies within r >= 1.2a
        assert (f[4], f[5], f[6]) == (float(o == 0), float(1 <= o <= 3), float(o >= 4))
        assert f[7] == Hd[jj, jj]
        assert np.isclose(f[8], np.linalg.norm(Hd[c * 9:(c + 1) * 9, c * 9:(c + 1) * 9]))
        row = Hd[jj, orb]
        assert np.isclose(f[14], np.abs(row).sum() - abs(Hd[jj, jj]))
        Hcc = Hd[c * 9:(c + 1) * 9, c * 9:(c + 1) * 9]
        ev = np.linalg.eigvalsh(Hcc)
        assert f[9] <= ev[0] + 1e-12 and ev[-1] <= f[10] + 1e-12       # Gershgorin encloses the spectrum
        # features 1, 3 and 15 from the dense matrices: nonzero 9x9 blocks of the cluster's principal
        # submatrix per atom; nonzero blocks in the cluster rows of c's neighbours; mean ||S_cb||_F over them
        def blk(A, a, b):
            return A[a * 9:(a + 1) * 9, b * 9:(b + 1) * 9]
        nzb = np.array([[np.any(blk(Hd, a, b) != 0) for b in atoms] for a in atoms])
        assert np.isclose(f[1], nzb.sum() / atoms.size)
        ci = int(np.searchsorted(atoms, c))
        nbrs = [i for i in range(atoms.size) if i != ci and nzb[ci, i]]
        assert f[3] == sum(int(nzb[i].sum()) for i in nbrs)
        assert np.isclose(f[15], np.mean([np.linalg.norm(blk(Sd, c, int(atoms[i]))) for i in nbrs]))
    # no hopping: neighbour block norms vanish
    q = make_problem(lattice="fcc", L=3, bdim=9, hop=(0.0, 0.0), K=4, nrhs=2, radius=(1.0, 1.2), seed_key=(1, 1, 1))
    fq = F.rhs_features(q, 0)
    assert fq[11] == fq[12] == fq[13] == 0.0 and fq[15] == 0.0
