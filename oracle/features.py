"""Oracle for the 16 RHS features — TEST INFRASTRUCTURE ONLY.

Computed from the problem's global block matrices restricted to RHS j's
cluster, in the library's feature order (see include/scocg.h).
"""
import numpy as np


def rhs_features(prob, j):
    bd = prob.bdim
    H, S = prob.H, prob.S
    atoms = prob.cluster(j).astype(np.int64)
    inset = np.zeros(prob.natoms, dtype=bool)
    inset[atoms] = True
    jj = int(prob.rhs[j])
    c, o = jj // bd, jj % bd

    def local_row(a):
        e = np.arange(H.rowptr[a], H.rowptr[a + 1])
        return e[inset[H.colidx[e]]]

    n = atoms.size
    entries = sum(local_row(a).size for a in atoms)
    ec = local_row(c)
    f = np.zeros(16)
    f[0] = n
    f[1] = entries / n
    f[2] = ec.size - 1
    nbr = [e for e in ec if H.colidx[e] != c]
    f[3] = sum(local_row(int(H.colidx[e])).size for e in nbr)
    f[4], f[5], f[6] = float(o == 0), float(1 <= o <= 3), float(o >= 4)
    dblk = [e for e in ec if H.colidx[e] == c][0]
    Hcc = H.vals[dblk]
    f[7] = Hcc[o, o]
    f[8] = np.linalg.norm(Hcc)
    rad = np.abs(Hcc).sum(1) - np.abs(np.diag(Hcc))
    f[9] = np.min(np.diag(Hcc) - rad)
    f[10] = np.max(np.diag(Hcc) + rad)
    fr = np.array([np.linalg.norm(H.vals[e]) for e in nbr])
    f[11] = fr.mean() if fr.size else 0.0
    f[12] = fr.max() if fr.size else 0.0
    f[13] = fr.std() if fr.size else 0.0
    row = np.concatenate([H.vals[e][o] for e in ec])
    f[14] = np.abs(row).sum() - abs(Hcc[o, o])
    f[15] = np.mean([np.linalg.norm(S.vals[e]) for e in nbr]) if (S is not None and nbr) else 0.0
    return f


def all_features(prob):
    return np.stack([rhs_features(prob, j) for j in range(prob.nrhs)])
