"""Synthetic tight-binding inputs (seeded).

The paper's workloads (real amorphous-polymer and carbon structures with
ASED-TB parameters) are not available, so stand-ins are generated with the
properties the paper states for the LCAO matrices (Sec. 8): H real
symmetric, S real symmetric positive definite with unit diagonal and
off-diagonal elements of magnitude below one, both block-sparse on an atomic
neighbour graph with one dense orbital block per atom pair.

Layout.  A block-sparse-row (BSR) matrix over ``nbrows`` atoms with square
``bdim`` x ``bdim`` orbital blocks:

* ``rowptr`` int64[nbrows+1], ``colidx`` int32[nblk] (ascending per row),
* ``vals`` float64[nblk, bdim, bdim], row-major inside each block, so that
  ``vals[e, r, c]`` is the matrix element (a*bdim + r, colidx[e]*bdim + c)
  for the entry ``e`` of block row ``a``.

Randomness.  Every configuration seeds ``numpy.random.default_rng`` from
``SeedSequence([1402, 7285, cfg])`` and spawns seven children, always in the
order (H on-site, H hopping, S hopping, right-hand sides, radii, MLP init,
MLP shuffle), so that every draw is reproducible bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

STREAMS = ("H_onsite", "H_hop", "S_hop", "rhs", "radii", "mlp_init", "mlp_shuffle")


@dataclass
class Bsr:
    nbrows: int
    bdim: int
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray

    @property
    def n(self) -> int:
        return self.nbrows * self.bdim

    @property
    def nblk(self) -> int:
        return int(self.colidx.shape[0])


@dataclass
class Problem:
    """A set of shifted systems (z_k S - H) x = e_j, plus the RHS metadata.

    ``cluster_ptr``/``cluster_atoms`` (CSR over RHS, ascending global atom
    indices) restrict RHS j to the principal submatrix on its local cluster;
    ``None`` means every RHS uses the whole system.  ``out_ptr``/``out_rows``
    list, per RHS, the global orbital indices i for which G_ij is wanted.
    """
    name: str
    lattice: str
    L: int
    bdim: int
    natoms: int
    H: Bsr
    S: Optional[Bsr]
    shifts: np.ndarray
    rhs: np.ndarray
    tol: float
    neighbors: np.ndarray
    coords: np.ndarray            # integer coordinates (see lattice_*)
    coord_scale2: int              # squared distance in a^2 = |coords|^2 / coord_scale2
    radii: Optional[np.ndarray] = None
    cluster_ptr: Optional[np.ndarray] = None
    cluster_atoms: Optional[np.ndarray] = None
    out_ptr: Optional[np.ndarray] = None
    out_rows: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.natoms * self.bdim

    @property
    def nrhs(self) -> int:
        return int(self.rhs.shape[0])

    @property
    def nshift(self) -> int:
        return int(self.shifts.shape[0])

    def cluster(self, j: int) -> np.ndarray:
        """Global atom indices of RHS number j's cluster (all atoms if global)."""
        if self.cluster_ptr is None:
            return np.arange(self.natoms, dtype=np.int32)
        return self.cluster_atoms[self.cluster_ptr[j]:self.cluster_ptr[j + 1]]

    def outs(self, j: int) -> np.ndarray:
        return self.out_rows[self.out_ptr[j]:self.out_ptr[j + 1]]

    def subset(self, idx) -> "Problem":
        """The same matrices with only the RHS numbers in ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        def sub_csr(ptr, vals):
            if ptr is None:
                return None, None
            parts = [vals[ptr[i]:ptr[i + 1]] for i in idx]
            lens = np.array([len(p) for p in parts], dtype=np.int64)
            nptr = np.zeros(len(idx) + 1, dtype=np.int64)
            nptr[1:] = np.cumsum(lens)
            nv = np.concatenate(parts).astype(vals.dtype) if parts else vals[:0]
            return nptr, nv
        cp, ca = sub_csr(self.cluster_ptr, self.cluster_atoms)
        op, orow = sub_csr(self.out_ptr, self.out_rows)
        return Problem(
            name=self.name + f"[{len(idx)}]", lattice=self.lattice, L=self.L,
            bdim=self.bdim, natoms=self.natoms, H=self.H, S=self.S,
            shifts=self.shifts, rhs=self.rhs[idx].copy(), tol=self.tol,
            neighbors=self.neighbors, coords=self.coords,
            coord_scale2=self.coord_scale2,
            radii=None if self.radii is None else self.radii[idx].copy(),
            cluster_ptr=cp, cluster_atoms=ca, out_ptr=op, out_rows=orow,
            meta=dict(self.meta))


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------

def lattice_sc(L: int):
    """Periodic simple-cubic lattice of L^3 atoms, lattice constant a = 1.

    Atom index (x*L + y)*L + z; integer coordinates in units of a; six
    nearest neighbours at distance a.
    """
    if L < 3:
        raise ValueError("simple-cubic lattice needs L >= 3 for distinct neighbours")
    idx = np.arange(L ** 3, dtype=np.int64)
    x, y, z = idx // (L * L), (idx // L) % L, idx % L
    coords = np.stack([x, y, z], axis=1)
    steps = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    nb = np.empty((L ** 3, 6), dtype=np.int64)
    for s, d in enumerate(steps):
        c = (coords + d) % L
        nb[:, s] = (c[:, 0] * L + c[:, 1]) * L + c[:, 2]
    return nb.astype(np.int32), coords.astype(np.int32), 1


_FCC_BASIS = np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]])
# basis index from parity bits (bx*4 + by*2 + bz) of half-unit coordinates
_FCC_FROM_BITS = np.array([0, -1, -1, 1, -1, 2, 3, -1])


def _fcc_index(X, Y, Z, L):
    X, Y, Z = X % (2 * L), Y % (2 * L), Z % (2 * L)
    bits = (X % 2) * 4 + (Y % 2) * 2 + (Z % 2)
    b = _FCC_FROM_BITS[bits]
    if np.any(b < 0):
        raise ValueError("not an fcc site")
    return (((X // 2) * L + (Y // 2)) * L + (Z // 2)) * 4 + b


def lattice_fcc(L: int):
    """Periodic fcc lattice of L^3 cubic cells (4 L^3 atoms), a = 1.

    Atom index ((cx*L + cy)*L + cz)*4 + basis.  Coordinates are integers in
    half-units of a (so every coordinate sum is even); twelve nearest
    neighbours at distance a/sqrt(2).
    """
    if L < 2:
        raise ValueError("fcc lattice needs L >= 2")
    n = 4 * L ** 3
    idx = np.arange(n, dtype=np.int64)
    cell, b = idx // 4, idx % 4
    cx, cy, cz = cell // (L * L), (cell // L) % L, cell % L
    coords = np.stack([2 * cx, 2 * cy, 2 * cz], axis=1) + _FCC_BASIS[b]
    steps = [d for d in _offsets_within(np.sqrt(2.0) / 2 + 1e-9, 4, fcc=True) if any(d)]
    nb = np.empty((n, len(steps)), dtype=np.int64)
    for s, d in enumerate(steps):
        nb[:, s] = _fcc_index(coords[:, 0] + d[0], coords[:, 1] + d[1], coords[:, 2] + d[2], L)
    return nb.astype(np.int32), coords.astype(np.int32), 4


def _offsets_within(r: float, scale2: int, fcc: bool):
    """Integer offset vectors d with |d|^2 <= r^2 * scale2 (fcc: even sums)."""
    R = int(np.floor(np.sqrt(r * r * scale2))) + 1
    g = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    n2 = X * X + Y * Y + Z * Z
    keep = n2 <= r * r * scale2
    if fcc:
        keep &= ((X + Y + Z) % 2) == 0
    out = np.stack([X[keep], Y[keep], Z[keep]], axis=1)
    order = np.lexsort((out[:, 2], out[:, 1], out[:, 0], n2[keep]))
    return out[order]


def cluster_offsets_fcc(r: float):
    return _offsets_within(r, 4, fcc=True)


def cluster_offsets_sc(r: float):
    return _offsets_within(r, 1, fcc=False)


def _cluster_atoms(lattice: str, L: int, coords: np.ndarray, center: int, r: float,
                   offs_cache: dict) -> np.ndarray:
    """Atoms whose minimum-image distance from ``center`` is <= r (units of a)."""
    key = (lattice, r)
    if key not in offs_cache:
        offs_cache[key] = cluster_offsets_fcc(r) if lattice == "fcc" else cluster_offsets_sc(r)
    d = offs_cache[key]
    c = coords[center].astype(np.int64)
    if lattice == "fcc":
        ids = _fcc_index(c[0] + d[:, 0], c[1] + d[:, 1], c[2] + d[:, 2], L)
    else:
        q = (c + d) % L
        ids = (q[:, 0] * L + q[:, 1]) * L + q[:, 2]
    return np.unique(ids).astype(np.int32)


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------

def _pattern(neighbors: np.ndarray):
    """BSR pattern: each atom's own block plus one block per neighbour."""
    n, z = neighbors.shape
    cols = np.concatenate([np.arange(n, dtype=np.int64)[:, None], neighbors.astype(np.int64)], axis=1)
    cols.sort(axis=1)
    rowptr = np.arange(0, (z + 1) * n + 1, z + 1, dtype=np.int64)
    return rowptr, cols.ravel().astype(np.int32)


def _bonds(neighbors: np.ndarray):
    n, z = neighbors.shape
    a = np.repeat(np.arange(n, dtype=np.int64), z)
    b = neighbors.ravel().astype(np.int64)
    keep = a < b
    pairs = np.stack([a[keep], b[keep]], axis=1)
    pairs = np.unique(pairs, axis=0)        # sorted by (a, b)
    return pairs


def _entry_pos(rowptr, colidx, n, rows, cols):
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr)) * n + colidx.astype(np.int64)
    want = rows.astype(np.int64) * n + cols.astype(np.int64)
    pos = np.searchsorted(keys, want)
    assert np.all(keys[pos] == want)
    return pos


def _symmetric_blocks(rng, count, bdim, mean, sd):
    """Blocks drawn on the upper triangle (with diagonal), then mirrored."""
    iu, ju = np.triu_indices(bdim)
    draw = rng.normal(mean, sd, size=(count, iu.size))
    out = np.zeros((count, bdim, bdim))
    out[:, iu, ju] = draw
    out[:, ju, iu] = draw
    return out


def build_H(neighbors, bdim, rng_on, rng_hop, onsite=(0.0, 1.0), hop=(-1.0, 0.5)):
    n = neighbors.shape[0]
    rowptr, colidx = _pattern(neighbors)
    vals = np.zeros((colidx.size, bdim, bdim))
    diag = _entry_pos(rowptr, colidx, n, np.arange(n), np.arange(n))
    vals[diag] = _symmetric_blocks(rng_on, n, bdim, *onsite)
    pairs = _bonds(neighbors)
    T = rng_hop.normal(hop[0], hop[1], size=(pairs.shape[0], bdim, bdim))
    vals[_entry_pos(rowptr, colidx, n, pairs[:, 0], pairs[:, 1])] = T
    vals[_entry_pos(rowptr, colidx, n, pairs[:, 1], pairs[:, 0])] = T.transpose(0, 2, 1)
    return Bsr(n, bdim, rowptr, colidx, vals)


def build_S(neighbors, bdim, rng_s, scale=0.03):
    """S = I + one random block per bond, S_ba = S_ab^T (unit diagonal)."""
    n = neighbors.shape[0]
    rowptr, colidx = _pattern(neighbors)
    vals = np.zeros((colidx.size, bdim, bdim))
    diag = _entry_pos(rowptr, colidx, n, np.arange(n), np.arange(n))
    vals[diag] = np.eye(bdim)
    pairs = _bonds(neighbors)
    T = rng_s.normal(0.0, scale, size=(pairs.shape[0], bdim, bdim))
    vals[_entry_pos(rowptr, colidx, n, pairs[:, 0], pairs[:, 1])] = T
    vals[_entry_pos(rowptr, colidx, n, pairs[:, 1], pairs[:, 0])] = T.transpose(0, 2, 1)
    return Bsr(n, bdim, rowptr, colidx, vals)


def energy_mesh(K: int, eta: float, lo: float = -8.0, hi: float = 8.0) -> np.ndarray:
    """Equally spaced real parts E_k = lo + (hi-lo) k/(K-1), imaginary part eta."""
    if K == 1:
        E = np.array([(lo + hi) / 2])
    else:
        E = lo + (hi - lo) * np.arange(K, dtype=np.float64) / (K - 1)
    return E + 1j * eta


def rngs_for(seed_key) -> dict:
    ss = np.random.SeedSequence(list(seed_key))
    kids = ss.spawn(len(STREAMS))
    return {name: np.random.default_rng(k) for name, k in zip(STREAMS, kids)}


def out_rows_for(neighbors, bdim, rhs):
    """Orbitals of atom c(j) and of its nearest neighbours, ascending."""
    ptr = [0]
    rows = []
    for j in rhs:
        c = int(j) // bdim
        atoms = np.unique(np.concatenate([[c], neighbors[c]]))
        r = (atoms[:, None] * bdim + np.arange(bdim)[None, :]).ravel()
        rows.append(r)
        ptr.append(ptr[-1] + r.size)
    return np.array(ptr, dtype=np.int64), np.concatenate(rows).astype(np.int32)


def make_problem(name="custom", lattice="sc", L=4, bdim=4, onsite=(0.0, 1.0),
                 hop=(-1.0, 0.5), s_scale: Optional[float] = None, K=32, eta=0.05,
                 nrhs=8, tol=1e-10, radius: Optional[tuple] = None,
                 seed_key=(1402, 7285, 1000), mats_key=None, rhs_exclude=None,
                 e_range=(-8.0, 8.0)) -> Problem:
    """Build a problem.  ``mats_key`` (default ``seed_key``) seeds H and S;
    ``seed_key`` seeds the RHS indices and cluster radii."""
    rg = rngs_for(seed_key)
    rgm = rg if mats_key is None or tuple(mats_key) == tuple(seed_key) else rngs_for(mats_key)
    if lattice == "sc":
        nb, coords, sc2 = lattice_sc(L)
    elif lattice == "fcc":
        nb, coords, sc2 = lattice_fcc(L)
    else:
        raise ValueError(lattice)
    natoms = nb.shape[0]
    H = build_H(nb, bdim, rgm["H_onsite"], rgm["H_hop"], onsite, hop)
    S = build_S(nb, bdim, rgm["S_hop"], s_scale) if s_scale is not None else None
    M = natoms * bdim
    pool = np.arange(M)
    if rhs_exclude is not None:
        pool = np.setdiff1d(pool, np.asarray(rhs_exclude))
    rhs = rg["rhs"].choice(pool, size=nrhs, replace=False).astype(np.int32)
    shifts = energy_mesh(K, eta, *e_range)
    prob = Problem(name=name, lattice=lattice, L=L, bdim=bdim, natoms=natoms, H=H, S=S,
                   shifts=shifts, rhs=rhs, tol=tol, neighbors=nb, coords=coords,
                   coord_scale2=sc2)
    prob.meta["rngs"] = rg
    if radius is not None:
        radii = rg["radii"].uniform(radius[0], radius[1], size=nrhs)
        cache: dict = {}
        ptr = [0]
        atoms = []
        for j, r in zip(rhs, radii):
            a = _cluster_atoms(lattice, L, coords, int(j) // bdim, float(r), cache)
            atoms.append(a)
            ptr.append(ptr[-1] + a.size)
        prob.radii = radii
        prob.cluster_ptr = np.array(ptr, dtype=np.int64)
        prob.cluster_atoms = np.concatenate(atoms).astype(np.int32)
    prob.out_ptr, prob.out_rows = out_rows_for(nb, bdim, rhs)
    return prob


# ----------------------------------------------------------------------------
# the five named workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    0: dict(name="cfg0_sc4_S=I", lattice="sc", L=4, bdim=4, hop=(-1.0, 0.5), s_scale=None,
            K=32, eta=0.05, nrhs=8, tol=1e-10),
    1: dict(name="cfg1_sc16_gen", lattice="sc", L=16, bdim=4, hop=(-1.0, 0.5), s_scale=0.03,
            K=128, eta=0.02, nrhs=256, tol=1e-10),
    2: dict(name="cfg2_fcc32_clusters", lattice="fcc", L=32, bdim=9, hop=(0.0, 0.5), s_scale=0.03,
            K=256, eta=0.01, nrhs=4096, tol=1e-10, radius=(2.0, 4.0)),
    # precision variant: the same inputs as config 2, metric tolerance
    3: dict(name="cfg3_fcc32_clusters_fp32", lattice="fcc", L=32, bdim=9, hop=(0.0, 0.5), s_scale=0.03,
            K=256, eta=0.01, nrhs=4096, tol=1e-6, radius=(2.0, 4.0)),
    # learned binning: config-3 shape, 16384 fresh RHS disjoint from config 2's
    4: dict(name="cfg4_fcc32_clusters_16k", lattice="fcc", L=32, bdim=9, hop=(0.0, 0.5), s_scale=0.03,
            K=256, eta=0.01, nrhs=16384, tol=1e-6, radius=(2.0, 4.0)),
}


def _cfg_kwargs(cfg, L=None):
    c = dict(CONFIGS[cfg])
    c.pop("name")
    if L is not None:
        c["L"] = L
    return c


def make_config(cfg: int, nrhs: Optional[int] = None, L: Optional[int] = None,
                radius: Optional[tuple] = None) -> Problem:
    """Build one of the named workloads.

    ``nrhs`` keeps only the first ``nrhs`` RHS in generation order (the
    matrices and the remaining draws are unchanged).  ``L`` shrinks the
    lattice for quick tests (the draws then differ from the full workload).
    ``radius`` replaces the cluster-radius range of configurations 2-4 (in
    lattice constants; the matrices, RHS indices and random streams are
    unchanged, only the uniform radii are rescaled to the new range).
    Configurations 3 and 4 use the matrices of configuration 2; 3 also uses
    its RHS, 4 draws fresh RHS disjoint from configuration 2's.
    """
    name = CONFIGS[cfg]["name"]
    c = _cfg_kwargs(cfg, L)
    if radius is not None:
        if "radius" not in c:
            raise ValueError("configuration has no clusters")
        c["radius"] = tuple(radius)
        name = name + f"_r{radius[0]:g}-{radius[1]:g}"
    full_nrhs = c["nrhs"]
    exclude = None
    if cfg == 3:
        seed_key = mats_key = (1402, 7285, 2)
    elif cfg == 4:
        seed_key, mats_key = (1402, 7285, 4), (1402, 7285, 2)
        c2 = _cfg_kwargs(2, L)
        M2 = 4 * c2["L"] ** 3 * c2["bdim"]
        exclude = rngs_for((1402, 7285, 2))["rhs"].choice(np.arange(M2), size=c2["nrhs"], replace=False)
    else:
        seed_key = mats_key = (1402, 7285, cfg)
    prob = make_problem(name=name, seed_key=seed_key, mats_key=mats_key, rhs_exclude=exclude, **c)
    if nrhs is not None and nrhs < full_nrhs:
        prob = prob.subset(np.arange(nrhs))
        prob.name = name + f"[first {nrhs}]"
    prob.meta["cfg"] = cfg
    return prob


# ----------------------------------------------------------------------------
# conversions (layout only)
# ----------------------------------------------------------------------------

def bsr_to_scipy(A: Bsr):
    import scipy.sparse as sp
    return sp.bsr_matrix((A.vals, A.colidx, A.rowptr), shape=(A.n, A.n)).tocsr()


def bsr_to_dense(A: Bsr) -> np.ndarray:
    return bsr_to_scipy(A).toarray()


# ----------------------------------------------------------------------------
# random draws for the RHS-cost network (initial weights, batch order)
# ----------------------------------------------------------------------------

def mlp_init_weights(rng, nin=16, nh=64):
    """Kaiming-uniform initial weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)),
    zero biases, in the layout W1[nh][nin], b1, W2[nh][nh], b2, W3[nh], b3."""
    w1 = rng.uniform(-np.sqrt(6.0 / nin), np.sqrt(6.0 / nin), size=nh * nin)
    w2 = rng.uniform(-np.sqrt(6.0 / nh), np.sqrt(6.0 / nh), size=nh * nh)
    w3 = rng.uniform(-np.sqrt(6.0 / nh), np.sqrt(6.0 / nh), size=nh)
    return np.concatenate([w1, np.zeros(nh), w2, np.zeros(nh), w3, np.zeros(1)])
