"""Seeded synthetic inputs for selected inversion.

This module only builds matrices (pattern + values) and the geometry that the
ordering step needs. It holds none of the method's arithmetic, so both the
HIP path and the CPU oracle can be fed from it.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014). A stream is seeded with
``(seed << 8) | stream``. Uniform draws are ``(x >> 11) * 2**-53``; normal
draws use the Box-Muller transform on consecutive uniform pairs.

Every matrix is returned as the lower triangle (diagonal included) in CSC form:
``colptr`` (int64, n+1), ``rowind`` (int32, sorted within a column, so the
diagonal comes first) and ``vals`` (float64). The paper's test matrices are
not available here; these grids and the jittered-lattice block matrix stand in
for its PDE and localized-basis classes (Section 4, Tables 1 and 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


class SplitMix64:
    """splitmix64 stream; ``next_u64(k)`` returns the next k outputs."""

    def __init__(self, seed: int, stream: int = 0):
        self.state = np.uint64(((int(seed) << 8) | int(stream)) & 0xFFFFFFFFFFFFFFFF)

    def next_u64(self, k: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            steps = np.arange(1, k + 1, dtype=np.uint64)
            z = self.state + steps * _GOLDEN
            self.state = self.state + np.uint64(k) * _GOLDEN
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, k: int) -> np.ndarray:
        x = self.next_u64(k)
        return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, k: int) -> np.ndarray:
        m = (k + 1) // 2
        u = self.uniform(2 * m)
        u1, u2 = u[0::2], u[1::2]
        r = np.sqrt(-2.0 * np.log1p(-u1))
        out = np.empty(2 * m)
        out[0::2] = r * np.cos(2.0 * math.pi * u2)
        out[1::2] = r * np.sin(2.0 * math.pi * u2)
        return out[:k]


@dataclass
class Matrix:
    """Sparse symmetric matrix as a lower-triangular CSC plus its geometry."""

    n: int
    colptr: np.ndarray  # int64[n+1]
    rowind: np.ndarray  # int32[nnz]
    vals: np.ndarray  # float64[nnz]
    ndim: int = 0  # 0: no geometry (natural order unless a perm is given)
    dims: tuple = (1, 1, 1)
    dofs: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def dense(self) -> np.ndarray:
        """Full symmetric dense matrix (small cases only)."""
        a = np.zeros((self.n, self.n))
        for j in range(self.n):
            for p in range(self.colptr[j], self.colptr[j + 1]):
                i = self.rowind[p]
                a[i, j] = self.vals[p]
                a[j, i] = self.vals[p]
        return a

    def coo_full(self):
        """(rows, cols, vals) of the full symmetric matrix."""
        cols = np.repeat(np.arange(self.n), np.diff(self.colptr))
        rows = self.rowind.astype(np.int64)
        off = rows != cols
        r = np.concatenate([rows, cols[off]])
        c = np.concatenate([cols, rows[off]])
        v = np.concatenate([self.vals, self.vals[off]])
        return r, c, v


def _lower_csc_from_pairs(n, rows, cols, vals):
    """Sum duplicates and return (colptr, rowind, vals) of the lower triangle."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    lo = np.maximum(rows, cols)
    hi = np.minimum(rows, cols)
    key = hi * n + lo
    order = np.argsort(key, kind="stable")
    key = key[order]
    v = np.asarray(vals, dtype=np.float64)[order]
    uniq, start = np.unique(key, return_index=True)
    sums = np.add.reduceat(v, start) if len(v) else v
    c = uniq // n
    r = uniq % n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, r.astype(np.int32), sums


def grid_edges(dims):
    """Interior edges of a box grid, axis-major, each axis ordered by the lower
    endpoint's index (x fastest); then ghost (boundary) edges by point index,
    directions -x,+x,-y,+y,-z,+z. Returns (u, v, is_ghost) with v=-1 for ghosts."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    full = list(dims) + [1] * (3 - nd)
    mx, my, mz = full
    n = mx * my * mz
    idx = np.arange(n, dtype=np.int64)
    x = idx % mx
    y = (idx // mx) % my
    z = idx // (mx * my)
    coords = [x, y, z]
    strides = [1, mx, mx * my]
    us, vs = [], []
    for d in range(nd):
        sel = coords[d] < full[d] - 1
        us.append(idx[sel])
        vs.append(idx[sel] + strides[d])
    gu, gd = [], []
    # ghost edges: for each point, for each direction with the neighbour outside
    gmask = np.zeros((n, 2 * nd), dtype=bool)
    for d in range(nd):
        gmask[:, 2 * d] = coords[d] == 0
        gmask[:, 2 * d + 1] = coords[d] == full[d] - 1
    pi, di = np.nonzero(gmask)  # row-major: point index then direction
    return (np.concatenate(us) if us else np.zeros(0, np.int64),
            np.concatenate(vs) if vs else np.zeros(0, np.int64),
            pi.astype(np.int64), di.astype(np.int64))


def laplacian(dims, coeff="const", lo=1.0, hi=1.0, shift=0.0, seed=0):
    """Finite-difference Laplacian on a box grid with Dirichlet ghost edges.

    A_ii = sum of incident edge weights (interior and ghost) + shift and
    A_ij = -c_ij. ``coeff``: "const" (c=1), "uniform" (U[lo,hi]) or
    "loguniform" (exp(U[ln lo, ln hi])); one draw per edge in edge order
    (interior, then ghost) from stream 0 of ``seed``.
    """
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    u, v, gp, gd = grid_edges(dims)
    ne = len(u) + len(gp)
    if coeff == "const":
        w = np.ones(ne)
    else:
        r = SplitMix64(seed, 0).uniform(ne)
        if coeff == "uniform":
            w = lo + (hi - lo) * r
        elif coeff == "loguniform":
            w = np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * r)
        else:
            raise ValueError(coeff)
    wi, wg = w[: len(u)], w[len(u):]
    diag = np.full(n, float(shift))
    np.add.at(diag, u, wi)
    np.add.at(diag, v, wi)
    np.add.at(diag, gp, wg)
    rows = np.concatenate([np.arange(n), v])
    cols = np.concatenate([np.arange(n), u])
    vals = np.concatenate([diag, -wi])
    colptr, rowind, vals = _lower_csc_from_pairs(n, rows, cols, vals)
    full = list(dims) + [1] * (3 - nd)
    return Matrix(n, colptr, rowind, vals, ndim=nd, dims=tuple(full), dofs=1,
                  meta=dict(kind="laplacian", dims=dims, coeff=coeff, lo=lo, hi=hi,
                            shift=shift, seed=seed))


def tridiag_1d(n, shift=0.0):
    """tridiag(-1, 2+shift, -1): the 1D Laplacian with Dirichlet ends."""
    return laplacian((n,), shift=shift)


def batch_2d(count=256, side_lo=32, side_hi=96, shift_lo=0.01, shift_hi=1.0, seed=3):
    """Independent 2D 5-point grids: sides ~ U{side_lo..side_hi} (all drawn
    first), then shifts ~ U[shift_lo, shift_hi], both from stream 0."""
    g = SplitMix64(seed, 0)
    span = side_hi - side_lo + 1
    sides = side_lo + np.floor(g.uniform(count) * span).astype(np.int64)
    shifts = shift_lo + (shift_hi - shift_lo) * g.uniform(count)
    return [laplacian((int(m), int(m)), shift=float(s)) for m, s in zip(sides, shifts)]


def molecular(side=16, dofs=8, cutoff=1.8, jitter=0.1, seed=4, shift=None):
    """Block-sparse symmetric matrix on a jittered cubic lattice of atoms.

    Atom a sits at its lattice point plus U[-jitter, jitter]^3 (stream 0, three
    draws per atom in atom order). Atoms a<b closer than ``cutoff`` (strict)
    get a dofs x dofs block of N(0,1) entries (stream 1, row-major, pairs in
    (a, b) order after all self blocks); a self block is (G+G^T)/2 with G
    N(0,1). Unknown dofs*a+k is basis function k of atom a. The matrix is made
    positive definite with shift = ceil(-lambda_min*1000)/1000 + 0.5 unless a
    shift is given; lambda_min comes from Lanczos (scipy eigsh).
    """
    na = side ** 3
    idx = np.arange(na)
    pos = np.stack([idx % side, (idx // side) % side, idx // (side * side)], 1).astype(np.float64)
    pos += -jitter + 2 * jitter * SplitMix64(seed, 0).uniform(3 * na).reshape(na, 3)
    pairs_a, pairs_b = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                off = dx + side * dy + side * side * dz
                if off <= 0:
                    continue
                x, y, z = pos[:, 0].round(), pos[:, 1].round(), pos[:, 2].round()
                ok = ((x + dx >= 0) & (x + dx < side) & (y + dy >= 0) & (y + dy < side)
                      & (z + dz >= 0) & (z + dz < side))
                a = idx[ok]
                b = a + off
                d = np.linalg.norm(pos[a] - pos[b], axis=1)
                keep = d < cutoff
                pairs_a.append(a[keep])
                pairs_b.append(b[keep])
    pa = np.concatenate(pairs_a)
    pb = np.concatenate(pairs_b)
    order = np.lexsort((pb, pa))
    pa, pb = pa[order], pb[order]
    g = SplitMix64(seed, 1)
    selfb = g.normal(na * dofs * dofs).reshape(na, dofs, dofs)
    selfb = 0.5 * (selfb + selfb.transpose(0, 2, 1))
    pairb = g.normal(len(pa) * dofs * dofs).reshape(len(pa), dofs, dofs)
    k = np.arange(dofs)
    rr, cc = np.meshgrid(k, k, indexing="ij")
    rows = [(dofs * idx[:, None, None] + rr).ravel(), (dofs * pb[:, None, None] + rr).ravel()]
    cols = [(dofs * idx[:, None, None] + cc).ravel(), (dofs * pa[:, None, None] + cc).ravel()]
    vals = [selfb.ravel(), pairb.ravel()]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    # keep the lower triangle of the self blocks once (they are symmetric)
    lowmask = rows >= cols
    n = na * dofs
    colptr, rowind, v = _lower_csc_from_pairs(n, rows[lowmask], cols[lowmask], vals[lowmask])
    if shift is None:
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        cc_ = np.repeat(np.arange(n), np.diff(colptr))
        low = sp.csc_matrix((v, rowind, colptr), shape=(n, n))
        full = low + sp.tril(low, -1).T
        lam = spla.eigsh(full, k=1, which="SA", tol=1e-8, return_eigenvectors=False,
                         v0=np.ones(n))[0]
        shift = math.ceil(-lam * 1000.0) / 1000.0 + 0.5
        del cc_
    diagpos = colptr[:-1]
    v = v.copy()
    v[diagpos] += shift
    return Matrix(n, colptr, rowind, v, ndim=3, dims=(side, side, side), dofs=dofs,
                  meta=dict(kind="molecular", side=side, dofs=dofs, cutoff=cutoff,
                            jitter=jitter, seed=seed, shift=shift))


def hamiltonian_overlap(side=8, dofs=8, cutoff=1.8, jitter=0.1, seed=6):
    """A pair (H, S) on one pattern, for the pole expansion A(z) = H - z S.

    H is the block matrix of ``molecular`` with no diagonal shift (real
    symmetric, indefinite).  S has the same lower pattern: identity plus
    0.1 x N(0,1) entries (stream 2 of the same seed; self blocks symmetrised
    through the lower-triangle storage), then shifted on the diagonal so that
    its smallest eigenvalue (Lanczos) is at least 0.5 (positive definite, like
    an overlap matrix of a localized basis).  Returns (H, S) as Matrix
    objects with identical colptr/rowind."""
    H = molecular(side=side, dofs=dofs, cutoff=cutoff, jitter=jitter, seed=seed, shift=0.0)
    g = SplitMix64(seed, 2)
    v = 0.1 * g.normal(H.nnz)
    v[H.colptr[:-1]] += 1.0
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    low = sp.csc_matrix((v, H.rowind, H.colptr), shape=(H.n, H.n))
    full = low + sp.tril(low, -1).T
    lam = spla.eigsh(full, k=1, which="SA", tol=1e-8, return_eigenvectors=False, v0=np.ones(H.n))[0]
    shift = max(0.0, math.ceil((0.5 - lam) * 1000.0) / 1000.0)
    v[H.colptr[:-1]] += shift
    S = Matrix(H.n, H.colptr, H.rowind, v, ndim=H.ndim, dims=H.dims, dofs=H.dofs,
               meta=dict(kind="overlap", seed=seed, shift=shift))
    H.meta["kind"] = "hamiltonian"
    return H, S


def indefinite_molecular(side=4, dofs=8, cutoff=1.8, jitter=0.1, seed=8, coupling=0.08):
    """Symmetric indefinite block matrix whose diagonal blocks need 2x2
    pivots.  On the ``molecular`` pattern, every atom's self block is the
    saddle-point block [[0, I], [I, 0]] (basis functions 0..dofs/2-1 paired
    with dofs/2..dofs-1, eigenvalues +1 and -1, zero diagonal), and every
    other entry is ``coupling`` times the ``molecular`` value (N(0,1)
    entries, no shift); the diagonal stays exactly 0.  An LDL^T with 1x1
    pivots and no interchanges stops at the first column; 2x2 pivots inside
    the diagonal blocks do not."""
    m = molecular(side=side, dofs=dofs, cutoff=cutoff, jitter=jitter, seed=seed, shift=0.0)
    v = coupling * m.vals
    cols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    rows = m.rowind.astype(np.int64)
    same_atom = rows // dofs == cols // dofs
    v[same_atom] = 0.0
    h = dofs // 2
    pair = same_atom & (rows % dofs == cols % dofs + h) & (cols % dofs < h)
    v[pair] = 1.0
    return Matrix(m.n, m.colptr, m.rowind, v, ndim=m.ndim, dims=m.dims, dofs=m.dofs,
                  meta=dict(kind="indefinite", side=side, dofs=dofs, seed=seed, coupling=coupling))


def poles(count, center, radius):
    """Poles z_k = center + radius * exp(i pi (k + 1/2) / count), k < count:
    points on the upper half of a circle around the spectrum, never real
    (Im z > 0 keeps A(z) = H - z S nonsingular for SPD S)."""
    k = np.arange(count)
    return center + radius * np.exp(1j * np.pi * (k + 0.5) / count)


def pencil_values(H, S, z):
    """Values of A(z) = H - z S on the common lower pattern (complex)."""
    assert np.array_equal(H.colptr, S.colptr) and np.array_equal(H.rowind, S.rowind)
    return H.vals - z * S.vals


def fig1_pattern():
    """The 29x29 example of Fig. 1 (Section 2.1): lower pattern, 0-based.

    Diagonal blocks of the ten supernodes are dense; off-diagonal blocks are
    read from the figure (rows 11 and 15 of block (5,2) and row 27 of block
    (10,6) are blank). Values: 10 on the diagonal, -1 off the diagonal, which
    keeps the matrix diagonally dominant.
    """
    sn = [(0, 2), (2, 4), (4, 8), (8, 10), (10, 16), (16, 18), (18, 20), (20, 23), (23, 25), (25, 29)]
    blocks = [
        ([2, 3], (0, 2)), ([10, 12, 13, 14], (2, 4)), ([8, 9], (4, 8)),
        (list(range(10, 16)), (8, 10)), ([23, 24], (10, 16)), ([20, 21, 22], (16, 18)),
        ([25, 26, 28], (16, 18)), ([20, 21, 22], (18, 20)), ([23, 24], (20, 23)),
        ([25, 26, 27, 28], (23, 25)),
    ]
    rows, cols = [], []
    for a, b in sn:
        for j in range(a, b):
            for i in range(j, b):
                rows.append(i)
                cols.append(j)
    for rs, (a, b) in blocks:
        for j in range(a, b):
            for i in rs:
                rows.append(i)
                cols.append(j)
    n = 29
    vals = [10.0 if r == c else -1.0 for r, c in zip(rows, cols)]
    colptr, rowind, v = _lower_csc_from_pairs(n, rows, cols, vals)
    return Matrix(n, colptr, rowind, v, ndim=0, meta=dict(kind="fig1"))


def random_spd_pattern(n, density, seed):
    """Random sparse symmetric diagonally dominant matrix (small tests)."""
    g = SplitMix64(seed, 0)
    m = n * n
    u = g.uniform(m).reshape(n, n)
    vals = g.uniform(m).reshape(n, n)
    rows, cols, vs = [], [], []
    for j in range(n):
        for i in range(j + 1, n):
            if u[i, j] < density:
                rows.append(i)
                cols.append(j)
                vs.append(-(0.5 + vals[i, j]))
    deg = np.zeros(n)
    for i, j, w in zip(rows, cols, vs):
        deg[i] += -w
        deg[j] += -w
    rows += list(range(n))
    cols += list(range(n))
    vs += list(deg + 1.0)
    colptr, rowind, v = _lower_csc_from_pairs(n, rows, cols, vs)
    return Matrix(n, colptr, rowind, v, ndim=0, meta=dict(kind="random", density=density, seed=seed))


CONFIGS = {
    "lap2d_32": dict(fn=laplacian, kw=dict(dims=(32, 32), shift=0.1), cap=128),
    "lap3d_40": dict(fn=laplacian, kw=dict(dims=(40, 40, 40), coeff="uniform", lo=0.5, hi=2.0,
                                          shift=1e-2, seed=2), cap=128),
    "lap3d_64": dict(fn=laplacian, kw=dict(dims=(64, 64, 64), coeff="loguniform", lo=0.1, hi=10.0,
                                          shift=1e-3, seed=5), cap=256),
    "molecular_16": dict(fn=molecular, kw=dict(side=16, dofs=8, seed=4), cap=128),
}


def make(name: str) -> Matrix:
    c = CONFIGS[name]
    return c["fn"](**c["kw"])
