"""Shared test helpers: error metrics, closed forms, pattern utilities.

Nothing here implements the method; these are the yardsticks the oracle and
the HIP path are measured with.
"""
from __future__ import annotations

import math

import numpy as np


def diag_positions(colptrL):
    """Index of the diagonal entry of each column in a canonical lower CSC."""
    return np.asarray(colptrL[:-1], dtype=np.int64)


def err_c8(x, o, colptrL, rowindL):
    """max |x_ij - o_ij| / sqrt(o_ii o_jj) over the pattern (selected entries).

    For SPD A, |Ainv_ij| <= sqrt(Ainv_ii Ainv_jj), so the scale is natural."""
    x = np.asarray(x, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    d = o[diag_positions(colptrL)]
    cols = np.repeat(np.arange(len(colptrL) - 1), np.diff(colptrL))
    scale = np.sqrt(np.abs(d[rowindL] * d[cols]))
    scale = np.where(scale > 0, scale, 1.0)
    if len(x) == 0:
        return 0.0
    return float(np.max(np.abs(x - o) / scale))


def colwise_rel(x, o, colptrL, rowindL, n):
    """Column-wise relative difference max_j ||x(:,j)-o(:,j)|| / ||o(:,j)||
    (the paper's accuracy metric, Section 4.2), on the symmetric pattern."""
    cols = np.repeat(np.arange(n), np.diff(colptrL))
    num = np.zeros(n)
    den = np.zeros(n)
    dif2 = (x - o) ** 2
    o2 = o ** 2
    np.add.at(num, cols, dif2)
    np.add.at(den, cols, o2)
    off = rowindL != cols
    np.add.at(num, rowindL[off], dif2[off])
    np.add.at(den, rowindL[off], o2[off])
    return float(np.max(np.sqrt(num) / np.sqrt(den)))


def sel_to_dict(sel, colptrL, rowindL, perm=None):
    """{(i, j): value} in original numbering (i >= j) from canonical values."""
    out = {}
    n = len(colptrL) - 1
    for j in range(n):
        for p in range(colptrL[j], colptrL[j + 1]):
            i = int(rowindL[p])
            a, b = (i, j) if perm is None else (int(perm[i]), int(perm[j]))
            out[(max(a, b), min(a, b))] = float(sel[p])
    return out


def sel_from_dense(ainv, colptrL, rowindL, perm=None):
    """Restrict a dense inverse (original numbering) to the canonical pattern."""
    n = len(colptrL) - 1
    cols = np.repeat(np.arange(n), np.diff(colptrL))
    rows = np.asarray(rowindL, dtype=np.int64)
    if perm is not None:
        perm = np.asarray(perm)
        rows, cols = perm[rows], perm[cols]
    return ainv[rows, cols]


def tridiag_inverse_entry(i, j, n, shift):
    """(A^{-1})_ij of tridiag(-1, 2+shift, -1), 1-based i, j (closed form)."""
    if i > j:
        i, j = j, i
    if shift == 0.0:
        return i * (n + 1 - j) / (n + 1)
    th = math.acosh(1.0 + shift / 2.0)
    return math.sinh(i * th) * math.sinh((n + 1 - j) * th) / (math.sinh(th) * math.sinh((n + 1) * th))


def laplacian_inverse_dense(dims, shift):
    """A^{-1} of the constant-coefficient Dirichlet Laplacian on a box grid
    (index x fastest) from its sine eigenbasis: A = Q diag(lam) Q^T with Q the
    Kronecker product of the 1D bases sqrt(2/(m+1)) sin(k pi p/(m+1))."""
    Qs, lams = [], []
    for m in dims:
        k = np.arange(1, m + 1)
        p = np.arange(1, m + 1)
        Qs.append(np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(p, k) * np.pi / (m + 1)))
        lams.append(4.0 * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2)
    # x fastest: index = x + mx*y + ...; kron order is reversed
    Q = Qs[0]
    lam = lams[0]
    for d in range(1, len(dims)):
        Q = np.kron(Qs[d], Q)
        lam = (lams[d][:, None] + lam[None, :]).ravel()
    lam = lam + shift
    return (Q / lam) @ Q.T


def row_identity(sel, m, colptrL, rowindL, perm):
    """r_i = sum_j A_ij Ainv_ji - 1 for every row, using only selected entries
    (A's pattern lies inside the symmetric pattern of L)."""
    d = sel_to_dict(sel, colptrL, rowindL, perm)
    r, c, v = m.coo_full()
    acc = np.zeros(m.n)
    for i, j, a in zip(r, c, v):
        acc[i] += a * d[(max(i, j), min(i, j))]
    return acc - 1.0


def row_identity_fast(sel, m, colptrL, rowindL, perm, with_scale=False):
    """Vectorised row identity (large cases): sum_j A_ij Ainv_ji - 1 per row,
    and with with_scale also sum_j |A_ij Ainv_ji| (the size of the terms
    that cancel)."""
    n = m.n
    cols = np.repeat(np.arange(n), np.diff(colptrL)).astype(np.int64)
    rows = np.asarray(rowindL, dtype=np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    lo = np.maximum(perm[rows], perm[cols])
    hi = np.minimum(perm[rows], perm[cols])
    key = hi * n + lo
    order = np.argsort(key)
    skey = key[order]
    r, c, v = m.coo_full()
    q = np.minimum(r, c).astype(np.int64) * n + np.maximum(r, c)
    pos = np.searchsorted(skey, q)
    assert np.all(skey[pos] == q), "A's pattern is not inside the pattern of L"
    vals = np.asarray(sel)[order[pos]]
    acc = np.zeros(n)
    np.add.at(acc, r, v * vals)
    if with_scale:
        mag = np.zeros(n)
        np.add.at(mag, r, np.abs(v * vals))
        return acc - 1.0, mag
    return acc - 1.0


def product_identity(sel, m, colptrL, rowindL, perm, rows=None):
    """(A Ainv)_ik - delta_ik over every pair (i, k) at which the product can
    be formed from selected entries alone: all j with A_ij != 0 have (j, k)
    in the symmetric pattern of L (rows: only these i, original numbering).
    Returns (max |residual| / sum_j |A_ij Ainv_jk|, number of pairs checked,
    number of them with i != k)."""
    import scipy.sparse as sp
    n = m.n
    cols = np.repeat(np.arange(n), np.diff(colptrL)).astype(np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    r0, c0 = perm[np.asarray(rowindL, dtype=np.int64)], perm[cols]
    off = r0 != c0
    rr = np.concatenate([r0, c0[off]])
    cc = np.concatenate([c0, r0[off]])
    vv = np.concatenate([np.asarray(sel), np.asarray(sel)[off]])
    S = sp.csr_matrix((vv, (rr, cc)), shape=(n, n))
    Sp = sp.csr_matrix((np.ones_like(vv), (rr, cc)), shape=(n, n))
    ar, ac, av = m.coo_full()
    A = sp.csr_matrix((av, (ar, ac)), shape=(n, n))
    if rows is not None:
        A = A[np.asarray(rows)]
    Ap = A.copy()
    Ap.data[:] = 1.0
    Aabs = abs(A)
    deg = np.diff(Ap.indptr)
    C = (Ap @ Sp).tocoo()  # C_ik = #{j : A_ij != 0 and (j, k) selected}
    full = C.data == deg[C.row]
    i, k = C.row[full], C.col[full]
    gi = np.asarray(rows)[i] if rows is not None else i  # i in the original numbering
    R = (A @ S).tocsr()
    M = (Aabs @ abs(S)).tocsr()
    res = np.asarray(R[i, k]).ravel() - (gi == k)
    mag = np.asarray(M[i, k]).ravel()
    return float(np.max(np.abs(res) / np.maximum(mag, 1e-300))), int(len(i)), int(np.sum(gi != k))
