"""Pins for the CPU oracle: each check comes from outside the oracle itself
(closed forms, the paper's worked example, brute force, invariants), and a
planted mistake in any part of the oracle fails at least one of them."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_0447_amd import workloads as W
from tests import helpers as H

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(autouse=True)
def _no_mutation():
    O.set_mutation(0)
    yield
    O.set_mutation(0)


# ---------------------------------------------------------------- ordering
def test_nd_order_hand_examples():
    # 1D, 7 points: halves {0,1,2} and {4,5,6} split at 1 and 5, root plane 3
    assert list(O.nd_order(1, (7,))) == [0, 2, 1, 4, 6, 5, 3]
    # 3x3 grid: x is split first (tie goes to the lowest axis)
    assert list(O.nd_order(2, (3, 3))) == [0, 6, 3, 2, 8, 5, 1, 4, 7]
    # dofs stay contiguous per point
    assert list(O.nd_order(1, (3,), dofs=2)) == [0, 1, 4, 5, 2, 3]


@pytest.mark.parametrize("dims", [(5,), (6, 4), (7, 3, 5), (16, 16), (9, 9, 9)])
def test_nd_order_is_a_separating_permutation(dims):
    p = O.nd_order(len(dims), dims)
    n = int(np.prod(dims))
    assert sorted(p) == list(range(n))
    # the last vertex eliminated is on a plane that splits the longest axis
    m = W.laplacian(dims)
    s = O.symbolic(m, cap=10 ** 9).sym
    # a separator ordered last: the root supernode's columns disconnect the rest
    assert s.parent[-1] == -1


# ---------------------------------------------------------------- Fig. 1
def test_fig1_structure():
    g = json.load(open(os.path.join(GOLD, "fig1.json")))
    m = W.fig1_pattern()
    s = O.symbolic(m, cap=6, perm="natural").sym
    assert s.nnzL == g["nnzL"]
    assert list(s.parent) == g["column_parent"]
    # the fill is exactly the "+" block of the figure
    A = set()
    for j in range(m.n):
        for p in range(m.colptr[j], m.colptr[j + 1]):
            A.add((int(m.rowind[p]), j))
    Lset = set()
    for j in range(m.n):
        for p in range(s.colptrL[j], s.colptrL[j + 1]):
            Lset.add((int(s.rowindL[p]), j))
    fill = Lset - A
    exp = {(r, c) for r in g["fill"]["rows"] for c in g["fill"]["cols"]}
    assert fill == exp
    got = [[int(s.xsuper[k]), int(s.xsuper[k + 1])] for k in range(s.N)]
    assert got == g["fundamental_supernodes_cap6"]


def test_fig1_block_tree_and_priorities():
    """Block etree and Algorithm 2 priorities for the paper's own partition,
    derived from the oracle's column tree."""
    g = json.load(open(os.path.join(GOLD, "fig1.json")))
    m = W.fig1_pattern()
    s = O.symbolic(m, cap=6, perm="natural").sym
    part = g["paper_supernodes"]
    sn = np.empty(m.n, dtype=int)
    for k, (a, b) in enumerate(part):
        sn[a:b] = k
    bpar = {}
    for k, (a, b) in enumerate(part):
        p = s.parent[b - 1]
        bpar[str(k + 1)] = None if p < 0 else int(sn[p]) + 1
    assert bpar == g["paper_block_parent"]
    sigma = {}
    for k in range(len(part), 0, -1):
        sigma[str(k)] = 1 if bpar[str(k)] is None else sigma[str(bpar[str(k)])] + 1
    assert sigma == g["paper_priority"]


def test_fig1_priority_levels_fundamental():
    m = W.fig1_pattern()
    s = O.symbolic(m, cap=6, perm="natural").sym
    # root = merged {23..28} -> 1; {10..15},{20..22} -> 2; four -> 3; two -> 4
    assert list(s.level) == [4, 3, 4, 3, 2, 3, 3, 2, 1]


# ---------------------------------------------------------------- brute force symbolic
def _brute_pattern(m, perm):
    n = m.n
    ip = np.empty(n, dtype=int)
    ip[perm] = np.arange(n)
    B = np.zeros((n, n), dtype=bool)
    r, c, _ = m.coo_full()
    B[ip[r], ip[c]] = True
    for k in range(n):  # Gaussian elimination on the pattern
        nz = np.nonzero(B[k + 1:, k])[0] + k + 1
        B[np.ix_(nz, nz)] = True
    return B


@pytest.mark.parametrize("seed", range(6))
def test_symbolic_vs_brute_force_elimination(seed):
    m = W.random_spd_pattern(40, 0.08, seed)
    perm = np.random.default_rng(seed).permutation(m.n).astype(np.int32)
    cap = 4 + seed
    s = O.symbolic(m, cap=cap, perm=perm).sym
    B = _brute_pattern(m, perm)
    for j in range(m.n):
        rows = [int(x) for x in s.rowindL[s.colptrL[j]:s.colptrL[j + 1]]]
        exp = [j] + [int(i) for i in np.nonzero(B[j + 1:, j])[0] + j + 1]
        assert rows == exp
        assert s.parent[j] == (exp[1] if len(exp) > 1 else -1)
    # supernodes: contiguous, dense diagonal block, same structure below, <= cap
    for k in range(s.N):
        a, b = int(s.xsuper[k]), int(s.xsuper[k + 1])
        assert 1 <= b - a <= cap
        below = set(np.nonzero(B[b:, a])[0] + b)
        for j in range(a, b):
            assert set(np.nonzero(B[j + 1:, j])[0] + j + 1) == set(range(j + 1, b)) | below
    # maximality: neighbours could not have been merged
    for k in range(s.N - 1):
        a, b = int(s.xsuper[k]), int(s.xsuper[k + 1])
        j = b - 1
        only_child = s.parent[j] == j + 1 and int(np.sum(s.parent == j + 1)) == 1
        same = set(np.nonzero(B[j + 1:, j])[0] + j + 1) == {j + 1} | set(np.nonzero(B[j + 2:, j + 1])[0] + j + 2)
        assert (b - a == cap) or not (only_child and same)


# ---------------------------------------------------------------- 1D closed form
@pytest.mark.parametrize("n,shift,perm", [(50, 0.0, "natural"), (63, 0.3, "nd"), (200, 1e-2, "nd")])
def test_tridiagonal_closed_form(n, shift, perm):
    m = W.tridiag_1d(n, shift)
    osym = O.symbolic(m, cap=8, perm=perm)
    s = osym.sym
    sel, _, st, _, _, _ = osym.factor_selinv(m.vals)
    assert st == 0
    exp = np.array([H.tridiag_inverse_entry(int(s.perm[i]) + 1, int(s.perm[j]) + 1, n, shift)
                    for j in range(n) for i in s.rowindL[s.colptrL[j]:s.colptrL[j + 1]]])
    assert H.err_c8(sel, exp, s.colptrL, s.rowindL) < 1e-12
    if perm == "natural":  # natural order: pattern = diagonal + subdiagonal (linear work)
        assert s.nnzL == 2 * n - 1


def test_tridiagonal_dense_tiers():
    n, shift = 40, 0.5
    m = W.tridiag_1d(n, shift)
    a = m.dense()
    inv = O.dense_inverse(a)
    exp = np.array([[H.tridiag_inverse_entry(i + 1, j + 1, n, shift) for j in range(n)] for i in range(n)])
    assert np.max(np.abs(inv - exp)) < 1e-13
    s = O.symbolic(m, cap=4, perm="nd").sym
    ap = a[np.ix_(s.perm, s.perm)]
    sel2 = O.selinv_columns(ap, s.colptrL, s.rowindL)
    assert H.err_c8(sel2, H.sel_from_dense(exp, s.colptrL, s.rowindL, s.perm), s.colptrL, s.rowindL) < 1e-13


# ---------------------------------------------------------------- 2D/3D closed form
@pytest.mark.parametrize("dims,shift,cap", [((8, 8), 0.0, 128), ((32, 32), 0.1, 128), ((5, 4, 3), 0.2, 4),
                                           ((9, 9, 9), 1e-2, 16)])
def test_grid_spectral_closed_form(dims, shift, cap):
    m = W.laplacian(dims, shift=shift)
    osym = O.symbolic(m, cap=cap)
    s = osym.sym
    sel, _, st, _, _, _ = osym.factor_selinv(m.vals)
    assert st == 0
    exact = H.laplacian_inverse_dense(dims, shift)
    exp = H.sel_from_dense(exact, s.colptrL, s.rowindL, s.perm)
    assert H.err_c8(sel, exp, s.colptrL, s.rowindL) < 1e-11
    # strict positivity (irreducible Stieltjes matrix)
    assert np.all(sel > 0)


def test_cfg1_sizes():
    m = W.make("lap2d_32")
    s = O.symbolic(m, cap=128).sym
    assert (m.n, m.nnz) == (1024, 3008)
    # symbolic sizes of the 32x32 grid under the bisection order
    assert s.nnzL == 15836 and s.N == 663 and int(s.level.max()) == 19


# ---------------------------------------------------------------- tiers agree
@pytest.mark.parametrize("seed", range(4))
def test_o3_o2_o1_random(seed):
    m = W.random_spd_pattern(120, 0.04, seed + 10)
    perm = np.random.default_rng(seed).permutation(m.n).astype(np.int32)
    osym = O.symbolic(m, cap=3 + 5 * seed, perm=perm)
    s = osym.sym
    sel3, _, st, _, _, _ = osym.factor_selinv(m.vals)
    assert st == 0
    a = m.dense()
    inv = O.dense_inverse(a)
    exp = H.sel_from_dense(inv, s.colptrL, s.rowindL, s.perm)
    sel2 = O.selinv_columns(a[np.ix_(s.perm, s.perm)], s.colptrL, s.rowindL)
    assert H.err_c8(sel3, exp, s.colptrL, s.rowindL) < 1e-12
    assert H.err_c8(sel2, exp, s.colptrL, s.rowindL) < 1e-12
    # O1 itself: A @ Ainv = I
    assert np.max(np.abs(a @ inv - np.eye(m.n))) < 1e-12


def test_molecular_small_tiers():
    m = W.molecular(side=3, dofs=4, seed=1)
    osym = O.symbolic(m, cap=16)
    s = osym.sym
    sel3, _, st, _, _, _ = osym.factor_selinv(m.vals)
    assert st == 0
    a = m.dense()
    inv = O.dense_inverse(a)
    exp = H.sel_from_dense(inv, s.colptrL, s.rowindL, s.perm)
    assert H.err_c8(sel3, exp, s.colptrL, s.rowindL) < 1e-11
    assert np.min(np.linalg.eigvalsh(a)) >= 0.5 - 1e-6  # shift recipe: lambda_min >= 0.5


# ---------------------------------------------------------------- invariants
def test_invariants_cfg1():
    m = W.make("lap2d_32")
    osym = O.symbolic(m, cap=128)
    s = osym.sym
    sel, _, st, _, _, _ = osym.factor_selinv(m.vals)
    r = H.row_identity_fast(sel, m, s.colptrL, s.rowindL, s.perm)
    assert np.max(np.abs(r)) < 1e-12
    d = sel[s.colptrL[:-1]]
    cols = np.repeat(np.arange(m.n), np.diff(s.colptrL))
    assert np.all(np.abs(sel) <= np.sqrt(d[s.rowindL] * d[cols]) * (1 + 1e-12))
    assert np.all(sel > 0)


@pytest.mark.parametrize("case", ["lap2d_32", "molecular_3", "lap3d_9x8x7", "random"])
def test_product_identity(case):
    """(A Ainv)_ik = delta_ik at every pair (i, k), i != k included, whose
    terms are all selected entries (A_ij != 0 implies (j, k) in the pattern):
    beyond the row identity, this pins entries of the pattern that are not
    entries of A."""
    m = {"lap2d_32": lambda: W.make("lap2d_32"), "molecular_3": lambda: W.molecular(side=3, dofs=8, seed=4),
         "lap3d_9x8x7": lambda: W.laplacian((9, 8, 7), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=2),
         "random": lambda: W.random_spd_pattern(300, 0.03, 11)}[case]()
    o = O.symbolic(m, cap=16)
    sel = o.factor_selinv(m.vals)[0]
    rel, npairs, noff = H.product_identity(sel, m, o.sym.colptrL, o.sym.rowindL, o.sym.perm)
    assert noff >= 500 and rel <= 1e-12, (rel, npairs, noff)


@pytest.mark.parametrize("mutation", [1, 2, 4])
def test_product_identity_catches_planted_mistakes(mutation):
    m = W.laplacian((9, 8, 7), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=2)
    o = O.symbolic(m, cap=16)
    O.set_mutation(mutation)
    try:
        sel = o.factor_selinv(m.vals)[0]
    finally:
        O.set_mutation(0)
    rel = H.product_identity(sel, m, o.sym.colptrL, o.sym.rowindL, o.sym.perm)[0]
    assert rel > 1e-6


def test_ordering_invariance():
    m = W.laplacian((12, 10), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=7)
    a = O.symbolic(m, cap=8, perm="nd")
    b = O.symbolic(m, cap=8, perm="natural")
    sa = a.factor_selinv(m.vals)[0]
    sb = b.factor_selinv(m.vals)[0]
    da = H.sel_to_dict(sa, a.sym.colptrL, a.sym.rowindL, a.sym.perm)
    db = H.sel_to_dict(sb, b.sym.colptrL, b.sym.rowindL, b.sym.perm)
    common = set(da) & set(db)
    assert len(common) > m.nnz
    assert max(abs(da[k] - db[k]) for k in common) < 1e-12


def test_pivot_failure_reported():
    m = W.laplacian((6, 6), shift=-10.0)
    osym = O.symbolic(m, cap=8)
    _, _, st, bad, _, _ = osym.factor_selinv(m.vals, require_spd=True)
    assert st == -3 and bad == int(osym.sym.perm[0])


# ---------------------------------------------------------------- gradient reference
def test_dense_gradient_vs_finite_differences():
    m = W.laplacian((4, 4), coeff="uniform", lo=0.5, hi=2.0, shift=0.3, seed=3)
    s = O.symbolic(m, cap=4, perm="natural").sym
    rng = np.random.default_rng(0)
    w = rng.standard_normal(s.nnzL)
    a = m.dense()
    inv = O.dense_inverse(a)
    g = O.dense_grad(inv, s.colptrL, s.rowindL, w, m.colptr, m.rowind)

    def f(mat):
        return float(np.dot(w, H.sel_from_dense(O.dense_inverse(mat), s.colptrL, s.rowindL)))

    cols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    h = 1e-5
    for p in range(m.nnz):
        i, j = int(m.rowind[p]), int(cols[p])
        e = np.zeros_like(a)
        e[i, j] = 1.0
        e[j, i] = 1.0
        fd = (f(a + h * e) - f(a - h * e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(g[p]))


# ---------------------------------------------------------------- planted mistakes
def _pin_suite_fails():
    """True if one of the numeric pins fails under the current mutation."""
    try:
        test_tridiagonal_closed_form(63, 0.3, "nd")
        test_grid_spectral_closed_form((8, 8), 0.0, 128)
        test_grid_spectral_closed_form((5, 4, 3), 0.2, 4)
        test_o3_o2_o1_random(1)
    except (AssertionError, ValueError):
        return True
    return False


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6, 7])
def test_planted_mistakes_are_caught(mutation):
    """1 sign of X, 2 dropped diagonal term, 3 L used for L_hat, 4 upper part
    of the gathered block dropped, 5 Schur update misses its diagonal,
    6 D instead of D^{-1}, 7 children's structures not merged."""
    O.set_mutation(mutation)
    try:
        assert _pin_suite_fails()
    finally:
        O.set_mutation(0)
    assert not _pin_suite_fails()


# ---------------------------------------------------------------- the exported factor (O3's L and D)
def _factor_cases():
    return [
        ("random", W.random_spd_pattern(120, 0.04, 21), 7, "random"),
        ("grid2d", W.laplacian((9, 8), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=3), 16, "nd"),
        ("grid3d", W.laplacian((5, 4, 3), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5), 4, "nd"),
        ("molecular", W.molecular(side=3, dofs=8, seed=2), 32, "nd"),
        ("fig1", W.fig1_pattern(), 6, "natural"),
    ]


def _unpack_factor(Lv, s):
    """Dense unit-lower L and diagonal D from values on the canonical pattern
    (D stored on the diagonal positions)."""
    n = s.n
    cols = np.repeat(np.arange(n), np.diff(s.colptrL))
    Ld = np.zeros((n, n))
    Ld[s.rowindL, cols] = Lv
    d = np.diag(Ld).copy()
    np.fill_diagonal(Ld, 1.0)
    return Ld, d


@pytest.mark.parametrize("name", [c[0] for c in _factor_cases()])
def test_o3_factor_export_reconstructs_A(name):
    """The L and D that O3 exports satisfy P A P^T = L D L^T (the LDL^T form
    of Section 2.1), equal the unique LDL^T of the dense permuted matrix given
    by a library Cholesky (L = C diag(C)^{-1}, D = diag(C)^2), and equal O1's
    dense factor on the pattern of L."""
    _, m, cap, how = next(c for c in _factor_cases() if c[0] == name)
    perm = np.random.default_rng(5).permutation(m.n).astype(np.int32) if how == "random" else how
    osym = O.symbolic(m, cap=cap, perm=perm)
    s = osym.sym
    _, Lv, st, _, _, _ = osym.factor_selinv(m.vals, want_L=True)
    assert st == 0
    Ld, d = _unpack_factor(Lv, s)
    ap = m.dense()[np.ix_(s.perm, s.perm)]
    scale = np.max(np.abs(ap))
    assert np.max(np.abs(Ld @ np.diag(d) @ Ld.T - ap)) <= 1e-13 * scale
    C = np.linalg.cholesky(ap)
    cd = np.diag(C)
    assert np.max(np.abs(Ld - C / cd[None, :])) <= 1e-12
    assert np.max(np.abs(d - cd ** 2) / (cd ** 2)) <= 1e-12
    L1, d1 = O.dense_ldlt(ap)
    assert np.max(np.abs(Ld - L1)) <= 1e-13 and np.max(np.abs(d - d1) / np.abs(d1)) <= 1e-13
    # entries of the dense factor outside the pattern of L are zero (no fill missed)
    outside = np.ones_like(L1, dtype=bool)
    cols = np.repeat(np.arange(m.n), np.diff(s.colptrL))
    outside[s.rowindL, cols] = False
    outside[np.triu_indices(m.n)] = False
    assert np.all(L1[outside] == 0.0)


# ---------------------------------------------------------------- flop and byte counts
# Work per supernode (s columns, c rows below): GEMM phase 2c^2 s + 2cs^2,
# factor c^2 s + cs^2 + s^3/3, whole selected inversion 2c^2 s + 3cs^2 + 2s^3/3,
# gathered bytes 8 c(c+1)/2.  The (s, c) lists below are read off by hand.
#
# Fig. 1 (Section 2.1) under the fundamental partition with a cap of 6: the
# paper's supernodes 9 and 10 merge; C of each supernode is the union of the
# row sets of the off-diagonal blocks in its block column, plus the fill block
# {25, 26, 28} below supernode 8.
FIG1_SC = [(2, 2),   # cols 0-1,   block (2,1): rows 2-3
           (2, 4),   # cols 2-3,   block (5,2): rows 10, 12, 13, 14
           (4, 2),   # cols 4-7,   block (4,3): rows 8-9
           (2, 6),   # cols 8-9,   block (5,4): rows 10-15
           (6, 2),   # cols 10-15, block (9,5): rows 23-24
           (2, 6),   # cols 16-17, blocks (8,6) rows 20-22 and (10,6) rows 25, 26, 28
           (2, 3),   # cols 18-19, block (8,7): rows 20-22
           (3, 5),   # cols 20-22, block (9,8) rows 23-24 and the fill rows 25, 26, 28
           (6, 0)]   # cols 23-28, the root
# totals of the formulas over that list, added up by hand
FIG1_GEMM, FIG1_FACTOR, FIG1_SELINV, FIG1_GATHER = 1100.0, 2213.0 / 3.0, 5125.0 / 3.0, 656.0


def _tridiag_natural_counts(n):
    """Natural order: columns 0..n-3 are single-column supernodes with C = {j+1};
    the last two columns form one supernode with C empty."""
    k = n - 2
    return 4.0 * k, k * 7.0 / 3.0 + 8.0 / 3.0, k * 17.0 / 3.0 + 16.0 / 3.0, 8.0 * k


def test_fig1_partition_matches_hand_list():
    m = W.fig1_pattern()
    s = O.symbolic(m, cap=6, perm="natural").sym
    got = [(int(s.xsuper[k + 1] - s.xsuper[k]), int(s.cptr[k + 1] - s.cptr[k])) for k in range(s.N)]
    assert got == FIG1_SC


def test_flop_counts_fig1_oracle_and_library():
    from paper_1404_0447_amd import selinv as S
    m = W.fig1_pattern()
    s = O.symbolic(m, cap=6, perm="natural").sym
    assert s.gemm_flops == pytest.approx(FIG1_GEMM, rel=1e-14)
    assert s.factor_flops == pytest.approx(FIG1_FACTOR, rel=1e-14)
    inf = S.Plan(m.n, m.colptr, m.rowind, max_super=6).info
    assert inf["flops_gemm"] == pytest.approx(FIG1_GEMM, rel=1e-14)
    assert inf["flops_factor"] == pytest.approx(FIG1_FACTOR, rel=1e-14)
    assert inf["flops_selinv"] == pytest.approx(FIG1_SELINV, rel=1e-14)
    assert inf["gather_bytes"] == pytest.approx(FIG1_GATHER, rel=1e-14)


@pytest.mark.parametrize("n", [3, 50, 257])
def test_flop_counts_tridiagonal_natural(n):
    from paper_1404_0447_amd import selinv as S
    m = W.tridiag_1d(n, 0.1)
    gemm, factor, selinv, gather = _tridiag_natural_counts(n)
    s = O.symbolic(m, cap=8, perm="natural").sym
    assert s.N == n - 1
    assert s.gemm_flops == pytest.approx(gemm, rel=1e-14)
    assert s.factor_flops == pytest.approx(factor, rel=1e-14)
    inf = S.Plan(m.n, m.colptr, m.rowind, max_super=8).info
    assert inf["nsuper"] == n - 1
    assert inf["flops_gemm"] == pytest.approx(gemm, rel=1e-14)
    assert inf["flops_factor"] == pytest.approx(factor, rel=1e-14)
    assert inf["flops_selinv"] == pytest.approx(selinv, rel=1e-14)
    assert inf["gather_bytes"] == pytest.approx(gather, rel=1e-14)


@pytest.mark.parametrize("mutation", [8, 9])
def test_planted_export_mistakes_are_caught(mutation):
    """8 exports L D instead of L below the diagonal, 9 exports D^{-1} instead
    of D; the reconstruction pins above catch both."""
    O.set_mutation(mutation)
    try:
        caught = 0
        for name in [c[0] for c in _factor_cases()]:
            try:
                test_o3_factor_export_reconstructs_A(name)
            except AssertionError:
                caught += 1
        assert caught == len(_factor_cases())
    finally:
        O.set_mutation(0)
    for name in [c[0] for c in _factor_cases()]:
        test_o3_factor_export_reconstructs_A(name)


# ---------------------------------------------------------------- rim-last separators
def test_nd_rim_last_hand_examples():
    # 5 x 5: the top separator is the column x = 2; its interior (y = 1..3)
    # comes before its rim (y = 0 and y = 4)
    assert list(O.nd_order(2, (5, 5), rim_last=True)[-5:]) == [7, 12, 17, 2, 22]
    assert list(O.nd_order(2, (5, 5))[-5:]) == [2, 7, 12, 17, 22]
    # 3 x 3 x 3: the top separator is the plane x = 1; only (y, z) = (1, 1) is interior
    assert list(O.nd_order(3, (3, 3, 3), rim_last=True)[-9:]) == [13, 1, 4, 7, 10, 16, 19, 22, 25]
    # 1D: a separator is one point, nothing to reorder
    assert list(O.nd_order(1, (7,), rim_last=True)) == list(O.nd_order(1, (7,)))


@pytest.mark.parametrize("dims", [(16, 16), (7, 9, 6)])
def test_rim_last_changes_pattern_not_values(dims):
    m = W.laplacian(dims, coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=11)
    a = O.symbolic(m, cap=16, perm="nd")
    b = O.symbolic(m, cap=16, perm="nd_rim")
    assert sorted(b.sym.perm) == list(range(m.n)) and not np.array_equal(a.sym.perm, b.sym.perm)
    sa, sb = a.factor_selinv(m.vals)[0], b.factor_selinv(m.vals)[0]
    da = H.sel_to_dict(sa, a.sym.colptrL, a.sym.rowindL, a.sym.perm)
    db = H.sel_to_dict(sb, b.sym.colptrL, b.sym.rowindL, b.sym.perm)
    common = set(da) & set(db)
    assert len(common) > m.nnz
    assert max(abs(da[k] - db[k]) for k in common) < 1e-12
    exact = np.linalg.inv(m.dense())
    assert H.err_c8(sb, H.sel_from_dense(exact, b.sym.colptrL, b.sym.rowindL, b.sym.perm), b.sym.colptrL,
                    b.sym.rowindL) < 1e-11


# ---------------------------------------------------------------- relaxed supernodes
@pytest.mark.parametrize("case", ["grid2d", "grid3d", "molecular", "random"])
def test_relaxed_values_are_the_inverse_on_the_superset_pattern(case):
    """With relaxed supernodes the pattern grows by explicit zeros of L; the
    selected values there are still entries of A^{-1} (checked against the
    dense inverse by a library routine), the exported L is exactly zero
    there, and on the fundamental pattern the values agree with the
    unrelaxed run."""
    if case == "grid2d":
        m, cap, rc, perm = W.laplacian((14, 12), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=3), 128, 128, "nd"
    elif case == "grid3d":
        m, cap, rc, perm = W.laplacian((7, 6, 5), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5), 16, 8, "nd"
    elif case == "molecular":
        m, cap, rc, perm = W.molecular(side=4, dofs=8, seed=2), 64, 64, "nd"
    else:
        m, cap, rc, perm = W.random_spd_pattern(120, 0.04, 4), 8, 8, "natural"
    r = O.symbolic(m, cap=cap, perm=perm, relax=rc)
    f = O.symbolic(m, cap=cap, perm=perm)
    assert r.sym.nnzL > f.sym.nnzL  # there are explicit zeros
    sel, Lv, st, _, _, _ = r.factor_selinv(m.vals, want_L=True)
    assert st == 0
    s = r.sym
    exact = np.linalg.inv(m.dense())
    assert H.err_c8(sel, H.sel_from_dense(exact, s.colptrL, s.rowindL, s.perm), s.colptrL, s.rowindL) < 1e-11
    # L: zero wherever the fundamental pattern has no entry
    n = m.n
    fkeys = set(zip(np.repeat(np.arange(n), np.diff(f.sym.colptrL)).tolist(), f.sym.rowindL.tolist()))
    cols = np.repeat(np.arange(n), np.diff(s.colptrL))
    extra = np.array([(int(c), int(i)) not in fkeys for c, i in zip(cols, s.rowindL)])
    assert extra.any() and np.all(Lv[extra] == 0.0)
    fsel = f.factor_selinv(m.vals)[0]
    dr = H.sel_to_dict(sel, s.colptrL, s.rowindL, s.perm)
    df = H.sel_to_dict(fsel, f.sym.colptrL, f.sym.rowindL, f.sym.perm)
    assert max(abs(dr[k] - df[k]) for k in df) < 1e-12


def test_relaxed_partition_hand_example():
    """Natural-order tridiagonal of 10 columns: fundamental supernodes are the
    single columns 0..7 and {8, 9}; each column's only child is the one
    before it, so relaxing with at most 4 columns gives [0,4), [4,8), [8,10),
    and the blocks' rows below them are {4}, {8} and none."""
    m = W.tridiag_1d(10, 0.1)
    s = O.symbolic(m, cap=8, perm="natural", relax=4).sym
    assert list(s.xsuper) == [0, 4, 8, 10]
    assert [list(s.crows[s.cptr[k]:s.cptr[k + 1]]) for k in range(s.N)] == [[4], [8], []]
    assert s.nnzL == (10 + 4) + (10 + 4) + 3


# ---------------------------------------------------------------- complex symmetric A(z) = H - z S
def _complex_cases():
    H, S = W.hamiltonian_overlap(side=3, dofs=8, seed=6)
    z = W.poles(4, 0.0, 30.0)
    m = W.random_spd_pattern(90, 0.05, 13)
    on_diag = m.rowind == np.repeat(np.arange(m.n), np.diff(m.colptr))
    return {
        "pencil_pole0": (H, W.pencil_values(H, S, z[0]), 32),
        "pencil_pole3": (H, W.pencil_values(H, S, z[3]), 16),
        "random_shifted": (m, m.vals - (1.5 + 0.7j) * on_diag, 8),
    }


def _dense_complex(m, vals):
    a = np.zeros((m.n, m.n), dtype=np.complex128)
    cols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    a[m.rowind, cols] = vals
    a[cols, m.rowind] = vals
    return a


@pytest.mark.parametrize("name", ["pencil_pole0", "pencil_pole3", "random_shifted"])
def test_complex_tiers_against_library_inverse(name):
    """O1 and O3 for a complex symmetric matrix against a library inverse
    (numpy's LU, no symmetry used), restricted to the pattern; symmetric, not
    Hermitian, so a conjugate anywhere would fail; row identity."""
    m, vals, cap = _complex_cases()[name]
    a = _dense_complex(m, vals)
    exact = np.linalg.inv(a)
    assert np.max(np.abs(O.dense_inverse_complex(a) - exact)) <= 1e-12 * np.max(np.abs(exact))
    osym = O.symbolic(m, cap=cap, perm="nd" if m.ndim > 0 else "natural")
    s = osym.sym
    sel, st, _ = osym.factor_selinv_complex(vals)
    assert st == 0
    cols = np.repeat(np.arange(m.n), np.diff(s.colptrL))
    ref = exact[s.perm[s.rowindL], s.perm[cols]]
    d = np.abs(ref[s.colptrL[:-1]])
    scale = np.sqrt(d[s.rowindL] * d[cols])
    assert np.max(np.abs(sel - ref) / scale) <= 1e-11
    # sum_j A_ij Ainv_ji = 1 using selected entries only
    full = {}
    for q, (i, j) in enumerate(zip(s.perm[s.rowindL], s.perm[cols])):
        full[(i, j)] = full[(j, i)] = sel[q]
    r = np.zeros(m.n, dtype=np.complex128)
    acols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    for i, j, v in zip(m.rowind, acols, vals):
        r[i] += v * full[(j, i)]
        if i != j:
            r[j] += v * full[(i, j)]
    assert np.max(np.abs(r - 1.0)) <= 1e-10


@pytest.mark.parametrize("n,z", [(40, 0.3 + 0.5j), (61, -1.0 + 0.2j), (25, 3.0 - 2.0j)])
def test_complex_tridiagonal_closed_form(n, z):
    """tridiag(-1, 2 - z, -1): (A^{-1})_ij = sinh(i t) sinh((n+1-j) t) / (sinh t sinh((n+1) t))
    for i <= j (1-based), cosh t = 1 - z/2, with complex t."""
    import cmath
    m = W.tridiag_1d(n, 0.0)
    vals = m.vals - z * (np.repeat(np.arange(n), np.diff(m.colptr)) == m.rowind)
    osym = O.symbolic(m, cap=4, perm="nd")
    s = osym.sym
    sel, st, _ = osym.factor_selinv_complex(vals)
    assert st == 0
    t = cmath.acosh(1.0 - z / 2.0)

    def exact(i, j):
        i, j = min(i, j), max(i, j)
        return cmath.sinh(i * t) * cmath.sinh((n + 1 - j) * t) / (cmath.sinh(t) * cmath.sinh((n + 1) * t))
    cols = np.repeat(np.arange(n), np.diff(s.colptrL))
    ref = np.array([exact(int(s.perm[i]) + 1, int(s.perm[j]) + 1) for i, j in zip(s.rowindL, cols)])
    assert np.max(np.abs(sel - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_planted_conjugation_is_caught():
    O.set_mutation(10)
    try:
        with pytest.raises(AssertionError):
            test_complex_tiers_against_library_inverse("pencil_pole0")
    finally:
        O.set_mutation(0)
    test_complex_tiers_against_library_inverse("pencil_pole0")


# ---------------------------------------------------------------- 1x1 / 2x2 pivots (symmetric indefinite)
@pytest.mark.parametrize("side,cap", [(3, 32), (4, 64), (4, 16), (5, 128)])
def test_pivoted_tier_on_indefinite_matrices(side, cap):
    """Zero diagonal entries: the unpivoted LDL^T reports a bad pivot; the
    LDL^T with Bunch-Kaufman 1x1/2x2 pivots inside the diagonal blocks gives
    the selected entries of the inverse (against a library LU inverse), the
    row identity holds, and on an SPD matrix it agrees with the unpivoted
    tier."""
    m = W.indefinite_molecular(side=side, seed=8)
    osym = O.symbolic(m, cap=cap)
    s = osym.sym
    _, _, st, _, _, _ = osym.factor_selinv(m.vals, require_spd=False)
    assert st == -3
    sel, st, _ = osym.factor_selinv_pivoted(m.vals)
    assert st == 0
    exact = np.linalg.inv(m.dense())
    ref = H.sel_from_dense(exact, s.colptrL, s.rowindL, s.perm)
    # indefinite: |Ainv_ij| <= sqrt(Ainv_ii Ainv_jj) does not hold, so the
    # error is taken relative to the largest entry (kappa is 10..1e3 here)
    assert np.max(np.abs(sel - ref)) <= 1e-12 * np.max(np.abs(ref))
    r = H.row_identity_fast(sel, m, s.colptrL, s.rowindL, s.perm)
    assert np.max(np.abs(r)) <= 1e-10


def test_pivoted_tier_equals_unpivoted_on_spd():
    m = W.laplacian((7, 6, 5), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5)
    osym = O.symbolic(m, cap=16)
    a = osym.factor_selinv(m.vals)[0]
    b, st, _ = osym.factor_selinv_pivoted(m.vals)
    assert st == 0
    s = osym.sym
    assert H.err_c8(b, a, s.colptrL, s.rowindL) <= 1e-12


def test_pivoted_tier_needs_2x2_pivots():
    """[[0, 1], [1, 0]] blocks on the diagonal, coupled: no 1x1 pivot exists
    in the first column, a 2x2 pivot does."""
    n = 6
    a = np.zeros((n, n))
    for k in range(0, n, 2):
        a[k, k + 1] = a[k + 1, k] = 1.0
    a[2:4, 0:2] = a[0:2, 2:4] = 0.25  # couple the blocks
    colptr, rowind, vals = _with_diagonal(a)
    m = W.Matrix(n, colptr, rowind, vals)
    osym = O.symbolic(m, cap=8, perm="natural")
    s = osym.sym
    assert osym.factor_selinv(vals, require_spd=False)[2] == -3
    sel, st, _ = osym.factor_selinv_pivoted(vals)
    assert st == 0
    ref = H.sel_from_dense(np.linalg.inv(a), s.colptrL, s.rowindL, s.perm)
    assert np.max(np.abs(sel - ref)) <= 1e-14


def _with_diagonal(a):
    """Lower CSC of a dense symmetric matrix with every diagonal entry stored."""
    n = a.shape[0]
    mask = np.tril(a != 0) | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    colptr = np.zeros(n + 1, np.int64)
    np.add.at(colptr, cols + 1, 1)
    return np.cumsum(colptr), rows.astype(np.int32), a[rows, cols]


def test_planted_missing_2x2_pivots_are_caught():
    O.set_mutation(11)
    try:
        with pytest.raises(AssertionError):
            test_pivoted_tier_needs_2x2_pivots()
        with pytest.raises(AssertionError):
            test_pivoted_tier_on_indefinite_matrices(4, 64)
    finally:
        O.set_mutation(0)
    test_pivoted_tier_needs_2x2_pivots()
