"""Symmetric indefinite matrices on the GPU: diagonal blocks factored with
1x1/2x2 pivots (Bunch-Kaufman rule) and symmetric interchanges inside the
block, T = F_KK^{-1} handed to the unchanged selected inversion
(Section 2.1: D may hold 2x2 blocks).

Bars: the selected entries against the oracle's pivoted tier and against a
library LU inverse to 1e-10 of the largest entry (indefinite: the
sqrt(Ainv_ii Ainv_jj) scale of the SPD metric does not bound the entries);
saddle-point blocks with no coupling, whose inverse is the matrix itself,
to 1e-14; gradients against the dense formula on a library inverse to
1e-10 of the largest entry."""
import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fwd(p, vals):
    torch = _torch()
    v = torch.as_tensor(vals, dtype=torch.float64, device="cuda")
    p.factor(v)
    sel = p.invert()
    p.sync_status()
    return sel.cpu().numpy()


@pytest.mark.parametrize("side,cap", [(3, 32), (4, 64), (4, 16), (5, 128)])
def test_pivoted_matches_oracle_and_library_inverse(side, cap):
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    from oracle import oracle as O
    m = W.indefinite_molecular(side=side, seed=8)
    print(f"[pivot] side={side} cap={cap} n={m.n}", flush=True)
    p = S.Plan.from_matrix(m, max_super=cap, pivoting=True).bind()
    sel = _fwd(p, m.vals)
    o = O.symbolic(m, cap=cap)
    cp, ri, pm = p.pattern()
    assert np.array_equal(cp, o.sym.colptrL) and np.array_equal(ri, o.sym.rowindL)
    osel, st, _ = o.factor_selinv_pivoted(m.vals)
    assert st == 0
    scale = np.max(np.abs(osel))
    assert np.max(np.abs(sel - osel)) <= 1e-10 * scale
    ref = H.sel_from_dense(np.linalg.inv(m.dense()), cp, ri, pm)
    assert np.max(np.abs(sel - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_unpivoted_path_reports_the_zero_pivot():
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.indefinite_molecular(side=3, seed=8)
    p = S.Plan.from_matrix(m, max_super=64, require_spd=False).bind()
    with pytest.raises(S.SelinvError) as ei:
        _fwd(p, m.vals)
    assert ei.value.status == S.SELINV_EPIVOT


def test_uncoupled_saddle_points_are_their_own_inverse():
    """Coupling 0: A is block diagonal with [[0, I], [I, 0]] per atom, so
    A^{-1} = A; the fill positions of L hold zeros of A^{-1}."""
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.indefinite_molecular(side=4, seed=8, coupling=0.0)
    p = S.Plan.from_matrix(m, max_super=64, pivoting=True).bind()
    sel = _fwd(p, m.vals)
    cp, ri, pm = p.pattern()
    ref = H.sel_from_dense(m.dense(), cp, ri, pm)
    assert np.max(np.abs(sel - ref)) <= 1e-14


def test_singular_block_is_reported():
    """One atom's saddle block zeroed with no coupling: the diagonal block
    that holds it is singular for every choice of pivots."""
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    from oracle import oracle as O
    m = W.indefinite_molecular(side=3, seed=8, coupling=0.0)
    vals = m.vals.copy()
    cols = np.repeat(np.arange(m.n), np.diff(m.colptr))
    vals[cols // 8 == 5] = 0.0
    p = S.Plan.from_matrix(m, max_super=32, pivoting=True).bind()
    with pytest.raises(S.SelinvError) as ei:
        _fwd(p, vals)
    assert ei.value.status == S.SELINV_EPIVOT
    assert O.symbolic(m, cap=32).factor_selinv_pivoted(vals)[1] != 0


def test_pivoted_equals_unpivoted_on_spd():
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((12, 12, 12), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5)
    a = _fwd(S.Plan.from_matrix(m, max_super=128).bind(), m.vals)
    b = _fwd(S.Plan.from_matrix(m, max_super=128, pivoting=True).bind(), m.vals)
    cp, ri, _ = S.Plan.from_matrix(m, max_super=128).pattern()
    assert H.err_c8(b, a, cp, ri) <= 1e-12


def test_pivoted_gradient_matches_dense_formula():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    from oracle import oracle as O
    m = W.indefinite_molecular(side=4, seed=8)
    p = S.Plan.from_matrix(m, max_super=64, pivoting=True).bind()
    _fwd(p, m.vals)
    w = np.random.default_rng(7).standard_normal(int(p.info["nnzL"]))
    g = p.backward(torch.as_tensor(w, device="cuda")).cpu().numpy()
    cp, ri, pm = p.pattern()
    cols = np.repeat(np.arange(m.n), np.diff(cp))
    r0, c0 = pm[ri].astype(np.int64), pm[cols].astype(np.int64)
    order = np.lexsort((r0, c0))
    colptrW = np.zeros(m.n + 1, np.int64)
    np.add.at(colptrW, c0[order] + 1, 1)
    colptrW = np.cumsum(colptrW)
    inv = np.linalg.inv(m.dense())
    ref = O.dense_grad(inv, colptrW, r0[order].astype(np.int32), w[order], m.colptr, m.rowind)
    assert np.max(np.abs(g - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_pivoted_plan_refuses_factor_export_and_tuning():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.indefinite_molecular(side=3, seed=8)
    p = S.Plan.from_matrix(m, max_super=32, pivoting=True).bind()
    _fwd(p, m.vals)
    with pytest.raises(S.SelinvError) as ei:
        p.factor_values()
    assert ei.value.status == S.SELINV_EUNSUPPORTED
    v = torch.as_tensor(m.vals, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SelinvError) as ei:
        p.tune(v)
    assert ei.value.status == S.SELINV_EUNSUPPORTED


def test_pivoted_run_and_graph_match_factor_invert():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.indefinite_molecular(side=4, seed=8)
    p = S.Plan.from_matrix(m, max_super=64, pivoting=True).bind()
    ref = _fwd(p, m.vals)
    v = torch.as_tensor(m.vals, dtype=torch.float64, device="cuda")
    out = p.run(v)
    p.sync_status()
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


def _dense_block(s, seed, zero_diag=False):
    """One dense symmetric indefinite s x s block (a single supernode in
    natural order): N(0,1) entries, a + a^T; zero_diag empties the diagonal
    so that every pivot step has to look past the candidate's diagonal."""
    from paper_1404_0447_amd import workloads as W
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((s, s))
    a = a + a.T
    if zero_diag:
        np.fill_diagonal(a, 0.0)
    rows, cols = np.tril_indices(s)
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    cp = np.zeros(s + 1, np.int64)
    np.add.at(cp, cols + 1, 1)
    return W.Matrix(s, np.cumsum(cp), rows.astype(np.int32), a[rows, cols])


@pytest.mark.parametrize("s,zero_diag", [(2, True), (7, False), (16, True), (33, False), (64, True), (100, False),
                                         (128, False), (128, True)])
def test_dense_indefinite_block_matches_library_inverse(s, zero_diag):
    """Every width class of the pivoted diagonal kernel (s <= 32, 64, 128),
    ragged widths, and zero diagonals (no 1x1 pivot on the first candidate
    is possible): the block's inverse against a library LU inverse and the
    oracle's pivoted tier, to 1e-10 of the largest entry."""
    from paper_1404_0447_amd import selinv as S
    from oracle import oracle as O
    m = _dense_block(s, 100 + s, zero_diag)
    print(f"[pivot] dense s={s} zero_diag={zero_diag}", flush=True)
    p = S.Plan(m.n, m.colptr, m.rowind, perm=np.arange(s), max_super=128, pivoting=True).bind()
    sel = _fwd(p, m.vals)
    cp, ri, pm = p.pattern()
    ref = H.sel_from_dense(np.linalg.inv(m.dense()), cp, ri, pm)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(sel - ref)) <= 1e-10 * scale
    o = O.symbolic(m, cap=128, perm="natural")
    assert np.array_equal(cp, o.sym.colptrL) and np.array_equal(ri, o.sym.rowindL)
    osel, st, _ = o.factor_selinv_pivoted(m.vals)
    assert st == 0
    assert np.max(np.abs(sel - osel)) <= 1e-10 * scale


def test_pivoted_full_size_against_oracle_and_sparse_lu():
    """The indefinite workload the benchmark times, at full size (saddle-point
    blocks on a jittered 16^3-atom lattice x 8, n = 32768, cap 128).  This
    matrix has a 1-norm condition number of about 4.4e6, and with pivots
    restricted to the diagonal blocks the oracle itself differs from an
    independent sparse LU solve by up to about 1.5e-8 of the largest entry,
    so the 1e-10 bar of the smaller cases (where the oracle matches a library
    LU inverse) cannot hold here for any FP64 method.  The bar instead: on
    the six columns where the GPU and the oracle differ most and on ten
    random columns, the GPU's selected entries lie within 5x the oracle's own
    distance from the sparse LU's column (floor 1e-9 of the largest entry);
    over all entries, GPU and oracle agree to 1e-6 of the largest entry."""
    _torch()
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    from oracle import oracle as O
    m = W.indefinite_molecular(side=16, dofs=8, seed=8)
    n = m.n
    print(f"[pivot] full size n={n}", flush=True)
    p = S.Plan.from_matrix(m, max_super=128, pivoting=True).bind()
    sel = _fwd(p, m.vals)
    cp, ri, pm = p.pattern()
    del p
    o = O.symbolic(m, cap=128)
    assert np.array_equal(cp, o.sym.colptrL) and np.array_equal(ri, o.sym.rowindL)
    osel, st, _ = o.factor_selinv_pivoted(m.vals)
    assert st == 0
    scale = np.max(np.abs(osel))
    d = np.abs(sel - osel)
    assert np.max(d) <= 1e-6 * scale
    cols = np.repeat(np.arange(n), np.diff(m.colptr))
    A = sp.csc_matrix((m.vals, (m.rowind, cols)), shape=(n, n))
    lu = sla.splu(sp.csc_matrix(A + sp.tril(A, -1).T))
    worst = np.argsort(np.maximum.reduceat(d, cp[:-1]))[::-1][:6]
    rand = np.random.default_rng(0).choice(n, 10, replace=False)
    for j in list(worst) + list(rand):
        e = np.zeros(n)
        e[pm[j]] = 1.0
        ref = lu.solve(e)[pm[ri[cp[j]:cp[j + 1]]]]
        g = np.max(np.abs(sel[cp[j]:cp[j + 1]] - ref))
        od = np.max(np.abs(osel[cp[j]:cp[j + 1]] - ref))
        assert g <= 5 * max(od, 1e-9 * scale), f"column {j}: GPU {g / scale:.2e}, oracle {od / scale:.2e} from LU"
