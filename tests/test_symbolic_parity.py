"""Host side of the library (no GPU needed): the library loads and exports
every declared symbol, its symbolic analysis equals the oracle's bit for bit,
and malformed inputs are rejected with a status code."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_0447_amd import selinv as S
from paper_1404_0447_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "selinv.h")).read()
    declared = set(re.findall(r"\b(selinv_[a-z_]+)\s*\(", hdr))
    assert declared == set(S.EXPORTS)
    L = ct.CDLL(S.LIB)
    for name in declared:
        assert hasattr(L, name), name


def _compare(m, cap, perm="nd", fuse=True):
    o = O.symbolic(m, cap=cap, perm=perm).sym
    if isinstance(perm, str):
        p = S.Plan.from_matrix(m, max_super=cap, fuse_chains=fuse) if perm == "nd" else \
            S.Plan(m.n, m.colptr, m.rowind, max_super=cap, fuse_chains=fuse)
    else:
        p = S.Plan(m.n, m.colptr, m.rowind, perm=perm, max_super=cap, fuse_chains=fuse)
    cp, ri, pm = p.pattern()
    sy = p.symbolic()
    assert np.array_equal(pm, o.perm)
    assert np.array_equal(cp, o.colptrL) and np.array_equal(ri, o.rowindL)
    assert np.array_equal(sy["parent"], o.parent)
    assert np.array_equal(sy["xsuper"], o.xsuper)
    assert np.array_equal(sy["sparent"], o.sparent)
    assert np.array_equal(sy["level"], o.level)
    assert np.array_equal(sy["cptr"], o.cptr) and np.array_equal(sy["crows"], o.crows)
    assert np.array_equal(sy["rptr"], o.rptr) and np.array_equal(sy["rel"], o.rel)
    inf = p.info
    assert inf["nnzL"] == o.nnzL and inf["nsuper"] == o.N and inf["depth"] == o.level.max()
    assert inf["flops_gemm"] == pytest.approx(o.gemm_flops, rel=1e-12)
    return p, o


def test_fig1_parity():
    _compare(W.fig1_pattern(), 6, perm="natural")


@pytest.mark.parametrize("dims,cap", [((32, 32), 128), ((7, 5), 3), ((9, 8, 7), 16), ((12, 12, 12), 128),
                                      ((1,), 4), ((50,), 8)])
def test_grid_parity(dims, cap):
    _compare(W.laplacian(dims, shift=0.1), cap)


@pytest.mark.parametrize("seed", range(5))
def test_random_pattern_parity(seed):
    m = W.random_spd_pattern(80, 0.05, seed)
    perm = np.random.default_rng(seed).permutation(m.n).astype(np.int32)
    _compare(m, 2 + 3 * seed, perm=perm)


def test_molecular_parity():
    _compare(W.molecular(side=4, dofs=8, seed=4, shift=30.0), 128)


@pytest.mark.slow
def test_lap3d_40_parity():
    p, o = _compare(W.make("lap3d_40"), 128)
    assert o.N == 42178 and o.level.max() == 311 and o.nnzL == 21285841


def test_exec_blocks_reduce_depth():
    m = W.laplacian((16, 16, 16), shift=0.1)
    a = S.Plan.from_matrix(m, fuse_chains=False).info
    b = S.Plan.from_matrix(m, fuse_chains=True).info
    assert a["nblocks"] == a["nsuper"] and a["exec_depth"] == a["depth"]
    assert b["nblocks"] < a["nblocks"] and b["exec_depth"] < a["depth"]
    assert b["exec_flops_gemm"] >= b["flops_gemm"]


def test_malformed_inputs_rejected():
    m = W.laplacian((4, 4))
    bad = m.rowind.copy()
    bad[1], bad[2] = bad[2], bad[1]  # unsorted rows in column 0
    with pytest.raises(S.SelinvError) as e:
        S.Plan(m.n, m.colptr, bad)
    assert e.value.status == S.SELINV_EINVAL
    up = m.rowind.copy()
    up[m.colptr[3]] = 1  # row above the diagonal in column 3
    with pytest.raises(S.SelinvError):
        S.Plan(m.n, m.colptr, up)
    with pytest.raises(S.SelinvError):
        S.Plan(m.n, m.colptr, m.rowind, perm=np.zeros(m.n, np.int32))  # not a permutation
    with pytest.raises(S.SelinvError) as e:
        S.Plan(m.n, m.colptr, m.rowind, geom=(2, (5, 5), 1))  # geometry mismatch
    assert e.value.status == S.SELINV_EINVAL
    with pytest.raises(S.SelinvError) as e:
        S.Plan(m.n, m.colptr, m.rowind, max_super=512)
    assert e.value.status == S.SELINV_EUNSUPPORTED


def test_degenerate_sizes():
    p = S.Plan(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert p.info["nnzL"] == 0 and p.info["nsuper"] == 0
    p = S.Plan(1, np.array([0, 1]), np.array([0], np.int32))
    assert p.info["nnzL"] == 1 and p.info["nsuper"] == 1
    # a matrix with an empty off-diagonal column structure (diagonal only)
    n = 5
    p = S.Plan(n, np.arange(n + 1), np.arange(n, dtype=np.int32))
    assert p.info["nnzL"] == n and p.info["depth"] == 1


def test_device_calls_need_a_workspace():
    m = W.laplacian((4, 4))
    p = S.Plan.from_matrix(m)
    L = S.lib()
    st = L.selinv_invert(p._h, None, None)
    assert st == S.SELINV_ESTATE


def test_real_entry_points_refuse_complex_plans():
    """A complex plan's values and arenas are (re, im) pairs: every real
    entry point, the allocation-free one included, refuses the plan before
    it touches a pointer or the device."""
    m = W.laplacian((4, 4))
    p = S.Plan.from_matrix(m, complex_values=True)
    L = S.lib()
    assert L.selinv_factor_invert_static(p._h, None, None, None, None) == S.SELINV_EINVAL
    assert b"complex" in L.selinv_last_error()
    assert L.selinv_factor(p._h, None, None) == S.SELINV_EINVAL
    assert b"complex" in L.selinv_last_error()


def test_complex_arenas_count_two_doubles_per_entry():
    """A complex plan's arenas hold (re, im) pairs: their sizes are twice
    those of a real plan with the same execution blocks (64 columns at
    most), and the adjoint arenas, which a complex plan lacks, are refused."""
    m = W.laplacian((6, 5, 4), shift=0.1)
    real = S.Plan.from_matrix(m, exec_cap=64)
    cx = S.Plan.from_matrix(m, complex_values=True)
    L = S.lib()
    for which in range(5):
        a, b = ct.c_int64(-1), ct.c_int64(-1)
        assert L.selinv_get_arena(real._h, which, None, ct.byref(a), None) == S.SELINV_OK
        assert L.selinv_get_arena(cx._h, which, None, ct.byref(b), None) == S.SELINV_OK
        assert b.value == 2 * a.value > 0 or (a.value == 0 and b.value == 0)
    for which in (5, 6, 7):
        assert L.selinv_get_arena(cx._h, which, None, None, None) == S.SELINV_EINVAL


@pytest.mark.parametrize("dims,cap", [((16, 16), 128), ((9, 8, 7), 16), ((12, 12, 12), 128)])
def test_rim_last_parity(dims, cap):
    m = W.laplacian(dims, shift=0.1)
    o = O.symbolic(m, cap=cap, perm="nd_rim").sym
    p = S.Plan.from_matrix(m, max_super=cap, sep_order="rim_last")
    cp, ri, pm = p.pattern()
    sy = p.symbolic()
    assert np.array_equal(pm, o.perm)
    assert np.array_equal(cp, o.colptrL) and np.array_equal(ri, o.rowindL)
    for k in ("parent", "xsuper", "sparent", "level", "cptr", "crows", "rptr", "rel"):
        assert np.array_equal(sy[k], getattr(o, k)), k


def test_options_are_validated():
    m = W.laplacian((6, 6), shift=0.1)
    for kw in (dict(sep_order=2), dict(deterministic=2), dict(relaxed=2), dict(relaxed=1, fuse=0)):
        o = S.Opts(128, kw.get("fuse", 1), 1, 0, kw.get("sep_order", 0), kw.get("deterministic", 0), 1,
                   kw.get("relaxed", 0))
        h = ct.c_void_p()
        st = S.lib().selinv_analyze(m.n, m.colptr.ctypes.data_as(ct.c_void_p),
                                    m.rowind.ctypes.data_as(ct.c_void_p), None, None, ct.byref(o), ct.byref(h))
        assert st == S.SELINV_EINVAL


@pytest.mark.parametrize("kw,want", [(dict(pivoting=2, spd=0), "EINVAL"), (dict(pivoting=1, spd=1), "EINVAL"),
                                     (dict(pivoting=1, spd=0, cplx=1), "EUNSUPPORTED")])
def test_pivoting_options_are_validated(kw, want):
    m = W.laplacian((6, 6), shift=0.1)
    o = S._opts(128, 1, kw["spd"], 0, 0, 0, 1, 0, kw.get("cplx", 0), kw["pivoting"])
    o.pivoting = kw["pivoting"]
    h = ct.c_void_p()
    st = S.lib().selinv_analyze(m.n, m.colptr.ctypes.data_as(ct.c_void_p), m.rowind.ctypes.data_as(ct.c_void_p),
                                None, None, ct.byref(o), ct.byref(h))
    assert st == getattr(S, "SELINV_" + want)


def test_pivoting_caps_blocks_and_drops_small_block_kernels():
    """Pivoted diagonal blocks sit whole in LDS (at most 128 columns), and
    the small-block kernels, which factor without pivots, take no block; the
    pattern of L is that of the default plan."""
    m = W.laplacian((9, 8, 7), shift=0.1)
    p = S.Plan.from_matrix(m, max_super=256, pivoting=True)
    q = S.Plan.from_matrix(m, max_super=256)
    assert p.blocks()["s"].max() <= 128
    kw = p.kernel_work()
    assert kw["sbfactor"][0] == 0.0 and kw["sbinvert"][0] == 0.0
    for a, b in zip(p.pattern(), q.pattern()):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_workspace_parts_and_checkpoint_store(k):
    m = W.laplacian((9, 8, 7), shift=0.1)
    p = S.Plan.from_matrix(m, max_super=16, checkpoint_every=k)
    nb = ct.c_size_t()
    assert S.lib().selinv_workspace_size(p._h, ct.byref(nb)) == 0
    assert nb.value == p.persistent_bytes + p.transient_bytes == p.info["workspace_bytes"]
    b = p.blocks()
    slot = ((b["level"] - 1) % k == 0) if k > 1 else np.zeros(len(b["level"]), bool)
    store = int(((b["s"].astype(np.int64) + b["c"]) * b["s"])[slot].sum())
    assert p.kernel_work()["checkpoint"][1] == 16.0 * store
    if k > 1:
        q = S.Plan.from_matrix(m, max_super=16)
        assert p.persistent_bytes >= q.persistent_bytes + 8 * store - 256  # an empty store still takes 256 B
        assert p.transient_bytes == q.transient_bytes


def _compare_relaxed(m, cap, exec_cap=0, perm="nd"):
    ecap = exec_cap if exec_cap > 0 else min(cap, 128)
    o = O.symbolic(m, cap=cap, perm=perm, relax=ecap).sym
    p = S.Plan.from_matrix(m, max_super=cap, exec_cap=exec_cap, relaxed=True) if perm == "nd" else \
        S.Plan(m.n, m.colptr, m.rowind, max_super=cap, exec_cap=exec_cap, relaxed=True)
    cp, ri, pm = p.pattern()
    sy = p.symbolic()
    assert np.array_equal(pm, o.perm)
    assert np.array_equal(cp, o.colptrL) and np.array_equal(ri, o.rowindL)
    for k in ("parent", "xsuper", "sparent", "level", "cptr", "crows", "rptr", "rel"):
        assert np.array_equal(sy[k], getattr(o, k)), k
    inf = p.info
    assert inf["nnzL"] == o.nnzL and inf["nsuper"] == o.N == inf["nblocks"]
    assert inf["flops_gemm"] == pytest.approx(o.gemm_flops, rel=1e-12)
    # the relaxed pattern contains the fundamental one
    f = O.symbolic(m, cap=cap, perm=perm).sym
    n = m.n
    fset = set(zip(np.repeat(np.arange(n), np.diff(f.colptrL)).tolist(), f.rowindL.tolist()))
    rset = set(zip(np.repeat(np.arange(n), np.diff(cp)).tolist(), ri.tolist()))
    assert fset <= rset and o.nnzL >= f.nnzL and o.N <= f.N
    return p, o


@pytest.mark.parametrize("dims,cap,exec_cap", [((16, 16), 128, 0), ((9, 8, 7), 16, 0), ((12, 12, 12), 128, 32),
                                               ((10, 10, 10), 256, 0), ((30,), 8, 0)])
def test_relaxed_parity(dims, cap, exec_cap):
    _compare_relaxed(W.laplacian(dims, shift=0.1), cap, exec_cap)


def test_relaxed_parity_molecular_and_random():
    _compare_relaxed(W.molecular(side=4, dofs=8, seed=4), 128)
    _compare_relaxed(W.random_spd_pattern(150, 0.03, 9), 8, perm="natural")


def test_complex_plans_on_the_host():
    """Complex plans: blocks of at most 64 columns, the pattern of the real
    plan, complex-sized arenas; a pole plan is count copies of one analysis."""
    m = W.laplacian((12, 12, 12), shift=0.1)
    r = S.Plan.from_matrix(m)
    z = S.Plan.from_matrix(m, complex_values=True)
    assert z.blocks()["s"].max() <= 64
    assert np.array_equal(r.pattern()[0], z.pattern()[0]) and np.array_equal(r.pattern()[1], z.pattern()[1])
    zo = O.symbolic(m, cap=128, relax=64).sym
    zb = z.blocks()
    assert np.array_equal(np.concatenate([zb["first"], [m.n]]), zo.xsuper)
    p = S.Plan.poles(m, 5)
    assert p.count == 5 and p.info["n"] == 5 * m.n and p.info["nnzL"] == 5 * z.info["nnzL"]
    assert np.array_equal(np.diff(p.nnzA_off), np.full(5, m.nnz))
