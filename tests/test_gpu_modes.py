"""Options of the C ABI on the GPU: the deterministic mode, checkpointing of
the inverse panels for the adjoint, the transient memory, the generation
guard of the autograd node and the rim-last separator order.

Bars: results against the CPU oracle at 1e-10 (the metric of the single-
matrix parity tests); the deterministic mode bitwise (run to run, graph
replay against direct launches, a batch against its matrices run alone);
gradients with checkpointing against gradients without it to 1e-12 of the
largest entry (the recomputed panels differ from the stored ones only by
the order of floating-point additions)."""
import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle(m, cap=128, perm="nd"):
    from oracle import oracle as O
    o = O.symbolic(m, cap=cap, perm=perm)
    sel, _, st, _, _, _ = o.factor_selinv(m.vals)
    assert st == 0
    return o.sym, sel


def _fwd(p, vals):
    torch = _torch()
    v = torch.as_tensor(vals, dtype=torch.float64, device="cuda")
    p.factor(v)
    sel = p.invert()
    p.sync_status()
    return sel


def _cases():
    from paper_1404_0447_amd import workloads as W
    return {
        "lap2d_24": (W.laplacian((24, 24), coeff="uniform", lo=0.5, hi=2.0, shift=0.1, seed=1), 128),
        "lap3d_12": (W.laplacian((12, 12, 12), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5), 128),
        "molecular_4": (W.molecular(side=4, dofs=8, seed=4), 128),
        "lap3d_14_wide": (W.laplacian((14, 14, 14), coeff="uniform", lo=0.5, hi=2.0, shift=1e-2, seed=2), 256),
    }


# ------------------------------------------------------------------ deterministic mode
@pytest.mark.parametrize("name", ["lap2d_24", "lap3d_12", "molecular_4", "lap3d_14_wide"])
def test_deterministic_matches_oracle_and_is_bitwise_repeatable(name):
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()[name]
    print(f"[det] {name} n={m.n}", flush=True)
    p = S.Plan.from_matrix(m, max_super=cap, deterministic=True).bind()
    a = _fwd(p, m.vals).cpu().numpy()
    b = _fwd(p, m.vals).cpu().numpy()
    assert np.array_equal(a, b)
    s, osel = _oracle(m, cap)
    cp, ri, _ = p.pattern()
    assert np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
    assert H.err_c8(a, osel, cp, ri) <= TOL
    # the small-block kernels (whose Schur updates use atomics) are off
    kw = p.kernel_work()
    assert kw["sbfactor"][0] == 0.0 and kw["sbinvert"][0] == 0.0


def test_deterministic_run_graph_and_direct_bitwise():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()["lap3d_12"]
    p = S.Plan.from_matrix(m, max_super=cap, deterministic=True).bind()
    v = torch.as_tensor(m.vals, dtype=torch.float64, device="cuda")
    ref = _fwd(p, m.vals).cpu().numpy()
    direct = p.run(v).cpu().numpy()
    out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device="cuda")
    for rep in range(3):
        out.fill_(0.0)  # eager work between replays
        p.run(v, out=out, graph=True)
        p.sync_status()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
    assert np.array_equal(direct, ref)
    with pytest.raises(S.SelinvError) as e:
        p.tune(v)
    assert e.value.status == S.SELINV_EUNSUPPORTED


def test_deterministic_batch_equals_matrices_alone_bitwise():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    ms = W.batch_2d(count=6, side_lo=10, side_hi=30, seed=8)
    ms.append(W.laplacian((7, 6, 5), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=6))
    ms.append(W.molecular(side=3, dofs=8, seed=2))
    pb = S.Plan.batch(ms, deterministic=True).bind()
    vals = torch.as_tensor(np.concatenate([m.vals for m in ms]), dtype=torch.float64, device="cuda")
    pb.factor(vals)
    sel = pb.invert()
    pb.sync_status()
    parts = [x.cpu().numpy() for x in pb.split(sel)]
    for k, m in enumerate(ms):
        q = S.Plan.from_matrix(m, deterministic=True).bind()
        alone = _fwd(q, m.vals).cpu().numpy()
        assert np.array_equal(parts[k], alone), f"matrix {k}"


def test_deterministic_backward_bitwise_and_dense_reference():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from tests.test_gpu_backward import _dense_reference
    m, cap = _cases()["lap3d_12"]
    p = S.Plan.from_matrix(m, max_super=cap, deterministic=True).bind()
    _fwd(p, m.vals)
    w = np.random.default_rng(0).standard_normal(int(p.info["nnzL"]))
    wt = torch.as_tensor(w, device="cuda")
    g1 = p.backward(wt).cpu().numpy()
    g2 = p.backward(wt).cpu().numpy()
    assert np.array_equal(g1, g2)
    ref = _dense_reference(m, p, w)
    assert np.abs(g1 - ref).max() <= 1e-10 * np.abs(ref).max()


# ------------------------------------------------------------------ checkpointing
@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("name", ["lap3d_12", "molecular_4"])
def test_checkpointed_gradient_equals_full(name, k):
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()[name]
    print(f"[ckpt] {name} k={k}", flush=True)
    w = None
    grads = {}
    for every in (1, k):
        p = S.Plan.from_matrix(m, max_super=cap, checkpoint_every=every).bind()
        if w is None:
            w = torch.as_tensor(np.random.default_rng(3).standard_normal(int(p.info["nnzL"])), device="cuda")
        v = torch.as_tensor(m.vals, device="cuda").requires_grad_(True)
        sel = S.selinv(v, p)
        if every > 1:
            assert p._tr is None  # transient memory released between forward and backward
        (g,) = torch.autograd.grad((sel * w).sum(), v)
        grads[every] = g.cpu().numpy()
        if every > 1:
            assert p.kernel_work()["checkpoint"][1] > 0
    g1, gk = grads[1], grads[k]
    assert np.abs(gk - g1).max() <= 1e-12 * np.abs(g1).max()


def test_checkpointed_deterministic_gradient_is_bitwise_full():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()["lap2d_24"]
    grads = []
    for every in (1, 3):
        p = S.Plan.from_matrix(m, max_super=cap, checkpoint_every=every, deterministic=True).bind()
        _fwd(p, m.vals)
        if every > 1:
            p.release_transient()
        w = torch.as_tensor(np.random.default_rng(1).standard_normal(int(p.info["nnzL"])), device="cuda")
        grads.append(p.backward(w).cpu().numpy())
    assert np.array_equal(grads[0], grads[1])


def test_released_transient_without_checkpoints_is_refused():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()["lap2d_24"]
    p = S.Plan.from_matrix(m, max_super=cap).bind()
    _fwd(p, m.vals)
    p.release_transient()
    w = torch.zeros(int(p.info["nnzL"]), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SelinvError) as e:
        p.backward(w)
    assert e.value.status == S.SELINV_ESTATE


# ------------------------------------------------------------------ autograd generation guard
def test_stale_plan_backward_raises():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((10, 10), coeff="uniform", lo=0.5, hi=2.0, shift=0.2, seed=4)
    p = S.Plan.from_matrix(m).bind()
    v1 = torch.as_tensor(m.vals, device="cuda").requires_grad_(True)
    v2 = torch.as_tensor(m.vals * 1.5, device="cuda").requires_grad_(True)
    s1 = S.selinv(v1, p)
    s2 = S.selinv(v2, p)
    with pytest.raises(RuntimeError, match="another factorization"):
        torch.autograd.grad(s1.sum(), v1)
    (g2,) = torch.autograd.grad(s2.sum(), v2)  # the latest forward is still differentiable
    assert torch.isfinite(g2).all()


def test_forward_reports_pivot_failure():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((6, 6), shift=-10.0)
    p = S.Plan.from_matrix(m).bind()
    v = torch.as_tensor(m.vals, device="cuda").requires_grad_(True)
    with pytest.raises(S.SelinvError) as e:
        S.selinv(v, p)
    assert e.value.status == S.SELINV_EPIVOT


# ------------------------------------------------------------------ rim-last separators
@pytest.mark.parametrize("dims", [(20, 20), (11, 10, 9)])
def test_rim_last_matches_oracle(dims):
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian(dims, coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=9)
    p = S.Plan.from_matrix(m, sep_order="rim_last").bind()
    sel = _fwd(p, m.vals).cpu().numpy()
    s, osel = _oracle(m, perm="nd_rim")
    cp, ri, pm = p.pattern()
    assert np.array_equal(pm, s.perm) and np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
    assert H.err_c8(sel, osel, cp, ri) <= TOL


# ------------------------------------------------------------------ relaxed supernodes
@pytest.mark.parametrize("name", ["lap2d_24", "lap3d_12", "molecular_4", "lap3d_14_wide"])
def test_relaxed_matches_oracle(name):
    from paper_1404_0447_amd import selinv as S
    m, cap = _cases()[name]
    ecap = min(cap, 128)
    p = S.Plan.from_matrix(m, max_super=cap, relaxed=True).bind()
    sel = _fwd(p, m.vals).cpu().numpy()
    Lv = p.factor_values().cpu().numpy()
    from oracle import oracle as O
    o = O.symbolic(m, cap=cap, relax=ecap)
    osel, oL, st, _, _, _ = o.factor_selinv(m.vals, want_L=True)
    assert st == 0
    cp, ri, pm = p.pattern()
    assert np.array_equal(cp, o.sym.colptrL) and np.array_equal(ri, o.sym.rowindL) and np.array_equal(pm, o.sym.perm)
    assert H.err_c8(sel, osel, cp, ri) <= TOL
    assert H.err_c8(Lv, oL, cp, ri) <= 1e-12


def test_relaxed_gradient_matches_dense_reference():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from tests.test_gpu_backward import _dense_reference
    m, cap = _cases()["lap3d_12"]
    p = S.Plan.from_matrix(m, max_super=cap, relaxed=True).bind()
    _fwd(p, m.vals)
    w = np.random.default_rng(5).standard_normal(int(p.info["nnzL"]))
    g = p.backward(torch.as_tensor(w, device="cuda")).cpu().numpy()
    ref = _dense_reference(m, p, w)
    assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()
