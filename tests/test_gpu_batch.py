"""Persistent work-queue path and batched form on the GPU, through the C ABI.

Every result is compared with the CPU oracle (matrix by matrix for a batch)
at the 1e-10 bar of the single-matrix tests; the persistent path and the
per-level path of the same plan agree to rounding (the order of FP64
atomic additions differs); graph replays agree with direct runs and follow
new values written into the same buffer."""
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


def _oracle_sel(m, cap=128):
    from oracle import oracle as O
    o = O.symbolic(m, cap=cap)
    sel, _, st, _, _, _ = o.factor_selinv(m.vals)
    assert st == 0
    return o.sym, sel


def _vals(ms):
    torch = _torch()
    return torch.as_tensor(np.concatenate([m.vals for m in ms]), dtype=torch.float64, device="cuda")


def _check_batch(p, ms, sel, cap=128):
    cp, ri, _ = p.pattern()
    sel = sel.cpu().numpy()
    worst = 0.0
    for k, m in enumerate(ms):
        s, osel = _oracle_sel(m, cap)
        n0, n1 = p.n_off[k], p.n_off[k + 1]
        l0, l1 = p.nnzL_off[k], p.nnzL_off[k + 1]
        assert np.array_equal(cp[n0:n1 + 1] - l0, s.colptrL) and np.array_equal(ri[l0:l1] - n0, s.rowindL)
        e = H.err_c8(sel[l0:l1], osel, s.colptrL, s.rowindL)
        worst = max(worst, e)
    assert worst <= TOL, f"batched selected inverse error {worst:.3e}"


def _batch():
    from paper_1404_0447_amd import workloads as W
    ms = W.batch_2d(count=9, side_lo=12, side_hi=40, seed=5)
    ms.append(W.laplacian((9, 8, 7), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=6))
    ms.append(W.molecular(side=4, dofs=8, seed=4))
    ms.append(W.tridiag_1d(50, shift=0.2))
    return ms


@pytest.mark.parametrize("case", ["lap2d_32", "lap3d_12_pieces", "molecular_4", "random"])
def test_persistent_single_matrix(case):
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    kw = {}
    if case == "lap2d_32":
        m = W.make("lap2d_32")
    elif case == "lap3d_12_pieces":
        m = W.laplacian((12, 12, 12), coeff="uniform", lo=0.5, hi=2.0, shift=0.01, seed=2)
        kw = dict(max_super=256, exec_cap=16)
    elif case == "molecular_4":
        m = W.molecular(side=4, dofs=8, seed=4)
    else:
        m = W.random_spd_pattern(300, 0.03, 11)
    p = S.Plan.from_matrix(m, **kw).bind()
    v = torch.as_tensor(m.vals, device="cuda")
    print(f"persistent single {case} n={m.n}", flush=True)
    sel = p.run(v)
    p.sync_status()
    s, osel = _oracle_sel(m, kw.get("max_super", 128))
    cp, ri, _ = p.pattern()
    assert H.err_c8(sel.cpu().numpy(), osel, cp, ri) <= TOL
    # same plan, per-level kernels: equal up to the order of atomic additions
    p.factor(v)
    ref = p.invert()
    p.sync_status()
    assert H.err_c8(sel.cpu().numpy(), ref.cpu().numpy(), cp, ri) <= 1e-13


@pytest.mark.parametrize("order,bn_cap,fill,grid,small,mb", [(0, 128, 512, 2, 16, 8), (1, 64, 0, 1, 0, 0),
                                                              (2, 32, 4096, 4, 4, 64), (3, 16, 512, 2, 1, 0),
                                                              (1, 128, 4096, 1, 16, 4096), (0, 64, 512, 2, 0, 4096)])
def test_batch_every_schedule_axis(order, bn_cap, fill, grid, small, mb):
    _torch()
    from paper_1404_0447_amd import selinv as S
    ms = _batch()
    p = S.Plan.batch(ms).bind()
    p.set_schedule(order=order, bn_cap=bn_cap, split_fill=fill, grid_mult=grid, small_s=small, mb_tiles=mb)
    print(f"batch schedule {order} {bn_cap} {fill} {grid} {small} {mb}", flush=True)
    sel = p.run(_vals(ms))
    p.sync_status()
    _check_batch(p, ms, sel)


def test_batch_per_level_path():
    _torch()
    from paper_1404_0447_amd import selinv as S
    ms = _batch()
    p = S.Plan.batch(ms).bind()
    p.factor(_vals(ms))
    sel = p.invert()
    p.sync_status()
    _check_batch(p, ms, sel)


def test_graph_replay_follows_buffer_contents():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    ms = _batch()
    p = S.Plan.batch(ms).bind()
    v = _vals(ms)
    out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device="cuda")
    direct = p.run(v).clone()
    p.sync_status()
    cp, ri, _ = p.pattern()
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for r in range(4):
        print(f"graph replay {r}", flush=True)
        out.fill_(float("nan"))
        p.run(v, out=out, graph=True)
        junk = junk * 1.0001 + 1.0  # eager work between replays
        torch.cuda.synchronize()
        p.sync_status()
        assert H.err_c8(out.cpu().numpy(), direct.cpu().numpy(), cp, ri) <= 1e-13
    # new values in the same buffer: the replay must use them
    ms2 = [W.laplacian((int(round(np.sqrt(m.n))),) * 2, shift=0.7) if m.ndim == 2 else m for m in ms]
    v.copy_(_vals(ms2))
    p.run(v, out=out, graph=True)
    p.sync_status()
    _check_batch(p, ms2, out)


def test_tuner_and_cache(tmp_path):
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    ms = _batch()
    p = S.Plan.batch(ms).bind()
    v = _vals(ms)
    cache = tmp_path / "tune.json"
    sc, ms_best, sel = p.tune(v, cache_path=str(cache))
    p.sync_status()
    assert ms_best > 0 and p.schedule() == sc
    _check_batch(p, ms, sel)
    text = cache.read_text()
    assert text.strip().startswith("{") and "selinv/" in text and '"bn_cap"' in text
    # a fresh plan of the same structure takes the cached choice
    q = S.Plan.batch(ms).bind()
    q.set_schedule(order=0, bn_cap=16, split_fill=0, grid_mult=1, small_s=0, mb_tiles=0)
    sc2, ms2, sel2 = q.tune(v, cache_path=str(cache))
    assert sc2 == sc and ms2 == pytest.approx(ms_best, rel=1e-5)
    q.run(v, out=sel2)
    q.sync_status()
    _check_batch(q, ms, sel2)
    torch.cuda.synchronize()


def test_queue_wait_limit_reports_error():
    """A poll limit of 0 makes every dependency wait give up at once: the
    kernels still finish and the error is reported; the limit restored, the
    same plan computes correct results again."""
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    ms = _batch()[:4]
    p = S.Plan.batch(ms).bind()
    # every block as dependent tile tasks, so that tasks do wait
    p.set_schedule(small_s=0, mb_tiles=0)
    v = _vals(ms)
    p.set_spin_limit(0)
    p.run(v)
    torch.cuda.synchronize()
    with pytest.raises(S.SelinvError) as e:
        p.sync_status()
    assert e.value.status == S.SELINV_EQUEUE
    p.set_spin_limit(1 << 22)
    sel = p.run(v)
    p.sync_status()
    _check_batch(p, ms, sel)


def test_batched_pivot_failure_names_column():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    ms = _batch()[:3]
    p = S.Plan.batch(ms).bind()
    vals = np.concatenate([m.vals for m in ms])
    # zero the diagonal entry of original column 5 of matrix 1
    m1 = ms[1]
    j = 5
    vals[p.nnzA_off[1] + m1.colptr[j]] = -1.0
    p.run(torch.as_tensor(vals, device="cuda"))
    with pytest.raises(S.SelinvError) as e:
        p.sync_status()
    assert e.value.status == S.SELINV_EPIVOT
    assert p.n_off[1] <= e.value.bad_col < p.n_off[2]


@pytest.mark.slow
def test_full_batch_256_grids():
    """The 256-grid batch (sides 32..96, seed 3) in the launch configuration
    the benchmark times (tuned schedule, graph replay): 24 sampled matrices
    entry by entry against the oracle, and the row identity
    sum_j A_ij Ainv_ji = 1 on every matrix."""
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    ms = W.batch_2d()
    p = S.Plan.batch(ms).bind()
    v = _vals(ms)
    p.tune(v)
    sel = p.run(v, graph=True)
    sel = p.run(v, out=sel, graph=True)
    p.sync_status()
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.choice(len(ms), 22, replace=False).tolist())
                    | {int(np.argmax([m.n for m in ms])), int(np.argmin([m.n for m in ms]))})
    host = sel.cpu().numpy()
    cp, ri, pm = p.pattern()
    worst = 0.0
    for k in sample:
        s, osel = _oracle_sel(ms[k])
        l0, l1 = p.nnzL_off[k], p.nnzL_off[k + 1]
        worst = max(worst, H.err_c8(host[l0:l1], osel, s.colptrL, s.rowindL))
    assert worst <= TOL, f"sampled error {worst:.3e}"
    for k, m in enumerate(ms):
        n0, n1 = p.n_off[k], p.n_off[k + 1]
        l0, l1 = p.nnzL_off[k], p.nnzL_off[k + 1]
        r = H.row_identity_fast(host[l0:l1], m, cp[n0:n1 + 1] - l0, ri[l0:l1] - n0, pm[n0:n1] - n0)
        assert np.max(np.abs(r)) <= 1e-10, f"row identity, matrix {k}"
