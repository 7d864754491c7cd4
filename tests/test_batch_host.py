"""Batched form, host side (no GPU): the batch plan is the block-diagonal
union of its matrices, so its symbolic analysis must equal the oracle's
analysis of that union matrix bit for bit; its per-level work queues must
cover every block's work exactly once, in an order in which every task's
dependencies come earlier in the queue (what makes the persistent kernel
drain), for every schedule the autotuner may pick."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_0447_amd import selinv as S
from paper_1404_0447_amd import workloads as W

OP = {name: i for i, name in enumerate(S.QOPS)}


def _small_batch():
    ms = W.batch_2d(count=6, side_lo=5, side_hi=13, seed=3)
    ms.append(W.laplacian((5, 4, 3), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=1))
    ms.append(W.molecular(side=3, dofs=2, seed=4))
    ms.append(W.tridiag_1d(17, shift=0.3))
    return ms


def _union(ms):
    """Block-diagonal matrix of the list, as a workloads.Matrix without geometry."""
    cps, ris, vals = [np.zeros(1, np.int64)], [], []
    n0 = a0 = 0
    for m in ms:
        cps.append(m.colptr[1:] + a0)
        ris.append(m.rowind + n0)
        vals.append(m.vals)
        n0 += m.n
        a0 += m.nnz
    return W.Matrix(n=n0, colptr=np.concatenate(cps), rowind=np.concatenate(ris).astype(np.int32),
                    vals=np.concatenate(vals), ndim=0, dims=(), dofs=1, meta={})


def test_batch_symbolic_equals_oracle_on_union():
    ms = _small_batch()
    p = S.Plan.batch(ms, max_super=8)
    # the oracle's ordering of each matrix, concatenated, is the union's
    offs = np.cumsum([0] + [m.n for m in ms])[:-1]
    perm = np.concatenate([(O.nd_order(m.ndim, m.dims, m.dofs) if m.ndim > 0 else np.arange(m.n)) + off
                           for m, off in zip(ms, offs)])
    o = O.symbolic(_union(ms), cap=8, perm=perm.astype(np.int32)).sym
    cp, ri, pm = p.pattern()
    sy = p.symbolic()
    assert np.array_equal(pm, o.perm)
    assert np.array_equal(cp, o.colptrL) and np.array_equal(ri, o.rowindL)
    for k in ("parent", "xsuper", "sparent", "level", "cptr", "crows", "rptr", "rel"):
        assert np.array_equal(sy[k], getattr(o, k)), k
    assert p.info["nnzL"] == o.nnzL and p.info["nsuper"] == o.N
    assert p.info["flops_gemm"] == pytest.approx(o.gemm_flops, rel=1e-12)


def test_batch_offsets_and_per_matrix_patterns():
    ms = _small_batch()
    p = S.Plan.batch(ms)
    assert p.count == len(ms)
    cp, ri, pm = p.pattern()
    for m, mat in enumerate(ms):
        q = S.Plan.from_matrix(mat)
        qcp, qri, qpm = q.pattern()
        n0, n1 = p.n_off[m], p.n_off[m + 1]
        l0, l1 = p.nnzL_off[m], p.nnzL_off[m + 1]
        assert n1 - n0 == mat.n and p.nnzA_off[m + 1] - p.nnzA_off[m] == mat.nnz
        assert np.array_equal(cp[n0:n1 + 1] - l0, qcp)
        assert np.array_equal(ri[l0:l1] - n0, qri)
        assert np.array_equal(pm[n0:n1] - n0, qpm)
    assert p.info["exec_depth"] == max(S.Plan.from_matrix(m).info["exec_depth"] for m in ms)


def test_empty_and_degenerate_batches():
    p = S.Plan.batch([])
    assert p.count == 0 and p.info["n"] == 0 and p.info["nnzL"] == 0
    e = W.Matrix(n=0, colptr=np.zeros(1, np.int64), rowind=np.zeros(0, np.int32), vals=np.zeros(0), ndim=0,
                 dims=(), dofs=1, meta={})
    ms = [W.tridiag_1d(3), e, W.tridiag_1d(1), e]
    p = S.Plan.batch(ms)
    assert list(p.n_off) == [0, 3, 3, 4, 4]
    assert list(p.nnzL_off) == [0, 5, 5, 6, 6]
    check_queues(p)


def test_malformed_matrix_is_named():
    ms = W.batch_2d(count=4, side_lo=4, side_hi=6, seed=1)
    bad = ms[2]
    bad.rowind = bad.rowind.copy()
    bad.rowind[1] = bad.rowind[0]  # rows not strictly increasing
    with pytest.raises(S.SelinvError) as e:
        S.Plan.batch(ms)
    assert e.value.status == S.SELINV_EINVAL and "matrix 2" in str(e.value)


def _block_matrix(p):
    """matrix index of every execution block (blocks are stored matrix by matrix)."""
    first = p.blocks()["first"]
    return np.searchsorted(p.n_off, first, side="right") - 1


def _exclusive(blk, level):
    """Blocks of a level whose row structure C shares no column with another
    block's C in that level (their Schur updates touch no common entry)."""
    lev, c, off, rows = blk["level"], blk["c"], blk["crow_off"], blk["rows"]
    ids = np.nonzero(lev == level)[0]
    cnt = {}
    for B in ids:
        for x in rows[off[B]:off[B] + c[B]]:
            cnt[int(x)] = cnt.get(int(x), 0) + 1
    return {int(B) for B in ids if all(cnt[int(x)] == 1 for x in rows[off[B]:off[B] + c[B]])}


def check_queues(p, sched=None):
    blk = p.blocks()
    lev, s, c = blk["level"], blk["s"], blk["c"]
    sched = sched or p.schedule()
    for l in range(1, int(p.info["exec_depth"]) + 1):
        excl = _exclusive(blk, l)
        qf = p.queue(0, l)
        for row in qf:
            if S.QOPS[row[6] >> 8] in ("schur", "mbfactor"):
                assert bool(row[6] & 4) == (int(row[0]) in excl), "exclusive-update flag"
        for sweep, phases, sb_op, mb_op in ((0, ("ldlt", "panel", "schur"), "sbfactor", "mbfactor"),
                                            (1, ("zero", "gemm", "sdiag"), "sbinvert", "mbinvert")):
            q = p.queue(sweep, l)
            op = q[:, 6] >> 8
            # medium blocks: one whole-block task each, tile width within the cap
            mb = op == OP[mb_op]
            mids = q[mb, 0]
            assert len(set(mids.tolist())) == len(mids)
            assert np.all(q[mb, 7] == 0) and np.all((q[mb, 6] & 3) == 0)
            assert np.all(q[mb, 3] <= sched["bn_cap"])
            for B, w in zip(mids, q[mb, 3]):
                assert not (s[B] <= sched["small_s"] and c[B] <= 256)
                assert ((c[B] + 63) // 64) * ((s[B] + w - 1) // w) <= sched["mb_tiles"]
            q = q[~mb]
            op = op[~mb]
            sb = op == OP[sb_op]
            # small blocks: whole, four to a task, each exactly once, listed first
            ids = q[sb, :4].ravel()
            ids = ids[ids >= 0]
            assert len(set(ids.tolist())) == len(ids)
            assert np.all((s[ids] <= sched["small_s"]) & (c[ids] <= 256))
            assert np.all(q[sb, 7] == 0) and np.all((q[sb, 6] & 3) == 0)
            if sb.any():
                assert np.all(sb[: int(sb.sum())]), "small-block tasks come first"
            t = q[~sb]
            b, i0, j0, bn, kb, ke, fl, need = (t[:, k] for k in range(8))
            top = fl >> 8
            assert not set(b.tolist()) & set(ids.tolist())
            assert not set(mids.tolist()) & (set(ids.tolist()) | set(b.tolist()))
            assert set(b.tolist()) | set(ids.tolist()) | set(mids.tolist()) == set(np.nonzero(lev == l)[0].tolist())
            for B in set(b.tolist()):
                bnB = max(16, min(sched["bn_cap"], 16 if s[B] <= 16 else 32 if s[B] <= 32 else 64 if s[B] <= 64
                                  else 128))
                assert not (s[B] <= sched["small_s"] and c[B] <= 256)
                assert ((c[B] + 63) // 64) * ((s[B] + bnB - 1) // bnB) > sched["mb_tiles"]
            phase = np.array([phases.index(S.QOPS[o]) for o in top], dtype=np.int64)
            assert np.all(np.diff(phase) >= 0), "tasks must be listed phase by phase"
            # every task waits for exactly the earlier-phase tasks of its block,
            # all of them sit at smaller queue indices and signal their block
            for B in np.unique(b):
                idx = np.nonzero(b == B)[0]
                for k in idx:
                    before = idx[phase[idx] < phase[k]]
                    assert need[k] == len(before)
                    assert np.all(before < k)
                    assert np.all((fl[before] & 2) == 2)
            for B in np.unique(b):
                sB, cB = int(s[B]), int(c[B])
                mine = b == B
                if sweep == 0:
                    assert np.sum(mine & (top == OP["ldlt"])) == 1
                    pt = mine & (top == OP["panel"])
                    cells = sum(min(64, cB - r) * min(w, sB - j) for r, j, w in zip(i0[pt], j0[pt], bn[pt]))
                    assert cells == cB * sB and len(set(zip(i0[pt], j0[pt]))) == pt.sum()
                    assert np.all(bn[pt] <= sched["bn_cap"])
                    st = mine & (top == OP["schur"])
                    nt = (cB + 63) // 64
                    assert sorted(zip(i0[st], j0[st])) == sorted((i * 64, k * 64) for k in range(nt)
                                                                 for i in range(k, nt))
                    assert np.all((fl[st] & 2) == 0)
                else:
                    gt = mine & (top == OP["gemm"])
                    dt = mine & (top == OP["sdiag"])
                    atomic = np.any((fl[gt] & 1) == 1) or np.any((fl[dt] & 1) == 1)
                    assert np.sum(mine & (top == OP["zero"])) == (1 if atomic else 0)
                    assert np.all((fl[dt] & 2) == 0)
                    for sel, keys in ((gt, list(zip(i0[gt], j0[gt]))), (dt, list(zip(i0[dt], j0[dt])))):
                        pieces = {}
                        for key, a, z, f in zip(keys, kb[sel], ke[sel], fl[sel]):
                            pieces.setdefault(key, []).append((a, z, f & 1))
                        for key, pc in pieces.items():
                            pc.sort()
                            lo = 0
                            for a, z, f in pc:
                                assert a == lo and z >= a
                                lo = z
                                assert f == (1 if len(pc) > 1 else 0)
                            assert lo == cB
                    nd = (sB + 31) // 32
                    assert set(zip(i0[dt], j0[dt])) == {(I * 32, J * 32) for I in range(nd) for J in range(I + 1)}
                    cells = sum(min(64, cB - r) * min(w, sB - j) for (r, j), w in
                                dict(zip(zip(i0[gt], j0[gt]), bn[gt])).items())
                    assert cells == cB * sB


@pytest.mark.parametrize("order,bn_cap,fill,small,mb", [(o, b, f, sm, mbt) for o, b, f in itertools.product(
    range(4), (16, 32, 64, 128), (0, 512, 4096)) for sm in ((0, 16) if b != 64 else (0, 1, 2, 4, 8, 16))
    for mbt in ((0, 8) if f != 512 else (0, 1, 8, 4096))])
def test_queue_invariants_every_schedule(order, bn_cap, fill, small, mb):
    p = S.Plan.batch(_small_batch(), max_super=24, exec_cap=24)
    sc = p.set_schedule(order=order, bn_cap=bn_cap, split_fill=fill, grid_mult=1, small_s=small, mb_tiles=mb)
    assert sc == dict(order=order, bn_cap=bn_cap, split_fill=fill, grid_mult=1, small_s=small, mb_tiles=mb)
    check_queues(p)


def test_queue_orders():
    ms = W.batch_2d(count=5, side_lo=20, side_hi=40, seed=9)
    p = S.Plan.batch(ms)
    bm = _block_matrix(p)
    blk = p.blocks()
    cost = 2.0 * blk["c"] ** 2 * blk["s"] + 2.0 * blk["c"] * blk["s"] ** 2 + blk["s"].astype(float) ** 3
    for l in range(1, int(p.info["exec_depth"]) + 1):
        p.set_schedule(order="plan", small_s=0, mb_tiles=0)
        q = p.queue(0, l)
        ld = q[(q[:, 6] >> 8) == OP["ldlt"], 0]
        assert np.all(np.diff(ld) > 0)
        p.set_schedule(order="lpt")
        ld = p.queue(0, l)
        ld = ld[(ld[:, 6] >> 8) == OP["ldlt"], 0]
        assert np.all(np.diff(cost[ld]) <= 0)
        p.set_schedule(order="round_robin")
        ld = p.queue(0, l)
        ld = ld[(ld[:, 6] >> 8) == OP["ldlt"], 0]
        rank = np.array([np.sum((bm[ld] == bm[B]) & (ld < B)) for B in ld])
        assert np.all(np.diff(rank) >= 0)
    check_queues(p)


def test_schedule_validation():
    p = S.Plan.batch(W.batch_2d(count=3, side_lo=8, side_hi=12, seed=2))
    for bad in (dict(order=7), dict(bn_cap=48), dict(split_fill=-1), dict(split_fill=4097), dict(grid_mult=0),
                dict(grid_mult=17), dict(small_s=3), dict(small_s=32), dict(mb_tiles=-1), dict(mb_tiles=5000)):
        with pytest.raises(S.SelinvError) as e:
            p.set_schedule(**bad)
        assert e.value.status == S.SELINV_EINVAL
    assert p.schedule() == dict(order=1, bn_cap=128, split_fill=512, grid_mult=2, small_s=16, mb_tiles=8)


def test_capacity_covers_every_valid_schedule():
    """The queue space the workspace reserves bounds every valid schedule."""
    p = S.Plan.from_matrix(W.laplacian((14, 14, 14), shift=0.1))
    for bn in (16, 32, 64, 128):
        for fill in (0, 1, 100, 511, 512, 2000, 4095, 4096):
            for small in (0, 1, 2, 4, 8, 16):
                for mb in (0, 3, 64, 4096):
                    p.set_schedule(bn_cap=bn, split_fill=fill, small_s=small, mb_tiles=mb)
