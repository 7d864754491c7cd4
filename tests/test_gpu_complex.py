"""Complex-symmetric selected inversion on the GPU (A(z) = H - z S, the
matrices of the pole expansion, Section 4.3), through the C ABI, against the
oracle's complex tier O3 (itself pinned to a library inverse and a closed
form).  Bar: max |x - o| / sqrt(|o_ii| |o_jj|) <= 1e-10 over the pattern."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _err(x, o, colptrL, rowindL):
    d = np.abs(o[colptrL[:-1]])
    cols = np.repeat(np.arange(len(colptrL) - 1), np.diff(colptrL))
    return float(np.max(np.abs(x - o) / np.sqrt(d[rowindL] * d[cols])))


def _oracle(m, vals, cap, perm="nd"):
    from oracle import oracle as O
    o = O.symbolic(m, cap=cap, perm=perm)
    sel, st, _ = o.factor_selinv_complex(vals)
    assert st == 0
    return o.sym, sel


def _gpu(p, vals):
    torch = _torch()
    v = torch.as_tensor(np.ascontiguousarray(vals, dtype=np.complex128), device="cuda")
    p.factor_complex(v)
    sel = p.invert_complex()
    p.sync_status()
    return sel.cpu().numpy()


def _cases():
    from paper_1404_0447_amd import workloads as W
    H, S = W.hamiltonian_overlap(side=5, dofs=8, seed=6)
    z = W.poles(8, 0.0, 30.0)
    lap = W.laplacian((12, 11, 10), coeff="loguniform", lo=0.1, hi=10.0, shift=0.0, seed=5)
    lap_diag = lap.rowind == np.repeat(np.arange(lap.n), np.diff(lap.colptr))
    g2 = W.laplacian((30, 28), coeff="uniform", lo=0.5, hi=2.0, shift=0.0, seed=3)
    g2_diag = g2.rowind == np.repeat(np.arange(g2.n), np.diff(g2.colptr))
    return {
        "pencil_z0": (H, W.pencil_values(H, S, z[0]), 128),
        "pencil_z5": (H, W.pencil_values(H, S, z[5]), 128),
        "lap3d_shifted": (lap, lap.vals - (0.5 + 0.25j) * lap_diag, 128),
        "lap2d_shifted": (g2, g2.vals - (1.0 + 1e-3j) * g2_diag, 64),
    }


@pytest.mark.parametrize("name", ["pencil_z0", "pencil_z5", "lap3d_shifted", "lap2d_shifted"])
def test_complex_matches_oracle(name):
    from paper_1404_0447_amd import selinv as S
    m, vals, cap = _cases()[name]
    print(f"[complex] {name} n={m.n}", flush=True)
    p = S.Plan.from_matrix(m, max_super=cap, complex_values=True).bind()
    assert p.blocks()["s"].max() <= 64
    got = _gpu(p, vals)
    s, ref = _oracle(m, vals, cap)
    cp, ri, pm = p.pattern()
    assert np.array_equal(pm, s.perm) and np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
    e = _err(got, ref, cp, ri)
    assert e <= TOL, f"complex selected inverse error {e:.3e}"
    assert np.abs(got.imag).max() > 0  # genuinely complex


def test_real_shift_through_complex_path_equals_real_path():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((16, 15), coeff="uniform", lo=0.5, hi=2.0, shift=0.1, seed=2)
    pz = S.Plan.from_matrix(m, complex_values=True).bind()
    got = _gpu(pz, m.vals.astype(np.complex128))
    pr = S.Plan.from_matrix(m).bind()
    pr.factor(torch.as_tensor(m.vals, device="cuda"))
    real = pr.invert().cpu().numpy()
    pr.sync_status()
    assert np.array_equal(pz.pattern()[1], pr.pattern()[1])
    assert np.abs(got.imag).max() == 0.0
    assert np.abs(got.real - real).max() <= 1e-12 * np.abs(real).max()


def test_pole_batch_one_analysis():
    """Eight poles z_k on a half circle, one analysis of H's pattern, one
    launch per level for all of them; every pole against the oracle."""
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    H, Sm = W.hamiltonian_overlap(side=4, dofs=8, seed=7)
    z = W.poles(8, 0.0, 25.0)
    p = S.Plan.poles(H, len(z)).bind()
    assert p.count == len(z)
    vals = np.concatenate([W.pencil_values(H, Sm, zk) for zk in z])
    got = _gpu(p, vals)
    parts = [got[int(p.nnzL_off[k]):int(p.nnzL_off[k + 1])] for k in range(len(z))]
    one = S.Plan.from_matrix(H, complex_values=True)
    cp, ri, _ = one.pattern()
    worst = 0.0
    for k, zk in enumerate(z):
        s, ref = _oracle(H, W.pencil_values(H, Sm, zk), 128)
        assert np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
        worst = max(worst, _err(parts[k], ref, cp, ri))
    assert worst <= TOL, f"pole batch error {worst:.3e}"


def test_complex_plan_refuses_real_calls():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((6, 6), shift=0.1)
    p = S.Plan.from_matrix(m, complex_values=True).bind()
    with pytest.raises(S.SelinvError) as e:
        p.factor(torch.as_tensor(m.vals, device="cuda"))
    assert e.value.status == S.SELINV_EINVAL
    q = S.Plan.from_matrix(m).bind()
    with pytest.raises(S.SelinvError) as e:
        q.factor_complex(torch.as_tensor(m.vals.astype(np.complex128), device="cuda"))
    assert e.value.status == S.SELINV_EINVAL


def test_complex_zero_pivot_reported_and_plan_recovers():
    """The first pivot of the elimination order set to exactly 0 + 0i: the
    complex factorization reports SELINV_EPIVOT with that original column;
    the same plan then factors a good matrix."""
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((6, 6), coeff="uniform", lo=0.5, hi=2.0, shift=0.1, seed=3)
    print("[complex] zero pivot n=36", flush=True)
    p = S.Plan.from_matrix(m, complex_values=True).bind()
    cp, ri, pm = p.pattern()
    vals = m.vals.astype(np.complex128) * (1.0 + 0.5j)
    first = int(pm[0])
    diag = np.flatnonzero((m.rowind == first) & (np.repeat(np.arange(m.n), np.diff(m.colptr)) == first))
    assert len(diag) == 1
    vals[diag[0]] = 0.0
    p.factor_complex(torch.as_tensor(vals, device="cuda"))
    with pytest.raises(S.SelinvError) as e:
        p.sync_status()
    assert e.value.status == S.SELINV_EPIVOT
    assert e.value.bad_col == first
    good = m.vals.astype(np.complex128) * (1.0 + 0.5j)
    got = _gpu(p, good)
    s, o = _oracle(m, good, 128)
    assert np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
    assert _err(got, o, s.colptrL, s.rowindL) <= TOL


def test_complex_path_is_bitwise_repeatable():
    """The complex schedule adds in a fixed order everywhere (Schur colour
    groups, split diagonal steps summed piece by piece): two runs on the same
    values agree bit for bit."""
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    H, Sm = W.hamiltonian_overlap(side=5, dofs=8, seed=6)
    vals = W.pencil_values(H, Sm, W.poles(8, 0.0, 30.0)[3])
    p = S.Plan.from_matrix(H, max_super=128, complex_values=True).bind()
    a = _gpu(p, vals)
    b = _gpu(p, vals)
    assert np.array_equal(a, b)


def test_pole_batch_full_size_against_oracle():
    """The pole workload the benchmark times, at full size: 32 poles of
    n = 8000 in one batch, in the benchmark's launch configuration.  Poles 0,
    15 and 31 of the batch, and pole 0 on a single-pole plan (every level of
    which cuts its gather-GEMM and diagonal-step contractions into pieces),
    against the oracle's complex tier to the C8 bar."""
    _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    H, Sm = W.hamiltonian_overlap(side=10, dofs=8, seed=6)
    z = W.poles(32, 0.0, 40.0)
    print(f"[complex] pole batch n={H.n} x {len(z)}", flush=True)
    p = S.Plan.poles(H, len(z)).bind()
    got = _gpu(p, np.concatenate([W.pencil_values(H, Sm, zk) for zk in z]))
    offs = [int(x) for x in p.nnzL_off]
    del p
    one = S.Plan.from_matrix(H, complex_values=True).bind()
    got1 = _gpu(one, W.pencil_values(H, Sm, z[0]))
    cp, ri, _ = one.pattern()
    for k in (0, 15, 31):
        print(f"[complex] oracle pole {k}", flush=True)
        s, ref = _oracle(H, W.pencil_values(H, Sm, z[k]), 128)
        assert np.array_equal(cp, s.colptrL) and np.array_equal(ri, s.rowindL)
        e = _err(got[offs[k]:offs[k + 1]], ref, cp, ri)
        assert e <= TOL, f"pole {k}: error {e:.3e}"
        if k == 0:
            e1 = _err(got1, ref, cp, ri)
            assert e1 <= TOL, f"single-pole plan: error {e1:.3e}"
