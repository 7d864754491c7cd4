"""Adjoint (reverse sweep) on the GPU, through the C ABI.

f(A) = sum over the pattern of L of w_q * Ainv_q.  The library's reverse
sweep must give df/da for every stored entry of A: checked against the
oracle's dense reference gradient -(A^{-1} S A^{-1}) (small cases, 1e-10),
against directional derivatives and against central finite differences of
the GPU forward (the molecular case of 16^3 atoms x 8, 64 entries, 1e-6).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(m, cap=128, exec_cap=0):
    from paper_1404_0447_amd import selinv as S
    return S.Plan.from_matrix(m, max_super=cap, exec_cap=exec_cap).bind()


def _forward(p, vals):
    torch = _torch()
    v = torch.as_tensor(vals, dtype=torch.float64, device="cuda")
    p.factor(v)
    sel = p.invert()
    p.sync_status()
    return sel


def _weights(p, seed):
    torch = _torch()
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(int(p.info["nnzL"]))
    return w, torch.as_tensor(w, device="cuda")


def _dense_reference(m, p, w):
    """Oracle dense gradient, everything in the original numbering."""
    from oracle import oracle as O
    cp, ri, pm = p.pattern()
    cols = np.repeat(np.arange(m.n), np.diff(cp))
    r0, c0 = pm[ri].astype(np.int64), pm[cols].astype(np.int64)
    order = np.lexsort((r0, c0))
    colptrW = np.zeros(m.n + 1, np.int64)
    np.add.at(colptrW, c0[order] + 1, 1)
    colptrW = np.cumsum(colptrW)
    inv = O.dense_inverse(m.dense())
    return O.dense_grad(inv, colptrW, r0[order].astype(np.int32), w[order], m.colptr, m.rowind)


@pytest.mark.parametrize("case", ["lap2d_16", "lap3d_7", "molecular_4", "random", "lap3d_10_pieces"])
def test_gradient_matches_dense_reference(case):
    _torch()
    from paper_1404_0447_amd import workloads as W
    kw = {}
    if case == "lap2d_16":
        m = W.laplacian((16, 16), coeff="uniform", lo=0.5, hi=2.0, shift=0.1, seed=1)
    elif case == "lap3d_7":
        m = W.laplacian((7, 7, 7), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-2, seed=2)
    elif case == "molecular_4":
        m = W.molecular(side=4, dofs=8, seed=4)
    elif case == "random":
        m = W.random_spd_pattern(200, 0.04, 5)
    else:
        m = W.laplacian((10, 10, 10), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=3)
        kw = dict(cap=256, exec_cap=16)
    p = _plan(m, **kw)
    _forward(p, m.vals)
    w, wt = _weights(p, 0)
    g = p.backward(wt).cpu().numpy()
    ref = _dense_reference(m, p, w)
    scale = np.abs(ref).max()
    err = np.abs(g - ref).max() / scale
    assert err <= 1e-10, f"gradient error {err:.3e}"


def test_directional_derivative():
    """<dA, T> equals (f(A + hT) - f(A - hT)) / 2h for a random symmetric T."""
    torch = _torch()
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((12, 12, 12), coeff="uniform", lo=0.5, hi=2.0, shift=0.05, seed=7)
    p = _plan(m)
    _forward(p, m.vals)
    w, wt = _weights(p, 1)
    g = p.backward(wt).cpu().numpy()
    rng = np.random.default_rng(2)
    T = rng.standard_normal(m.nnz) * np.abs(m.vals)
    h = 1e-5

    def f(v):
        return float(np.dot(w, _forward(p, v).cpu().numpy()))

    fd = (f(m.vals + h * T) - f(m.vals - h * T)) / (2 * h)
    ad = float(np.dot(g, T))
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_autograd_function():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((14, 14), coeff="uniform", lo=0.5, hi=2.0, shift=0.2, seed=4)
    p = _plan(m)
    v = torch.as_tensor(m.vals, device="cuda").requires_grad_(True)
    w, wt = _weights(p, 3)
    sel = S.selinv(v, p)
    loss = (sel * wt).sum()
    (gv,) = torch.autograd.grad(loss, v)
    ref = _dense_reference(m, p, w)
    assert np.abs(gv.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


def test_backward_requires_forward():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((5, 5))
    p = _plan(m)
    with pytest.raises(S.SelinvError) as e:
        p.backward(torch.zeros(int(p.info["nnzL"]), dtype=torch.float64, device="cuda"))
    assert e.value.status == S.SELINV_ESTATE


@pytest.mark.slow
def test_finite_differences_molecular():
    """Central differences on 64 seeded entries of the 16^3-atom matrix."""
    torch = _torch()
    from paper_1404_0447_amd import workloads as W
    m = W.molecular(side=16, dofs=8, seed=4)
    assert m.meta["shift"] == pytest.approx(28.896)
    p = _plan(m)
    _forward(p, m.vals)
    w, wt = _weights(p, 4)
    g = p.backward(wt).cpu().numpy()
    rng = np.random.default_rng(4)
    idx = rng.choice(m.nnz, 64, replace=False)
    gmax = np.abs(g).max()

    def f(v):
        sel = _forward(p, v)
        return float(torch.dot(sel, wt).item())

    # the noise of f itself: repeated evaluations differ by the order of the
    # split contractions' atomic additions; never below a few ulps of f
    f0 = [f(m.vals) for _ in range(4)]
    delta = max(max(f0) - min(f0), 4e-16 * abs(f0[0]))
    worst, resolved, unresolved = 0.0, 0, []
    for q in idx:
        # Richardson over (h, h/2) removes the h^2 truncation term, so h can be
        # large enough that the rounding noise of f (30M terms) / h stays small
        h = 1e-3 * max(1.0, abs(m.vals[q]))
        def fd(step):
            vp = m.vals.copy()
            vm = m.vals.copy()
            vp[q] += step
            vm[q] -= step
            return (f(vp) - f(vm)) / (2 * step)
        d1, d2 = fd(h), fd(h / 2)
        rich = (4 * d2 - d1) / 3  # Richardson: removes the h^2 term
        # each difference quotient carries at most delta / step of f's noise,
        # so the Richardson value at most (4 (2 delta / h) + delta / h) / 3 = 3 delta / h
        noise = 3 * delta / h
        err = abs(rich - g[q])
        if abs(g[q]) >= 1e4 * noise:
            resolved += 1
            worst = max(worst, err / abs(g[q]))
        else:
            unresolved.append((int(q), float(g[q]), float(err), float(noise)))
            assert err <= 1e-6 * abs(g[q]) + 2 * noise, f"entry {q}: error {err:.3e} above its noise bound {noise:.3e}"
    msg = (f"relative FD error {worst:.3e} on {resolved} entries resolved above the noise of f (delta {delta:.2e}); "
           f"{len(unresolved)} entries within their noise bound")
    print(msg, flush=True)
    assert resolved >= 16, msg
    assert worst <= 1e-6, msg
