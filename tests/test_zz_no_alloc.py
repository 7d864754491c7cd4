"""The static-scratch entry point (selinv_factor_invert_static) through the
C ABI, against the bound-workspace path (selinv_factor + selinv_invert) of
the same plans, at the parity bar of the other GPU tests, on two calls in a
row with the second on a smaller input, then back on the first plan."""
import ctypes as ct

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


def _static(p, vals, out):
    """Direct C-ABI call: no allocation inside (out is given)."""
    from paper_1404_0447_amd import selinv as S
    torch = _torch()
    bad = ct.c_int64(-1)
    st = S.lib().selinv_factor_invert_static(p._h, ct.c_void_p(vals.data_ptr()), ct.c_void_p(out.data_ptr()),
                                             ct.byref(bad), ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, bad.value


def _bound(p, vals):
    p.factor(vals)
    sel = p.invert()
    p.sync_status()
    return sel.cpu().numpy()


def test_static_entry_matches_bound_workspace_two_calls():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    big = W.laplacian((10, 9, 8), coeff="loguniform", lo=0.1, hi=10.0, shift=1e-3, seed=5)
    small = W.laplacian((12, 11), coeff="uniform", lo=0.5, hi=2.0, shift=0.1, seed=1)
    assert small.n < big.n
    plans, vals, outs = [], [], []
    for m in (big, small):
        p = S.Plan.from_matrix(m)
        assert p.info["workspace_bytes"] <= S.STATIC_SCRATCH_BYTES
        plans.append(p)
        vals.append(torch.as_tensor(m.vals, dtype=torch.float64, device="cuda"))
        outs.append(torch.full((int(p.info["nnzL"]),), float("nan"), dtype=torch.float64, device="cuda"))
    for k, m in enumerate((big, small)):  # first the larger input, then the smaller
        print(f"[static] call {k}: n={m.n}", flush=True)
        st, bad = _static(plans[k], vals[k], outs[k])
        assert st == S.SELINV_OK and bad == -1
    # back on the first plan: its tables were replaced in the array and come back
    again = torch.full_like(outs[0], float("nan"))
    st, _ = _static(plans[0], vals[0], again)
    assert st == S.SELINV_OK
    torch.cuda.synchronize()
    for k, m in enumerate((big, small)):
        ref = _bound(plans[k].bind(), vals[k])
        cp, ri, _ = plans[k].pattern()
        got = outs[k].cpu().numpy()
        assert np.all(np.isfinite(got))
        assert H.err_c8(got, ref, cp, ri) <= TOL, f"call {k}"
    cp, ri, _ = plans[0].pattern()
    assert H.err_c8(again.cpu().numpy(), outs[0].cpu().numpy(), cp, ri) <= TOL


def test_static_entry_rejects_large_plans_and_reports_pivots():
    torch = _torch()
    from paper_1404_0447_amd import selinv as S
    from paper_1404_0447_amd import workloads as W
    m = W.laplacian((40, 40, 40), shift=0.1)
    p = S.Plan.from_matrix(m)
    assert p.info["workspace_bytes"] > S.STATIC_SCRATCH_BYTES
    v = torch.as_tensor(m.vals, dtype=torch.float64, device="cuda")
    out = torch.empty(int(p.info["nnzL"]), dtype=torch.float64, device="cuda")
    st, _ = _static(p, v, out)
    assert st == S.SELINV_ENOMEM
    m2 = W.laplacian((6, 6), shift=-10.0)
    p2 = S.Plan.from_matrix(m2)
    v2 = torch.as_tensor(m2.vals, dtype=torch.float64, device="cuda")
    out2 = torch.empty(int(p2.info["nnzL"]), dtype=torch.float64, device="cuda")
    st, bad = _static(p2, v2, out2)
    assert st == S.SELINV_EPIVOT and bad >= 0
