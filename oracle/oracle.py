"""ctypes driver for the C oracle (oracle.c) -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module. It builds liboracle.so with gcc when asked (``build()``) or when
nothing is built yet.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        vp = ct.c_void_p
        L.orc_nd_order.argtypes = [ct.c_int, _i32p, ct.c_int, _i32p]
        L.orc_nd_order.restype = ct.c_int64
        L.orc_nd_order_sep.argtypes = [ct.c_int, _i32p, ct.c_int, ct.c_int, _i32p]
        L.orc_nd_order_sep.restype = ct.c_int64
        L.orc_symbolic.argtypes = [ct.c_int, _i64p, _i32p, vp, ct.c_int]
        L.orc_symbolic.restype = vp
        L.orc_symbolic_relaxed.argtypes = [ct.c_int, _i64p, _i32p, vp, ct.c_int, ct.c_int]
        L.orc_symbolic_relaxed.restype = vp
        for f in ("orc_sym_error", "orc_sym_nsuper"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = ct.c_int
        for f in ("orc_sym_nnzL", "orc_sym_relsize", "orc_sym_arena"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = ct.c_int64
        L.orc_sym_free.argtypes = [vp]
        L.orc_sym_get.argtypes = [vp] + [vp] * 7
        L.orc_sym_rel.argtypes = [vp, _i64p, _i32p]
        L.orc_sym_pattern.argtypes = [vp, _i64p, _i32p]
        L.orc_sym_flops.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.orc_factor_selinv.argtypes = [vp, _i64p, _i32p, _f64p, ct.c_int, vp, vp,
                                        ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double),
                                        ct.POINTER(ct.c_double)]
        L.orc_factor_selinv.restype = ct.c_int
        L.orc_dense_inverse.argtypes = [ct.c_int, _f64p, _f64p]
        L.orc_dense_inverse.restype = ct.c_int
        L.orc_dense_ldlt.argtypes = [ct.c_int, _f64p, _f64p]
        L.orc_dense_ldlt.restype = ct.c_int
        L.orc_factor_selinv_bk.argtypes = [vp, _i64p, _i32p, _f64p, _f64p, ct.POINTER(ct.c_int64)]
        L.orc_factor_selinv_bk.restype = ct.c_int
        L.orc_factor_selinv_z.argtypes = [vp, _i64p, _i32p, _f64p, _f64p, ct.POINTER(ct.c_int64)]
        L.orc_factor_selinv_z.restype = ct.c_int
        L.orc_dense_inverse_z.argtypes = [ct.c_int, _f64p, _f64p]
        L.orc_dense_inverse_z.restype = ct.c_int
        L.orc_selinv_columns.argtypes = [ct.c_int, _f64p, _i64p, _i32p, _f64p]
        L.orc_selinv_columns.restype = ct.c_int
        L.orc_dense_grad.argtypes = [ct.c_int, _f64p, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p]
        L.orc_set_mutation.argtypes = [ct.c_int]
        L.orc_get_threads.restype = ct.c_int
        L.orc_set_threads.argtypes = [ct.c_int]
        L.orc_set_threads.restype = ct.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def set_mutation(m: int) -> None:
    lib().orc_set_mutation(int(m))


def threads() -> int:
    return int(lib().orc_get_threads())


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's later calls; returns the setting."""
    return int(lib().orc_set_threads(int(n)))


def nd_order(ndim, dims, dofs=1, rim_last=False):
    dims = np.asarray(list(dims) + [1] * (3 - len(dims)), dtype=np.int32)[:3]
    n = int(np.prod(dims[:max(ndim, 1)])) * dofs
    perm = np.empty(n, dtype=np.int32)
    got = lib().orc_nd_order_sep(int(ndim), dims, int(dofs), int(bool(rim_last)), perm)
    assert got == n
    return perm


@dataclass
class Symbolic:
    n: int
    N: int
    perm: np.ndarray
    parent: np.ndarray
    xsuper: np.ndarray
    sparent: np.ndarray
    level: np.ndarray
    cptr: np.ndarray
    crows: np.ndarray
    colptrL: np.ndarray
    rowindL: np.ndarray
    gemm_flops: float
    factor_flops: float
    handle: int = 0
    _maps: tuple = None
    _owner: object = None  # the OracleSym that owns handle (keeps it alive)

    @property
    def nnzL(self):
        return int(self.colptrL[-1])

    def _index_maps(self):
        """Block index maps (built on first use; quadratic in |C|)."""
        if self._maps is None:
            L = lib()
            rs = L.orc_sym_relsize(self.handle)
            rptr = np.empty(self.N + 1, np.int64)
            rel = np.empty(max(rs, 1), np.int32)
            L.orc_sym_rel(self.handle, rptr, rel)
            self._maps = (rptr, rel[:rs])
        return self._maps

    @property
    def rptr(self):
        return self._index_maps()[0]

    @property
    def rel(self):
        return self._index_maps()[1]


class OracleSym:
    """Owns an orc_sym handle."""

    def __init__(self, colptr, rowind, perm, cap, relax=0):
        L = lib()
        n = len(colptr) - 1
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        self._perm = p
        self.h = L.orc_symbolic_relaxed(n, self._colptr, self._rowind, _ptr(p), int(cap), int(relax))
        err = L.orc_sym_error(self.h)
        if err:
            raise ValueError(f"oracle symbolic error {err}")
        N = L.orc_sym_nsuper(self.h)
        nnzL = L.orc_sym_nnzL(self.h)
        perm_o = np.empty(n, np.int32)
        parent = np.empty(n, np.int32)
        xsuper = np.empty(N + 1, np.int32)
        sparent = np.empty(max(N, 1), np.int32)
        level = np.empty(max(N, 1), np.int32)
        cptr = np.empty(N + 1, np.int64)
        L.orc_sym_get(self.h, _ptr(perm_o), _ptr(parent), _ptr(xsuper), _ptr(sparent), _ptr(level),
                      _ptr(cptr), None)
        crows = np.empty(max(int(cptr[-1]), 1), np.int32)
        L.orc_sym_get(self.h, None, None, None, None, None, _ptr(cptr), _ptr(crows))
        colptrL = np.empty(n + 1, np.int64)
        rowindL = np.empty(max(nnzL, 1), np.int32)
        L.orc_sym_pattern(self.h, colptrL, rowindL)
        g, f = ct.c_double(), ct.c_double()
        L.orc_sym_flops(self.h, ct.byref(g), ct.byref(f))
        self.sym = Symbolic(n, N, perm_o, parent, xsuper, sparent[:N], level[:N], cptr,
                            crows[: int(cptr[-1])], colptrL, rowindL[:nnzL], g.value, f.value, self.h,
                            _owner=self)

    def factor_selinv(self, vals, require_spd=True, want_L=False):
        """O3: returns (sel, L_or_None, status, bad_col, t_factor, t_selinv)."""
        L = lib()
        nnzL = self.sym.nnzL
        sel = np.empty(max(nnzL, 1))
        Lv = np.empty(max(nnzL, 1)) if want_L else None
        bad = ct.c_int64(-1)
        tf, ts = ct.c_double(), ct.c_double()
        st = L.orc_factor_selinv(self.h, self._colptr, self._rowind,
                                 np.ascontiguousarray(vals, dtype=np.float64), int(require_spd),
                                 _ptr(sel), _ptr(Lv), ct.byref(bad), ct.byref(tf), ct.byref(ts))
        return (sel[:nnzL], None if Lv is None else Lv[:nnzL], st, bad.value, tf.value, ts.value)

    def factor_selinv_pivoted(self, vals):
        """O3 with 1x1/2x2 (Bunch-Kaufman) pivots inside each diagonal block,
        for symmetric indefinite matrices: returns (sel, status, bad_col)."""
        nnzL = self.sym.nnzL
        out = np.empty(max(nnzL, 1))
        bad = ct.c_int64(-1)
        st = lib().orc_factor_selinv_bk(self.h, self._colptr, self._rowind,
                                        np.ascontiguousarray(vals, dtype=np.float64), out, ct.byref(bad))
        return out[:nnzL], st, bad.value

    def factor_selinv_complex(self, vals):
        """O3 on complex values (a complex array, nnzA): returns
        (complex sel on the pattern, status, bad_col)."""
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.complex128)).view(np.float64)
        nnzL = self.sym.nnzL
        out = np.empty(2 * max(nnzL, 1))
        bad = ct.c_int64(-1)
        st = lib().orc_factor_selinv_z(self.h, self._colptr, self._rowind, v, out, ct.byref(bad))
        return out[: 2 * nnzL].view(np.complex128).copy(), st, bad.value

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_sym_free(self.h)
                self.h = None
        except Exception:
            pass


def symbolic(m, cap=128, perm="nd", relax=0):
    """Oracle symbolic for a workloads.Matrix. perm: "nd" (from geometry),
    "nd_rim" (separator rims last), "natural", or an explicit new->old array.
    relax > 0: relaxed supernodes of at most `relax` columns."""
    if isinstance(perm, str):
        if perm in ("nd", "nd_rim") and m.ndim > 0:
            p = nd_order(m.ndim, m.dims, m.dofs, rim_last=perm == "nd_rim")
        else:
            p = None
    else:
        p = perm
    return OracleSym(m.colptr, m.rowind, p, cap, relax)


def dense_inverse(a):
    """O1 with plain C arrays (column-major in, column-major out)."""
    n = a.shape[0]
    src = np.ascontiguousarray(np.asarray(a, dtype=np.float64).T).ravel()
    dst = np.empty(n * n)
    st = lib().orc_dense_inverse(n, src, dst)
    if st != 0:
        raise ValueError("dense LDL^T hit a zero pivot")
    return dst.reshape(n, n).T.copy()


def dense_inverse_complex(a):
    """O1 for a complex symmetric matrix (no conjugation anywhere)."""
    n = a.shape[0]
    src = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).T).view(np.float64).ravel()
    dst = np.empty(2 * n * n)
    if lib().orc_dense_inverse_z(n, src, dst) != 0:
        raise ValueError("dense LDL^T hit a zero pivot")
    return dst.view(np.complex128).reshape(n, n).T.copy()


def dense_ldlt(a):
    """O1's dense factor: (L unit lower, d) with A = L diag(d) L^T."""
    n = a.shape[0]
    src = np.ascontiguousarray(np.asarray(a, dtype=np.float64).T).ravel()
    dst = np.empty(n * n)
    if lib().orc_dense_ldlt(n, src, dst) != 0:
        raise ValueError("dense LDL^T hit a zero pivot")
    f = dst.reshape(n, n).T
    return np.tril(f, -1) + np.eye(n), np.diag(f).copy()


def selinv_columns(a_perm, colptrL, rowindL):
    """O2 on a dense permuted matrix and the canonical pattern of L."""
    n = a_perm.shape[0]
    src = np.ascontiguousarray(np.asarray(a_perm, dtype=np.float64).T).ravel()
    sel = np.empty(int(colptrL[-1]))
    st = lib().orc_selinv_columns(n, src, np.ascontiguousarray(colptrL, dtype=np.int64),
                                  np.ascontiguousarray(rowindL, dtype=np.int32), sel)
    if st != 0:
        raise ValueError("dense LDL^T hit a zero pivot")
    return sel


def dense_grad(ainv_perm, colptrL, rowindL, w, colptrA, rowindA):
    n = ainv_perm.shape[0]
    src = np.ascontiguousarray(np.asarray(ainv_perm, dtype=np.float64).T).ravel()
    g = np.empty(int(colptrA[-1]))
    lib().orc_dense_grad(n, src, np.ascontiguousarray(colptrL, np.int64),
                         np.ascontiguousarray(rowindL, np.int32), np.ascontiguousarray(w, np.float64),
                         np.ascontiguousarray(colptrA, np.int64), np.ascontiguousarray(rowindA, np.int32), g)
    return g
