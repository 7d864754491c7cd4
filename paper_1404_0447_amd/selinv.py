"""Python binding of libselinv.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; torch only provides
device memory (the workspace and the value/output tensors) and the stream.
If the library is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libselinv.so")

SELINV_OK, SELINV_EINVAL, SELINV_ESTATE, SELINV_EPIVOT = 0, -1, -2, -3
SELINV_ENOMEM, SELINV_EHIP, SELINV_EUNSUPPORTED, SELINV_EQUEUE = -4, -5, -6, -7
_NAMES = {0: "OK", -1: "EINVAL", -2: "ESTATE", -3: "EPIVOT", -4: "ENOMEM", -5: "EHIP", -6: "EUNSUPPORTED",
          -7: "EQUEUE"}

# every symbol include/selinv.h declares
EXPORTS = ["selinv_analyze", "selinv_workspace_size", "selinv_workspace_sizes", "selinv_bind_workspace",
           "selinv_bind_transient", "selinv_generation", "selinv_factor", "selinv_invert", "selinv_backward",
           "selinv_get_factor", "selinv_sync_status", "selinv_get_info", "selinv_get_pattern",
           "selinv_symbolic_sizes", "selinv_get_symbolic", "selinv_profile", "selinv_profile_read",
           "selinv_kernel_work", "selinv_get_arena", "selinv_get_blocks", "selinv_get_exec_rows",
           "selinv_analyze_batch", "selinv_analyze_poles", "selinv_factor_complex", "selinv_invert_complex",
           "selinv_batch_offsets", "selinv_set_schedule", "selinv_get_schedule",
           "selinv_get_queue", "selinv_set_spin_limit", "selinv_run", "selinv_tune", "selinv_measure_peaks",
           "selinv_factor_invert_static", "selinv_last_error", "selinv_destroy"]
STATIC_SCRATCH_BYTES = 64 << 20
ARENAS = {"L": 0, "Ainv": 1, "Lhat": 2, "W": 3, "T": 4, "Fbar": 5, "Lhat_bar": 6, "T_bar": 7}
KINDS = ["assemble", "ldlt", "panel", "schur", "gemm", "sdiag", "export", "revsel", "revfac", "qfactor", "qinvert",
         "sbfactor", "sbinvert", "checkpoint"]
QOPS = ["ldlt", "panel", "schur", "zero", "gemm", "sdiag", "sbfactor", "sbinvert", "mbfactor", "mbinvert"]
ORDERS = ["plan", "lpt", "round_robin", "tile_lpt"]


class SelinvError(RuntimeError):
    def __init__(self, status, msg, bad_col=-1):
        super().__init__(f"selinv {_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.bad_col = bad_col


class Geom(ct.Structure):
    _fields_ = [("ndim", ct.c_int32), ("dims", ct.c_int32 * 3), ("dofs_per_point", ct.c_int32)]


class Opts(ct.Structure):
    _fields_ = [("max_super", ct.c_int32), ("fuse_chains", ct.c_int32), ("require_spd", ct.c_int32),
                ("exec_cap", ct.c_int32), ("sep_order", ct.c_int32), ("deterministic", ct.c_int32),
                ("checkpoint_every", ct.c_int32), ("relaxed", ct.c_int32), ("complex_values", ct.c_int32),
                ("pivoting", ct.c_int32)]


def _opts(max_super, fuse_chains, require_spd, exec_cap, sep_order, deterministic, checkpoint_every, relaxed,
          complex_values=False, pivoting=False):
    so = {"lex": 0, "rim_last": 1}.get(sep_order, sep_order)
    return Opts(int(max_super), int(bool(fuse_chains)), int(bool(require_spd)), int(exec_cap), int(so),
                int(bool(deterministic)), int(checkpoint_every), int(bool(relaxed)), int(bool(complex_values)),
                int(bool(pivoting)))


class Sched(ct.Structure):
    _fields_ = [("order", ct.c_int32), ("bn_cap", ct.c_int32), ("split_fill", ct.c_int32), ("grid_mult", ct.c_int32),
                ("small_s", ct.c_int32), ("mb_tiles", ct.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Info(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("nnzA", ct.c_int64), ("nnzL", ct.c_int64), ("nsuper", ct.c_int64),
                ("depth", ct.c_int64), ("nblocks", ct.c_int64), ("exec_depth", ct.c_int64),
                ("workspace_bytes", ct.c_int64), ("flops_factor", ct.c_double), ("flops_gemm", ct.c_double),
                ("flops_selinv", ct.c_double), ("gather_bytes", ct.c_double), ("exec_flops_gemm", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built; run __graft_entry__.build() (no fallback exists)")
        L = ct.CDLL(LIB)
        vp, i64, i32 = ct.c_void_p, ct.c_int64, ct.c_int32
        L.selinv_analyze.argtypes = [i64, vp, vp, vp, vp, vp, ct.POINTER(vp)]
        L.selinv_workspace_size.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.selinv_workspace_sizes.argtypes = [vp, ct.POINTER(ct.c_size_t), ct.POINTER(ct.c_size_t)]
        L.selinv_bind_workspace.argtypes = [vp, vp, ct.c_size_t, vp]
        L.selinv_bind_transient.argtypes = [vp, vp, ct.c_size_t]
        L.selinv_generation.argtypes = [vp, ct.POINTER(ct.c_uint64)]
        L.selinv_factor.argtypes = [vp, vp, vp]
        L.selinv_invert.argtypes = [vp, vp, vp]
        L.selinv_get_factor.argtypes = [vp, vp, vp]
        L.selinv_backward.argtypes = [vp, vp, vp, vp]
        L.selinv_sync_status.argtypes = [vp, vp, ct.POINTER(i64)]
        L.selinv_get_info.argtypes = [vp, ct.POINTER(Info)]
        L.selinv_get_pattern.argtypes = [vp, vp, vp, vp]
        L.selinv_symbolic_sizes.argtypes = [vp, ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(i64)]
        L.selinv_get_symbolic.argtypes = [vp] + [vp] * 8
        L.selinv_profile.argtypes = [vp, ct.c_int32]
        L.selinv_profile_read.argtypes = [vp, vp, vp]
        L.selinv_kernel_work.argtypes = [vp, vp, vp]
        L.selinv_get_arena.argtypes = [vp, ct.c_int32, vp, ct.POINTER(i64), vp]
        L.selinv_get_blocks.argtypes = [vp] + [vp] * 8
        L.selinv_get_exec_rows.argtypes = [vp, vp]
        L.selinv_analyze_batch.argtypes = [i32, vp, vp, vp, vp, vp, ct.POINTER(vp)]
        L.selinv_analyze_poles.argtypes = [i64, vp, vp, vp, vp, vp, i32, ct.POINTER(vp)]
        L.selinv_factor_complex.argtypes = [vp, vp, vp]
        L.selinv_invert_complex.argtypes = [vp, vp, vp]
        L.selinv_batch_offsets.argtypes = [vp, ct.POINTER(i32), vp, vp, vp]
        L.selinv_set_schedule.argtypes = [vp, ct.POINTER(Sched), vp]
        L.selinv_get_schedule.argtypes = [vp, ct.POINTER(Sched)]
        L.selinv_get_queue.argtypes = [vp, i32, i32, vp, ct.POINTER(i64)]
        L.selinv_set_spin_limit.argtypes = [vp, ct.c_uint32]
        L.selinv_run.argtypes = [vp, vp, vp, i32, vp]
        L.selinv_tune.argtypes = [vp, vp, vp, ct.c_char_p, ct.POINTER(Sched), ct.POINTER(ct.c_double), vp]
        L.selinv_measure_peaks.argtypes = [vp, ct.c_size_t, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), vp]
        L.selinv_factor_invert_static.argtypes = [vp, vp, vp, ct.POINTER(i64), vp]
        L.selinv_last_error.restype = ct.c_char_p
        L.selinv_destroy.argtypes = [vp]
        for f in EXPORTS:
            if f not in ("selinv_last_error", "selinv_destroy"):
                getattr(L, f).restype = ct.c_int
        _lib = L
    return _lib


def _check(st, bad=-1):
    if st != SELINV_OK:
        msg = lib().selinv_last_error().decode(errors="replace")
        raise SelinvError(st, msg, bad)


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class Plan:
    """Symbolic analysis + bound device workspace for one sparsity pattern."""

    def __init__(self, n, colptr, rowind, geom=None, perm=None, max_super=128, fuse_chains=True,
                 require_spd=True, exec_cap=0, sep_order=0, deterministic=False, checkpoint_every=1,
                 relaxed=False, complex_values=False, pivoting=False, _handle=None):
        L = lib()
        self.n = int(n)
        if _handle is not None:
            self.checkpoint_every, self.deterministic = 1, False  # set by the caller (batch)
            self._adopt(_handle)
            return
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        g = None
        if geom is not None:
            ndim, dims, dofs = geom
            d3 = list(dims) + [1] * (3 - len(dims))
            g = Geom(int(ndim), (ct.c_int32 * 3)(*[int(x) for x in d3[:3]]), int(dofs))
        pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        if pivoting:
            require_spd = False  # a pivoted factorization takes indefinite blocks
        o = _opts(max_super, fuse_chains, require_spd, exec_cap, sep_order, deterministic, checkpoint_every,
                  relaxed, complex_values, pivoting)
        self.checkpoint_every = max(1, int(checkpoint_every))
        self.deterministic = bool(deterministic)
        h = ct.c_void_p()
        st = L.selinv_analyze(self.n, _p(self._colptr), _p(self._rowind), ct.byref(g) if g is not None else None,
                              _p(pm), ct.byref(o), ct.byref(h))
        _check(st)
        self._adopt(h)

    def _adopt(self, h):
        L = lib()
        self._h = h
        self._ws = None
        self._tr = None
        self._bound = False
        pb, tb = ct.c_size_t(), ct.c_size_t()
        _check(L.selinv_workspace_sizes(self._h, ct.byref(pb), ct.byref(tb)))
        self.persistent_bytes, self.transient_bytes = int(pb.value), int(tb.value)
        inf = Info()
        _check(L.selinv_get_info(self._h, ct.byref(inf)))
        self.info = {k: getattr(inf, k) for k, _ in Info._fields_}
        cnt = ct.c_int32()
        _check(L.selinv_batch_offsets(self._h, ct.byref(cnt), None, None, None))
        self.count = int(cnt.value)
        offs = [np.empty(self.count + 1, np.int64) for _ in range(3)]
        _check(L.selinv_batch_offsets(self._h, None, *[_p(o) for o in offs]))
        self.n_off, self.nnzA_off, self.nnzL_off = offs

    @classmethod
    def batch(cls, matrices, max_super=128, fuse_chains=True, require_spd=True, exec_cap=0, sep_order=0,
              deterministic=False, checkpoint_every=1, relaxed=False):
        """One plan for a list of independent workloads.Matrix (their
        block-diagonal union); values and results concatenate in list order."""
        L = lib()
        cnt = len(matrices)
        cps = [np.ascontiguousarray(m.colptr, dtype=np.int64) for m in matrices]
        ris = [np.ascontiguousarray(m.rowind, dtype=np.int32) for m in matrices]
        ns = np.array([m.n for m in matrices], dtype=np.int64)
        cp_arr = (ct.c_void_p * max(cnt, 1))(*[c.ctypes.data for c in cps])
        ri_arr = (ct.c_void_p * max(cnt, 1))(*[r.ctypes.data if r.size else None for r in ris])
        geoms = (Geom * max(cnt, 1))()
        for i, m in enumerate(matrices):
            d3 = list(m.dims) + [1] * (3 - len(m.dims))
            geoms[i] = Geom(int(m.ndim), (ct.c_int32 * 3)(*[int(x) for x in d3[:3]]), int(m.dofs))
        o = _opts(max_super, fuse_chains, require_spd, exec_cap, sep_order, deterministic, checkpoint_every,
                  relaxed)
        h = ct.c_void_p()
        st = L.selinv_analyze_batch(cnt, _p(ns), cp_arr, ri_arr, geoms, ct.byref(o), ct.byref(h))
        _check(st)
        p = cls(int(ns.sum()), None, None, _handle=h)
        p.checkpoint_every, p.deterministic = max(1, int(checkpoint_every)), bool(deterministic)
        return p

    @classmethod
    def poles(cls, m, count, max_super=128, fuse_chains=True, exec_cap=0, sep_order=0, relaxed=False):
        """One analysis of the pattern of workloads.Matrix m for `count` complex
        matrices A(z_k) = H - z_k S on that pattern (block-diagonal union, one
        launch per level for all poles)."""
        L = lib()
        cp = np.ascontiguousarray(m.colptr, dtype=np.int64)
        ri = np.ascontiguousarray(m.rowind, dtype=np.int32)
        g = None
        if m.ndim > 0:
            d3 = list(m.dims) + [1] * (3 - len(m.dims))
            g = Geom(int(m.ndim), (ct.c_int32 * 3)(*[int(x) for x in d3[:3]]), int(m.dofs))
        o = _opts(max_super, fuse_chains, False, exec_cap, sep_order, False, 1, relaxed, True)
        h = ct.c_void_p()
        _check(L.selinv_analyze_poles(m.n, _p(cp), _p(ri), ct.byref(g) if g is not None else None, None, ct.byref(o),
                                      int(count), ct.byref(h)))
        p = cls(m.n * int(count), None, None, _handle=h)
        p.deterministic = True
        return p

    @classmethod
    def from_matrix(cls, m, **kw):
        geom = (m.ndim, m.dims, m.dofs) if m.ndim > 0 else None
        return cls(m.n, m.colptr, m.rowind, geom=geom, **kw)

    # ------------------------------------------------------------ host queries
    def pattern(self):
        nnzL = int(self.info["nnzL"])
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(max(nnzL, 1), np.int32)
        pm = np.empty(max(self.n, 1), np.int32)
        _check(lib().selinv_get_pattern(self._h, _p(cp), _p(ri), _p(pm)))
        return cp, ri[:nnzL], pm[: self.n]

    def symbolic(self):
        L = lib()
        N, nc, nr = ct.c_int64(), ct.c_int64(), ct.c_int64()
        _check(L.selinv_symbolic_sizes(self._h, ct.byref(N), ct.byref(nc), ct.byref(nr)))
        N, nc, nr = N.value, nc.value, nr.value
        out = dict(parent=np.empty(max(self.n, 1), np.int32), xsuper=np.empty(N + 1, np.int32),
                   sparent=np.empty(max(N, 1), np.int32), level=np.empty(max(N, 1), np.int32),
                   cptr=np.empty(N + 1, np.int64), crows=np.empty(max(nc, 1), np.int32),
                   rptr=np.empty(N + 1, np.int64), rel=np.empty(max(nr, 1), np.int32))
        _check(L.selinv_get_symbolic(self._h, *[_p(out[k]) for k in
                                                ("parent", "xsuper", "sparent", "level", "cptr", "crows", "rptr",
                                                 "rel")]))
        out["parent"] = out["parent"][: self.n]
        out["sparent"] = out["sparent"][:N]
        out["level"] = out["level"][:N]
        out["crows"] = out["crows"][:nc]
        out["rel"] = out["rel"][:nr]
        return out

    # ------------------------------------------------------------ device calls
    def bind(self, device="cuda", stream=None):
        """Allocate and bind the persistent workspace and a separate transient
        buffer (released with release_transient, re-allocated on demand)."""
        import torch
        self._ws = torch.empty(max(self.persistent_bytes, 1), dtype=torch.uint8, device=device)
        _check(lib().selinv_bind_workspace(self._h, ct.c_void_p(self._ws.data_ptr()), self.persistent_bytes,
                                           _stream(stream)))
        self._bound = True
        self._tr = None
        self._ensure_transient()
        return self

    def _ensure_transient(self):
        import torch
        if self._tr is None:
            self._tr = torch.empty(max(self.transient_bytes, 1), dtype=torch.uint8, device=self._ws.device)
            _check(lib().selinv_bind_transient(self._h, ct.c_void_p(self._tr.data_ptr()), self.transient_bytes))

    def release_transient(self, stream=None):
        """Give the transient buffer back to torch's caching allocator (in
        stream order: work already queued on `stream` still reads it).  The
        inverse panels are lost; selinv_backward then needs
        checkpoint_every > 1."""
        if self._tr is not None:
            if stream is not None:
                self._tr.record_stream(stream)
            _check(lib().selinv_bind_transient(self._h, None, 0))
            self._tr = None

    def generation(self):
        g = ct.c_uint64()
        _check(lib().selinv_generation(self._h, ct.byref(g)))
        return int(g.value)

    def _need(self, t, n, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == n):
            raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor with {n} entries")

    def factor(self, vals, stream=None):
        if not self._bound:
            self.bind(device=vals.device)
        self._need(vals, int(self.info["nnzA"]), "vals")
        _check(lib().selinv_factor(self._h, ct.c_void_p(vals.data_ptr()), _stream(stream)))

    def invert(self, out=None, stream=None):
        import torch
        nnzL = int(self.info["nnzL"])
        if out is None:
            out = torch.empty(nnzL, dtype=torch.float64, device=self._ws.device)
        self._need(out, nnzL, "out")
        self._ensure_transient()
        _check(lib().selinv_invert(self._h, ct.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def _need_z(self, t, n, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                and t.numel() == n):
            raise ValueError(f"{name}: expected a contiguous complex128 CUDA tensor with {n} entries")

    def factor_complex(self, vals, stream=None):
        """LDL^T of a complex symmetric matrix (complex128 values on A's pattern)."""
        if not self._bound:
            self.bind(device=vals.device)
        self._need_z(vals, int(self.info["nnzA"]), "vals")
        _check(lib().selinv_factor_complex(self._h, ct.c_void_p(vals.data_ptr()), _stream(stream)))

    def invert_complex(self, out=None, stream=None):
        import torch
        nnzL = int(self.info["nnzL"])
        if out is None:
            out = torch.empty(nnzL, dtype=torch.complex128, device=self._ws.device)
        self._need_z(out, nnzL, "out")
        self._ensure_transient()
        _check(lib().selinv_invert_complex(self._h, ct.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def backward(self, gsel, out=None, stream=None):
        """d(sum gsel * Ainv on L's pattern)/d(A's stored entries), on the device."""
        import torch
        self._need(gsel, int(self.info["nnzL"]), "gsel")
        if out is None:
            out = torch.empty(int(self.info["nnzA"]), dtype=torch.float64, device=self._ws.device)
        self._need(out, int(self.info["nnzA"]), "out")
        self._ensure_transient()
        _check(lib().selinv_backward(self._h, ct.c_void_p(gsel.data_ptr()), ct.c_void_p(out.data_ptr()),
                                     _stream(stream)))
        return out

    # ------------------------------------------------------------ persistent path
    def schedule(self):
        sc = Sched()
        _check(lib().selinv_get_schedule(self._h, ct.byref(sc)))
        return sc.as_dict()

    def set_schedule(self, order=None, bn_cap=None, split_fill=None, grid_mult=None, small_s=None, mb_tiles=None,
                     stream=None):
        cur = self.schedule()
        for k, v in (("order", order), ("bn_cap", bn_cap), ("split_fill", split_fill), ("grid_mult", grid_mult),
                     ("small_s", small_s), ("mb_tiles", mb_tiles)):
            if v is not None:
                cur[k] = ORDERS.index(v) if (k == "order" and isinstance(v, str)) else int(v)
        sc = Sched(**cur)
        _check(lib().selinv_set_schedule(self._h, ct.byref(sc), _stream(stream) if self._bound else None))
        return self.schedule()

    def queue(self, sweep, level):
        """Host copy of one level's work queue: int32 array (tasks, 8)."""
        cnt = ct.c_int64()
        _check(lib().selinv_get_queue(self._h, int(sweep), int(level), None, ct.byref(cnt)))
        out = np.empty((max(cnt.value, 1), 8), np.int32)
        _check(lib().selinv_get_queue(self._h, int(sweep), int(level), _p(out), ct.byref(cnt)))
        return out[: cnt.value]

    def set_spin_limit(self, polls):
        _check(lib().selinv_set_spin_limit(self._h, int(polls)))

    def run(self, vals, out=None, graph=False, stream=None):
        """Factor + invert on the persistent level kernels (graph=True:
        replayed from a captured HIP graph)."""
        import torch
        if not self._bound:
            self.bind(device=vals.device)
        self._need(vals, int(self.info["nnzA"]), "vals")
        nnzL = int(self.info["nnzL"])
        if out is None:
            out = torch.empty(nnzL, dtype=torch.float64, device=self._ws.device)
        self._need(out, nnzL, "out")
        self._ensure_transient()
        _check(lib().selinv_run(self._h, ct.c_void_p(vals.data_ptr()), ct.c_void_p(out.data_ptr()),
                                int(bool(graph)), _stream(stream)))
        return out

    def tune(self, vals, out=None, cache_path=None, stream=None):
        """Autotune the persistent schedule on these values; returns
        (schedule dict, best ms, selected inverse)."""
        import torch
        if not self._bound:
            self.bind(device=vals.device)
        self._need(vals, int(self.info["nnzA"]), "vals")
        nnzL = int(self.info["nnzL"])
        if out is None:
            out = torch.empty(nnzL, dtype=torch.float64, device=self._ws.device)
        self._need(out, nnzL, "out")
        sc = Sched()
        ms = ct.c_double()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._ensure_transient()
        _check(lib().selinv_tune(self._h, ct.c_void_p(vals.data_ptr()), ct.c_void_p(out.data_ptr()), path,
                                 ct.byref(sc), ct.byref(ms), _stream(stream)))
        return sc.as_dict(), float(ms.value), out

    def factor_invert_static(self, vals, out=None, check=True, stream=None):
        """Factor + invert in the library's static device scratch (no device
        allocation inside the call; out must be given to allocate nothing
        here either).  check=True synchronises and reports a pivot failure."""
        import torch
        nnzL = int(self.info["nnzL"])
        self._need(vals, int(self.info["nnzA"]), "vals")
        if out is None:
            out = torch.empty(nnzL, dtype=torch.float64, device=vals.device)
        self._need(out, nnzL, "out")
        bad = ct.c_int64(-1)
        st = lib().selinv_factor_invert_static(self._h, ct.c_void_p(vals.data_ptr()), ct.c_void_p(out.data_ptr()),
                                               ct.byref(bad) if check else None, _stream(stream))
        _check(st, bad.value)
        return out

    def split(self, sel):
        """Per-matrix views of a batch's concatenated selected values."""
        return [sel[int(self.nnzL_off[m]):int(self.nnzL_off[m + 1])] for m in range(self.count)]

    def factor_values(self, out=None, stream=None):
        import torch
        nnzL = int(self.info["nnzL"])
        if out is None:
            out = torch.empty(nnzL, dtype=torch.float64, device=self._ws.device)
        self._need(out, nnzL, "out")
        _check(lib().selinv_get_factor(self._h, ct.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def sync_status(self, stream=None):
        bad = ct.c_int64(-1)
        st = lib().selinv_sync_status(self._h, _stream(stream), ct.byref(bad))
        _check(st, bad.value)

    def profile(self, enable=True):
        _check(lib().selinv_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{kind: (ms, launches)} for the launches recorded since the last read."""
        ms = np.zeros(len(KINDS))
        nl = np.zeros(len(KINDS), np.int64)
        _check(lib().selinv_profile_read(self._h, _p(ms), _p(nl)))
        return {k: (float(ms[i]), int(nl[i])) for i, k in enumerate(KINDS)}

    def kernel_work(self):
        """{kind: (flops, bytes)} of one factor (assemble..schur) / invert (gemm..export) call."""
        f = np.zeros(len(KINDS))
        b = np.zeros(len(KINDS))
        _check(lib().selinv_kernel_work(self._h, _p(f), _p(b)))
        return {k: (float(f[i]), float(b[i])) for i, k in enumerate(KINDS)}

    def blocks(self):
        """Execution blocks: dict of arrays (first, s, c, level, poff, hoff, woff, crow_off, rows)."""
        nb = int(self.info["nblocks"])
        out = {k: np.empty(max(nb, 1), np.int32) for k in ("first", "s", "c", "level")}
        out.update({k: np.empty(max(nb, 1), np.int64) for k in ("poff", "hoff", "woff", "crow_off")})
        _check(lib().selinv_get_blocks(self._h, *[_p(out[k]) for k in ("first", "s", "c", "level", "poff", "hoff",
                                                                         "woff", "crow_off")]))
        out = {k: v[:nb] for k, v in out.items()}
        rows = np.empty(max(int(out["c"].sum()) if nb else 0, 1), np.int32)
        _check(lib().selinv_get_exec_rows(self._h, _p(rows)))
        out["rows"] = rows[: int(out["c"].sum()) if nb else 0]
        return out

    def arena(self, which, stream=None):
        """Copy of a device arena ("L", "Ainv", "Lhat", "W", "T") as a CUDA
        tensor of doubles (a complex plan's: (re, im) pairs, for a view as
        complex128)."""
        import torch
        n = ct.c_int64()
        _check(lib().selinv_get_arena(self._h, ARENAS[which], None, ct.byref(n), None))
        out = torch.empty(max(n.value, 1), dtype=torch.float64, device=self._ws.device)
        _check(lib().selinv_get_arena(self._h, ARENAS[which], ct.c_void_p(out.data_ptr()), ct.byref(n),
                                      _stream(stream)))
        return out[: n.value]

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().selinv_destroy(self._h)
                self._h = None
        except Exception:
            pass


def measure_peaks(device="cuda", nbytes=2 << 30, stream=None):
    """Measured FP64 MFMA TFLOP/s and copy GB/s of the device (roofline
    ceilings beside the published ones)."""
    import torch
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    tf, gb = ct.c_double(), ct.c_double()
    st = lib().selinv_measure_peaks(ct.c_void_p(buf.data_ptr()), nbytes, ct.byref(tf), ct.byref(gb),
                                    _stream(stream))
    if st != SELINV_OK:
        raise SelinvError(st, "measure_peaks failed")
    return float(tf.value), float(gb.value)


def _autograd_function():
    import torch

    class SelInv(torch.autograd.Function):
        """vals (A's stored lower entries, nnzA) -> selected entries of A^{-1}
        on the pattern of L (nnzL).  The backward is the library's reverse
        sweep; an off-diagonal entry of A stands for A_ij and A_ji.

        The forward synchronises once to report a pivot failure.  The plan
        holds the factor and the inverse the backward differentiates: a later
        forward on the same plan replaces them, and the backward of the
        earlier one then raises.  With checkpoint_every > 1 the transient
        memory is released between forward and backward (the backward
        rebuilds the inverse panels from the checkpoints)."""

        @staticmethod
        def forward(ctx, vals, plan):
            plan.factor(vals.contiguous())
            sel = plan.invert()
            plan.sync_status()
            ctx.plan = plan
            ctx.generation = plan.generation()
            if plan.checkpoint_every > 1:
                plan.release_transient()
            return sel

        @staticmethod
        def backward(ctx, gsel):
            plan = ctx.plan
            if plan.generation() != ctx.generation:
                raise RuntimeError("selinv backward: the plan ran another factorization after this forward; "
                                   "its factor and inverse belong to other values (use one plan per forward)")
            g = plan.backward(gsel.contiguous().to(torch.float64))
            return g, None

    return SelInv


_SelInv = None


def selinv(vals, plan):
    """Differentiable selected inversion: ``selinv(vals, plan)`` with ``vals``
    a float64 CUDA tensor of A's stored lower entries."""
    global _SelInv
    if _SelInv is None:
        _SelInv = _autograd_function()
    return _SelInv.apply(vals, plan)


def selected_inverse(m, vals=None, **kw):
    """One-shot helper: analyze, factor and invert a workloads.Matrix on the
    current CUDA device. Returns (plan, selected values tensor)."""
    import torch
    plan = Plan.from_matrix(m, **kw).bind()
    v = torch.as_tensor(m.vals if vals is None else vals, dtype=torch.float64).cuda()
    plan.factor(v)
    sel = plan.invert()
    plan.sync_status()
    return plan, sel
