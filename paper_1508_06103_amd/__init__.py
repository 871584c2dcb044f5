"""Python binding of libstkkt (include/stkkt.h): argument marshalling only.

Every step of the solve runs in the HIP library.  PyTorch provides device
memory (through the allocator callbacks) and the HIP stream.  If the compiled
library is missing, importing this package raises: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np
import torch  # imported first so that the teardown below runs before torch's own

_HERE = os.path.dirname(os.path.abspath(__file__))
# STKKT_LIB may name another build of the same library (e.g. an instrumented one)
LIB_PATH = os.environ.get("STKKT_LIB", os.path.join(_HERE, "libstkkt.so"))

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, EBREAKDOWN = 0, 1, -1, -2, -3, -4
DTO, OTD = 0, 1
F64, F32 = 0, 1
RESTRICT_TRANSPOSE, RESTRICT_INJECTION = 0, 1
COARSE_LU, COARSE_GMRES_RAS = 0, 1
RHS_SCRATCH_BYTES = 1 << 20   # STKKT_RHS_SCRATCH_BYTES: staging array of kkt_rhs_noalloc


class StkktError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1508_06103_amd/build.py (no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.POINTER(ctypes.c_double)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Alloc(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("nt", ctypes.c_int32), ("len", ctypes.c_double * 3),
                ("T", ctypes.c_double), ("a_elem", _c_dp), ("v", ctypes.c_double * 3),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("n_sensors", ctypes.c_int32),
                ("sensor_node", _c_i32p), ("data", _c_dp), ("dirichlet_faces", ctypes.c_uint32),
                ("variant", ctypes.c_int32), ("regularization", ctypes.c_int32)]


class _RasParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32 * 4), ("overlap", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ilu_level", ctypes.c_int32)]


class _CoarseParams(ctypes.Structure):
    _fields_ = [("factor", ctypes.c_int32 * 4), ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("restrict_kind", ctypes.c_int32), ("p", ctypes.c_int32 * 4), ("overlap", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double)]


class _SolveParams(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("flexible", ctypes.c_int32), ("fixed_iters", ctypes.c_int32), ("graph", ctypes.c_int32)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_res_est", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("t_ms", ctypes.c_double * 4)]


_vp = ctypes.c_void_p
_sig = {
    "kkt_assemble": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_Alloc), _vp, ctypes.POINTER(_vp), _vp]),
    "kkt_rhs": (ctypes.c_int, [_vp, _c_dp, _vp, _vp]),
    "kkt_rhs_noalloc": (ctypes.c_int, [_vp, _c_dp, _vp, _vp]),
    "kkt_matvec": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "kkt_size": (ctypes.c_int64, [_vp]),
    "ras_setup": (ctypes.c_int, [_vp, ctypes.POINTER(_RasParams), _vp, ctypes.POINTER(_vp)]),
    "ras_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ras_num_subdomains": (ctypes.c_int, [_vp]),
    "ras_query_boxes": (ctypes.c_int, [_vp, _c_i32p]),
    "ras_factor_bytes": (ctypes.c_int64, [_vp]),
    "ras_query_apply_rows": (ctypes.c_int32, [_vp]),
    "ras_subdomain_blocks": (ctypes.c_int64, [_vp, ctypes.c_int32]),
    "ras_export_factors_csr": (ctypes.c_int, [_vp, ctypes.c_int32, _c_i32p, _c_i32p, _c_dp]),
    "ras_export_factors": (ctypes.c_int, [_vp, ctypes.c_int32, _c_dp]),
    "coarse_setup": (ctypes.c_int, [_vp, ctypes.POINTER(_CoarseParams), _vp, ctypes.POINTER(_vp)]),
    "coarse_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "coarse_apply_multi": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp]),
    "kkt_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_SolveParams), _vp, _vp, _vp,
                                 ctypes.POINTER(_Stats)]),
    "kkt_solve_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                       ctypes.POINTER(_SolveParams), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp,
                                       ctypes.POINTER(_Stats)]),
    "kkt_server_create": (ctypes.c_int, [ctypes.POINTER(_ServerParams), ctypes.POINTER(_Alloc), _vp,
                                         ctypes.POINTER(_vp)]),
    "kkt_server_submit": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_dp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "kkt_server_step": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "kkt_server_poll": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.POINTER(_Stats)]),
    "kkt_server_destroy": (None, [_vp]),
    "kkt_op_destroy": (None, [_vp]),
    "ras_destroy": (None, [_vp]),
    "coarse_destroy": (None, [_vp]),
    "kkt_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)

# Handles are released before the interpreter shuts down: releasing them later
# would call the allocator callbacks into a finalising interpreter.
_live = []
_finalizing = False


def _track(obj):
    if len(_live) > 256:
        _live[:] = [r for r in _live if r() is not None]
    _live.append(weakref.ref(obj))


@atexit.register
def _release_all():
    global _finalizing
    for ref in reversed(_live):
        obj = ref()
        if obj is not None:
            obj.close()
    _finalizing = True


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise StkktError(rc, _lib.kkt_last_error().decode(errors="replace"))
    return rc


def _torch():
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class TorchAllocator:
    """Device memory for the library's handles, from torch's caching allocator."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, ctx):
            self.live.pop(ptr, None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = _Alloc(self._alloc_cb, self._free_cb, None)

    @property
    def bytes_live(self):
        return sum(t.numel() for t in self.live.values())


def _problem_struct(prob):
    a = np.ascontiguousarray(prob.a_elem, dtype=np.float64)
    sn = np.ascontiguousarray(prob.sensor_node, dtype=np.int32)
    data = np.ascontiguousarray(prob.data, dtype=np.float64)
    p = _Problem()
    p.n = (ctypes.c_int32 * 3)(*prob.n)
    p.nt = int(prob.M)
    p.len = (ctypes.c_double * 3)(*prob.length)
    p.T = float(prob.T)
    p.a_elem = a.ctypes.data_as(_c_dp)
    p.v = (ctypes.c_double * 3)(*prob.v)
    p.beta1 = float(prob.beta1)
    p.beta2 = float(prob.beta2)
    p.n_sensors = int(sn.size)
    p.sensor_node = sn.ctypes.data_as(_c_i32p)
    p.data = data.ctypes.data_as(_c_dp)
    p.dirichlet_faces = int(prob.dirichlet_faces)
    p.variant = int(prob.variant)
    p.regularization = int(getattr(prob, "reg", 0))
    return p, (a, sn, data)


class KKTOperator:
    """Handle of F_h (and the right-hand side b of the given data)."""

    def __init__(self, prob, stream=None, allocator=None):
        torch = _torch()
        self.prob = prob
        self.alloc = allocator if allocator is not None else TorchAllocator()
        p, keep = _problem_struct(prob)
        self.n = int(3 * (prob.M + 1) * np.prod([k + 1 for k in prob.n]))
        self.b = torch.empty(self.n, dtype=torch.float64, device=self.alloc.device)
        h = ctypes.c_void_p()
        _check(_lib.kkt_assemble(ctypes.byref(p), ctypes.byref(self.alloc.struct), _stream(stream),
                                 ctypes.byref(h), _ptr(self.b)))
        self.handle = h
        _track(self)
        assert _lib.kkt_size(h) == self.n

    def rhs(self, data, out=None, stream=None):
        torch = _torch()
        d = np.ascontiguousarray(data, dtype=np.float64)
        out = torch.empty(self.n, dtype=torch.float64, device=self.alloc.device) if out is None else out
        _check(_lib.kkt_rhs(self.handle, d.ctypes.data_as(_c_dp), _stream(stream), _ptr(out)))
        return out

    def rhs_noalloc(self, data, out, stream=None):
        """kkt_rhs_noalloc: b for new sensor data into `out`, staged in the
        library's static device array (no device allocation)."""
        d = np.ascontiguousarray(data, dtype=np.float64)
        _check(_lib.kkt_rhs_noalloc(self.handle, d.ctypes.data_as(_c_dp), _stream(stream), _ptr(out)))
        return out

    def matvec(self, x, y=None, stream=None):
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        _check(_lib.kkt_matvec(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def close(self):
        if getattr(self, "handle", None):
            _lib.kkt_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if not _finalizing:
            self.close()


class RAS:
    """One-level space-time restricted additive Schwarz preconditioner."""

    def __init__(self, op: KKTOperator, parts, overlap, precision=F64, stream=None, ilu_level=0):
        self.op = op
        self.alloc = op.alloc   # the library frees this handle's memory through these callbacks
        rp = _RasParams()
        rp.p = (ctypes.c_int32 * 4)(*parts)
        rp.overlap = int(overlap)
        rp.precision = int(precision)
        rp.ilu_level = int(ilu_level)
        self.ilu_level = int(ilu_level)
        h = ctypes.c_void_p()
        _check(_lib.ras_setup(op.handle, ctypes.byref(rp), _stream(stream), ctypes.byref(h)))
        self.handle = h
        _track(self)
        self.nsub = _lib.ras_num_subdomains(h)

    def apply(self, r, z=None, stream=None):
        torch = _torch()
        z = torch.empty_like(r) if z is None else z
        _check(_lib.ras_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def boxes(self):
        out = np.zeros((self.nsub, 16), dtype=np.int32)
        _check(_lib.ras_query_boxes(self.handle, out.ctypes.data_as(_c_i32p)))
        return out

    @property
    def factor_bytes(self):
        return int(_lib.ras_factor_bytes(self.handle))

    def export_factors_csr(self, sub):
        """(indptr, indices, blocks[n, 3, 3]) of one subdomain in natural row order
        (L left of the diagonal, inv(U_rr) on it, U right of it), any ILU level."""
        n = int(_lib.ras_subdomain_blocks(self.handle, int(sub)))
        if n < 0:
            raise ValueError("bad subdomain")
        b = self.boxes()[sub]
        rows = int(np.prod(b[12:16] - b[8:12]))
        indptr = np.zeros(rows + 1, dtype=np.int32)
        indices = np.zeros(n, dtype=np.int32)
        blocks = np.zeros((n, 3, 3))
        _check(_lib.ras_export_factors_csr(self.handle, int(sub), indptr.ctypes.data_as(_c_i32p),
                                           indices.ctypes.data_as(_c_i32p), blocks.ctypes.data_as(_c_dp)))
        return indptr, indices, blocks

    @property
    def apply_rows(self):
        """Rows per phase of the sweep kernel: 256 or 64 (LDS ring), 0 (local vector in global memory)."""
        return int(_lib.ras_query_apply_rows(self.handle))

    def export_factors(self, sub):
        b = self.boxes()[sub]
        dims = b[12:16] - b[8:12]
        out = np.zeros((int(np.prod(dims)), 81, 3, 3))
        _check(_lib.ras_export_factors(self.handle, int(sub), out.ctypes.data_as(_c_dp)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.ras_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if not _finalizing:
            self.close()


class Coarse:
    """Coarse space-time level of the two-level preconditioner.

    factor: coarsening in (x, y, z, t).  method COARSE_LU (default): exact
    block elimination in time; COARSE_GMRES_RAS: F_c^{-1} is at most `maxit`
    steps of GMRES (relative tolerance `rtol`) from zero with the coarse mesh's
    RAS (parts, overlap), as in the paper's experiments.
    """

    def __init__(self, op: KKTOperator, factor, parts=(1, 1, 1, 1), overlap=1, maxit=4, rtol=0.1, precision=F64,
                 restrict=RESTRICT_TRANSPOSE, method=COARSE_LU, stream=None):
        self.op = op
        self.alloc = op.alloc
        cp = _CoarseParams()
        cp.factor = (ctypes.c_int32 * 4)(*factor)
        cp.method = int(method)
        cp.precision = int(precision)
        cp.restrict_kind = int(restrict)
        cp.p = (ctypes.c_int32 * 4)(*parts)
        cp.overlap = int(overlap)
        cp.maxit = int(maxit)
        cp.rtol = float(rtol)
        h = ctypes.c_void_p()
        _check(_lib.coarse_setup(op.handle, ctypes.byref(cp), _stream(stream), ctypes.byref(h)))
        self.handle = h
        _track(self)

    def apply(self, x, y=None, stream=None):
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        _check(_lib.coarse_apply(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def apply_multi(self, x, y=None, stream=None):
        """y[i] = apply(x[i]) for the rows of the 2-D float64 device tensors x, y
        (q rows of the fine size, unit stride within a row)."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        if x.dim() != 2 or y.shape != x.shape or x.stride(1) != 1 or y.stride(1) != 1:
            raise ValueError("apply_multi: x and y must be (q, n) tensors with unit stride in a row")
        for t in (x, y):
            if not t.is_cuda or t.dtype != torch.float64:
                raise TypeError("apply_multi: expected float64 CUDA tensors")
        _check(_lib.coarse_apply_multi(self.handle, int(x.shape[0]), ctypes.c_void_p(x.data_ptr()),
                                       int(x.stride(0)), ctypes.c_void_p(y.data_ptr()), int(y.stride(0)),
                                       _stream(stream)))
        return y

    def close(self):
        if getattr(self, "handle", None):
            _lib.coarse_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if not _finalizing:
            self.close()


@dataclass
class SolveStats:
    iters: int
    restarts: int
    converged: bool
    status: int
    rel_res_est: float
    rel_res_true: float
    bnorm: float
    ms: float


def solve(op: KKTOperator, ras: RAS, b=None, x=None, *, coarse: Coarse = None, restart=30, rtol=1e-6,
          maxit=10000, flexible=False, fixed_iters=0, stream=None, raise_on_fail=True):
    """Solve F_h x = b with right-preconditioned (F)GMRES; x holds x0 on entry."""
    torch = _torch()
    b = op.b if b is None else b
    x = torch.zeros_like(b) if x is None else x
    sp = _SolveParams(int(restart), int(maxit), float(rtol), int(bool(flexible)), int(fixed_iters))
    st = _Stats()
    rc = _lib.kkt_solve(op.handle, ras.handle, coarse.handle if coarse is not None else None, ctypes.byref(sp),
                        _ptr(b), _ptr(x), _stream(stream), ctypes.byref(st))
    if raise_on_fail:
        _check(rc, allow=(OK, NOT_CONVERGED))
    return x, SolveStats(st.iters, st.restarts, bool(st.converged), st.status, st.rel_res_est, st.rel_res_true,
                         st.bnorm, st.t_ms[0])


def _to_stats(st):
    return SolveStats(st.iters, st.restarts, bool(st.converged), st.status, st.rel_res_est, st.rel_res_true,
                      st.bnorm, st.t_ms[0])


def solve_batch(ops, pres, bs=None, xs=None, *, restart=30, rtol=1e-6, maxit=10000, fixed_iters=0, stream=None,
                raise_on_fail=True, graph=True):
    """Solve F_i x_i = b_i for every instance together (batched FGMRES); x_i holds x0 on entry.

    graph: replay each cycle's Arnoldi steps from captured HIP graphs (rotations
    and convergence flags on the device) instead of checking on the host every step."""
    torch = _torch()
    count = len(ops)
    if count == 0 or len(pres) != count:
        raise ValueError("solve_batch: need one preconditioner per operator")
    bs = [op.b for op in ops] if bs is None else list(bs)
    xs = [torch.zeros_like(b) for b in bs] if xs is None else list(xs)
    arr = _vp * count
    h_ops = arr(*[op.handle for op in ops])
    h_ras = arr(*[p.handle for p in pres])
    h_b = arr(*[_ptr(b) for b in bs])
    h_x = arr(*[_ptr(x) for x in xs])
    sp = _SolveParams(int(restart), int(maxit), float(rtol), 1, int(fixed_iters), 1 if graph else 0)
    st = (_Stats * count)()
    rc = _lib.kkt_solve_batch(count, h_ops, h_ras, ctypes.byref(sp), h_b, h_x, _stream(stream), st)
    if raise_on_fail:
        _check(rc, allow=(OK, NOT_CONVERGED))
    return xs, [_to_stats(st[i]) for i in range(count)]


class Server:
    """Request server: continuous batching of source-identification solves.

    submit() queues a request (operator, preconditioner, optional coarse
    level, new sensor data); step() admits what fits, advances every running
    request by one FGMRES cycle and retires the finished ones; poll() returns
    (x, stats) once a request is done.  stats.ms is the submit-to-result
    latency.
    """

    def __init__(self, restart=50, maxit=10000, rtol=1e-6, device_bytes=8 << 30, max_active=64, stream=None,
                 allocator=None):
        self.alloc = allocator if allocator is not None else TorchAllocator()
        self.stream = stream
        p = _ServerParams(int(restart), int(maxit), float(rtol), int(device_bytes), int(max_active))
        h = ctypes.c_void_p()
        _check(_lib.kkt_server_create(ctypes.byref(p), ctypes.byref(self.alloc.struct), _stream(stream),
                                      ctypes.byref(h)))
        self.handle = h
        _track(self)
        self._out = {}
        self._keep = {}

    def submit(self, op, pre, data, coarse=None):
        torch = _torch()
        d = np.ascontiguousarray(data, dtype=np.float64)
        x = torch.empty(op.n, dtype=torch.float64, device=self.alloc.device)
        t = ctypes.c_int64()
        _check(_lib.kkt_server_submit(self.handle, op.handle, pre.handle, coarse.handle if coarse is not None else None,
                                      d.ctypes.data_as(_c_dp), _ptr(x), ctypes.byref(t)))
        self._out[t.value] = x
        self._keep[t.value] = (op, pre, coarse)   # handles must outlive the request
        return t.value

    def step(self):
        r, q = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.kkt_server_step(self.handle, ctypes.byref(r), ctypes.byref(q)))
        return r.value, q.value

    def poll(self, ticket):
        st = _Stats()
        rc = _lib.kkt_server_poll(self.handle, int(ticket), ctypes.byref(st))
        _check(rc, allow=(0, 1))
        if rc == 0:
            return None
        self._keep.pop(ticket, None)
        return self._out.pop(ticket), _to_stats(st)

    def close(self):
        if getattr(self, "handle", None):
            _lib.kkt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if not _finalizing:
            self.close()
