"""ctypes binding of libpdlpb.so (include/pdlpb.h).

Argument marshalling only: every function forwards to the C entry point of
the same name, and the ``Context`` class strings those calls together.  Host
arrays are numpy; device arrays may be torch tensors on the context's GPU
(passed by ``data_ptr()`` with ``mem=MEM_DEVICE``).  No computation of the
solver happens here, and there is no fallback: if the shared library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import importlib.util
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdlpb.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
STATUS_RUNNING, STATUS_OPTIMAL, STATUS_ITERATION_LIMIT = 0, 1, 2
STATUS_INFEASIBLE_BOUNDS, STATUS_NUMERICAL_ERROR, STATUS_INVALID_INPUT = 3, 4, 5
STATUS_PRIMAL_INFEASIBLE, STATUS_DUAL_INFEASIBLE = 6, 7
BASE, SET_LO, SET_HI, OBJ_UNIT = 0, 1, 2, 3
FP64, MIXED32 = 0, 1
RESTART_PER_LP, RESTART_BATCH_AVG = 0, 1
WARM_NONE, WARM_SHARED, WARM_PER_LP, WARM_BASE = 0, 1, 2, 3
MEM_HOST, MEM_DEVICE = 0, 1
NOALLOC_SCRATCH_BYTES = 32 << 20   # PDLPB_NOALLOC_SCRATCH_BYTES: staging of pdlpb_get_batch_noalloc

STATUS_NAMES = {0: "RUNNING", 1: "OPTIMAL", 2: "ITERATION_LIMIT", 3: "INFEASIBLE_BOUNDS",
                4: "NUMERICAL_ERROR", 5: "INVALID_INPUT", 6: "PRIMAL_INFEASIBLE",
                7: "DUAL_INFEASIBLE"}

EXPORTED = ["pdlpb_default_options", "pdlpb_create", "pdlpb_set_batch", "pdlpb_solve",
            "pdlpb_get", "pdlpb_get_batch", "pdlpb_get_trace", "pdlpb_get_dual_objective",
            "pdlpb_obbt_tighten", "pdlpb_branch_scores", "pdlpb_set_tile",
            "pdlpb_get_step_size", "pdlpb_get_scaling", "pdlpb_set_base_warm",
            "pdlpb_serve_begin", "pdlpb_submit",
            "pdlpb_serve_launch", "pdlpb_serve_wait", "pdlpb_poll", "pdlpb_result",
            "pdlpb_release",
            "pdlpb_set_kernel_timing", "pdlpb_kernel_times", "pdlpb_kernel_columns",
            "pdlpb_device_bytes", "pdlpb_graph_captures", "pdlpb_estimate_batch",
            "pdlpb_get_batch_noalloc", "pdlpb_serve_ready", "pdlpb_serve_footprint",
            "pdlpb_serve_trim", "pdlpb_set_result_buffers",
            "pdlpb_destroy", "pdlpb_last_error"]


class Delta(C.Structure):
    _fields_ = [("kind", C.c_int32), ("var", C.c_int32), ("value", C.c_double)]


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("precision", C.c_int32),
                ("restart_scope", C.c_int32), ("eval_every", C.c_int32),
                ("beta_sufficient", C.c_double), ("beta_necessary", C.c_double),
                ("beta_artificial", C.c_double), ("theta", C.c_double),
                ("step_size", C.c_double), ("cross_sign", C.c_double),
                ("infeas_tol", C.c_double),
                ("pw_ratio", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
                ("max_batch", C.c_int32), ("use_graphs", C.c_int32),
                ("tile_lanes", C.c_int32), ("tile_vec", C.c_int32),
                ("autotune", C.c_int32), ("shared_start", C.c_int32),
                ("dual_tol", C.c_double), ("max_blocks", C.c_int32),
                ("scaling", C.c_int32), ("tail_cols", C.c_int32), ("stop_every", C.c_int32),
                ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p),
                ("alloc_user", C.c_void_p)]


class PdlpbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pdlpb error {code}: {msg}")
        self.code = code


def _share_torch_runtime():
    """When PyTorch is installed, load the HIP runtime it bundles before this
    library, so that the library binds to it and the process holds one runtime
    whichever of the two is used first: with two runtimes in one process the
    one that starts second finds no GPU."""
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return
    libdir = os.path.join(os.path.dirname(spec.origin), "lib")
    for name in ("libhsa-runtime64.so", "libamdhip64.so"):
        path = os.path.join(libdir, name)
        if os.path.exists(path):
            C.CDLL(path, mode=C.RTLD_GLOBAL)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    _share_torch_runtime()
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    d, i32, i64 = C.c_double, C.c_int32, C.c_int64
    dp, i32p, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "pdlpb_default_options": (None, [C.POINTER(Options)]),
        "pdlpb_create": (C.c_int, [C.POINTER(P), i32, i32, i64, P, P, P, P, P, P, P, P,
                                    C.POINTER(Options)]),
        "pdlpb_set_batch": (C.c_int, [P, i32, P, P, P, P, i32, i32]),
        "pdlpb_solve": (C.c_int, [P, d, i64]),
        "pdlpb_get": (C.c_int, [P, i32, P, P, i32p, dp, dp, i64p, i32]),
        "pdlpb_get_batch": (C.c_int, [P, P, P, i32p, dp, dp, i64p, i32]),
        "pdlpb_get_batch_noalloc": (C.c_int, [P, P, P, i32p, dp, dp, i64p, i32]),
        "pdlpb_set_result_buffers": (C.c_int, [P, P, P, i32]),
        "pdlpb_get_trace": (C.c_int, [P, i32, dp, dp, dp, i32p, i32p, i32]),
        "pdlpb_get_dual_objective": (C.c_int, [P, dp]),
        "pdlpb_obbt_tighten": (C.c_int, [P, d, d, dp, dp, i32p, i32p]),
        "pdlpb_branch_scores": (C.c_int, [P, d, d, dp, dp]),
        "pdlpb_set_tile": (C.c_int, [P, i32, i32]),
        "pdlpb_set_base_warm": (C.c_int, [P, P, P, d, i32]),
        "pdlpb_serve_begin": (C.c_int, [P, i32]),
        "pdlpb_submit": (C.c_int, [P, i32, P, i32, d, i64, i32, i64p]),
        "pdlpb_serve_launch": (C.c_int, [P]),
        "pdlpb_serve_wait": (C.c_int, [P, i32p, i32p]),
        "pdlpb_poll": (C.c_int, [P, i64p, i32, i32p]),
        "pdlpb_result": (C.c_int, [P, i64, P, P, i32p, dp, dp, i64p, i32]),
        "pdlpb_release": (C.c_int, [P, i64]),
        "pdlpb_serve_ready": (C.c_int, [P]),
        "pdlpb_serve_footprint": (C.c_int, [P, i32, i64p]),
        "pdlpb_serve_trim": (C.c_int, [P]),
        "pdlpb_get_step_size": (C.c_int, [P, dp, dp]),
        "pdlpb_get_scaling": (C.c_int, [P, dp, dp]),
        "pdlpb_set_kernel_timing": (C.c_int, [P, i32]),
        "pdlpb_kernel_times": (C.c_int, [P, i64p, dp]),
        "pdlpb_kernel_columns": (C.c_int, [P, i64p]),
        "pdlpb_device_bytes": (C.c_int64, [P]),
        "pdlpb_graph_captures": (C.c_int64, [P]),
        "pdlpb_estimate_batch": (C.c_int, [P, i32p, i32, i32, dp, i32p]),
        "pdlpb_destroy": (None, [P]),
        "pdlpb_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# C entry points under their own names
pdlpb_default_options = lib.pdlpb_default_options
pdlpb_create = lib.pdlpb_create
pdlpb_set_batch = lib.pdlpb_set_batch
pdlpb_solve = lib.pdlpb_solve
pdlpb_get = lib.pdlpb_get
pdlpb_get_batch = lib.pdlpb_get_batch
pdlpb_get_batch_noalloc = lib.pdlpb_get_batch_noalloc
pdlpb_get_trace = lib.pdlpb_get_trace
pdlpb_get_dual_objective = lib.pdlpb_get_dual_objective
pdlpb_obbt_tighten = lib.pdlpb_obbt_tighten
pdlpb_branch_scores = lib.pdlpb_branch_scores
pdlpb_set_tile = lib.pdlpb_set_tile
pdlpb_set_base_warm = lib.pdlpb_set_base_warm
pdlpb_serve_begin = lib.pdlpb_serve_begin
pdlpb_submit = lib.pdlpb_submit
pdlpb_serve_launch = lib.pdlpb_serve_launch
pdlpb_serve_wait = lib.pdlpb_serve_wait
pdlpb_poll = lib.pdlpb_poll
pdlpb_result = lib.pdlpb_result
pdlpb_release = lib.pdlpb_release
pdlpb_serve_ready = lib.pdlpb_serve_ready
pdlpb_serve_footprint = lib.pdlpb_serve_footprint
pdlpb_serve_trim = lib.pdlpb_serve_trim
pdlpb_get_step_size = lib.pdlpb_get_step_size
pdlpb_get_scaling = lib.pdlpb_get_scaling
pdlpb_set_kernel_timing = lib.pdlpb_set_kernel_timing
pdlpb_kernel_times = lib.pdlpb_kernel_times
pdlpb_kernel_columns = lib.pdlpb_kernel_columns
pdlpb_device_bytes = lib.pdlpb_device_bytes
pdlpb_graph_captures = lib.pdlpb_graph_captures
pdlpb_estimate_batch = lib.pdlpb_estimate_batch
pdlpb_destroy = lib.pdlpb_destroy
pdlpb_last_error = lib.pdlpb_last_error


# device-memory callbacks of pdlpb_options (dev_alloc, dev_free)
DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class TorchAllocator:
    """pdlpb_options.dev_alloc / dev_free backed by PyTorch's caching allocator
    on one device.  Keep the object alive as long as the context (Context does
    when it is passed as ``allocator=``).  Counts requests and returns."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = int(device)
        self.live = {}
        self.allocs = 0
        self.frees = 0

        def _alloc(nbytes, _user):
            try:
                p = self._torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device)
            except RuntimeError:
                return None
            self.live[int(p)] = int(nbytes)
            self.allocs += 1
            return int(p)

        def _free(ptr, nbytes, _user):
            self.live.pop(int(ptr), None)
            self.frees += 1
            self._torch.cuda.caching_allocator_delete(int(ptr))

        self.c_alloc = DEV_ALLOC(_alloc)
        self.c_free = DEV_FREE(_free)

    def install(self, opts: Options) -> None:
        opts.dev_alloc = C.cast(self.c_alloc, C.c_void_p).value
        opts.dev_free = C.cast(self.c_free, C.c_void_p).value
        opts.alloc_user = None


def default_options(**kw) -> Options:
    o = Options()
    lib.pdlpb_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(a) -> Optional[int]:
    """Address of a numpy array (host) or a torch tensor (device); None for None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    raise TypeError(f"unsupported buffer type {type(a)}")


def _device_f64(name, t, count, device):
    """Check a device tensor the library reads or writes through its address:
    contiguous float64 on `device` with at least `count` entries."""
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError(f"{name} must be a device tensor")
    if str(t.dtype) != "torch.float64" or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if t.device.index != device:
        raise ValueError(f"{name} is on device {t.device.index}, the context on {device}")
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} entries, fewer than {count}")


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} entries, got {a.size}")
    return a


def deltas_array(kinds, vars_, values) -> np.ndarray:
    d = np.zeros(len(kinds), dtype=[("kind", "<i4"), ("var", "<i4"), ("value", "<f8")])
    d["kind"], d["var"], d["value"] = kinds, vars_, values
    return d


class Context:
    """One constraint matrix on the GPU and its current batch of LPs."""

    def __init__(self, m, n, row_ptr, col_idx, val, c, b, sense, l, u,
                 options: Optional[Options] = None, allocator=None, **opt_kw):
        opts = options if options is not None else default_options(**opt_kw)
        self._allocator = allocator          # its callbacks must outlive the context
        if allocator is not None:
            allocator.install(opts)
        self.m, self.n = int(m), int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        vv = _f64(val)
        cc, bb = _f64(c, self.n), _f64(b, self.m)
        ss = np.ascontiguousarray(np.frombuffer(bytes(sense), dtype=np.uint8)
                                  if isinstance(sense, (bytes, bytearray)) else sense,
                                  dtype=np.uint8)
        ll, uu = _f64(l, self.n), _f64(u, self.n)
        # the library reads these by address: m + 1 row pointers, nnz = row_ptr[m]
        # entries of col_idx and val, m row senses
        if rp.size != self.m + 1:
            raise ValueError(f"row_ptr needs m + 1 = {self.m + 1} entries, got {rp.size}")
        nnz = int(rp[-1])
        if nnz > 0 and (ci.size < nnz or vv.size < nnz):
            raise ValueError(f"col_idx and val need row_ptr[m] = {nnz} entries, got "
                             f"{ci.size} and {vv.size}")
        if ss.size != self.m:
            raise ValueError(f"sense needs m = {self.m} entries, got {ss.size}")
        h = C.c_void_p()
        rc = lib.pdlpb_create(C.byref(h), self.m, self.n, nnz,
                              _ptr(rp), _ptr(ci), _ptr(vv), _ptr(cc), _ptr(bb), _ptr(ss),
                              _ptr(ll), _ptr(uu), C.byref(opts))
        if rc != OK:
            raise PdlpbError(rc, lib.pdlpb_last_error(None).decode())
        self._h = h
        self.options = opts
        self.B = 0

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.m, inst.n, inst.row_ptr, inst.col_idx, inst.val, inst.c, inst.b,
                   inst.sense, inst.l, inst.u, **kw)

    def _check(self, rc):
        if rc != OK:
            raise PdlpbError(rc, lib.pdlpb_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.pdlpb_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def step_size(self):
        eta, na = C.c_double(), C.c_double()
        self._check(lib.pdlpb_get_step_size(self._h, C.byref(eta), C.byref(na)))
        return eta.value, na.value

    def scaling(self):
        dr, dc = np.empty(self.m), np.empty(self.n)
        self._check(lib.pdlpb_get_scaling(self._h, dr.ctypes.data_as(C.POINTER(C.c_double)),
                                          dc.ctypes.data_as(C.POINTER(C.c_double))))
        return dr, dc

    @property
    def device_bytes(self) -> int:
        return int(lib.pdlpb_device_bytes(self._h))

    @property
    def graph_captures(self) -> int:
        return int(lib.pdlpb_graph_captures(self._h))

    def set_batch(self, deltas, x_warm=None, y_warm=None, w_warm=None,
                  warm_mode: Optional[int] = None, mem: int = MEM_HOST):
        """B LPs, one change each (deltas: B records); warm start from one
        point (x_warm n, y_warm m) or one per LP (B*n, B*m), inferred from the
        size of x_warm unless warm_mode says; w_warm: B primal weights.  With
        mem = MEM_DEVICE every array is a device tensor on the context's
        device (deltas: any dtype, B 16-byte records)."""
        if mem == MEM_HOST:
            dd = np.ascontiguousarray(deltas)
            if dd.dtype.itemsize != 16:
                raise ValueError("deltas must have the 16-byte (kind, var, value) layout")
            B = len(dd)
        else:
            dd = deltas
            if not (hasattr(dd, "is_cuda") and dd.is_cuda and dd.is_contiguous()):
                raise TypeError("deltas must be a contiguous device tensor")
            if dd.numel() * dd.element_size() % 16:
                raise ValueError("deltas must hold whole 16-byte (kind, var, value) records")
            B = dd.numel() * dd.element_size() // 16
        if warm_mode is None:
            if x_warm is None:
                warm_mode = WARM_NONE
            else:
                nx = x_warm.size if hasattr(x_warm, "size") and not callable(x_warm.size) \
                    else x_warm.numel()
                warm_mode = WARM_SHARED if nx == self.n else WARM_PER_LP
        per = B if warm_mode == WARM_PER_LP else 1
        warm = warm_mode in (WARM_SHARED, WARM_PER_LP)
        if mem == MEM_HOST:
            xw = _f64(x_warm, per * self.n) if warm and x_warm is not None else None
            yw = _f64(y_warm, per * self.m) if warm and y_warm is not None else None
            ww = None if w_warm is None else _f64(w_warm, B)
        else:
            dev = int(self.options.device)
            if dd.device.index != dev:
                raise ValueError(f"deltas are on device {dd.device.index}, the context on {dev}")
            xw = x_warm if warm else None
            yw = y_warm if warm else None
            ww = w_warm
            if xw is not None:
                _device_f64("x_warm", xw, per * self.n, dev)
            if yw is not None:
                _device_f64("y_warm", yw, per * self.m, dev)
            if ww is not None:
                _device_f64("w_warm", ww, B, dev)
        self._check(lib.pdlpb_set_batch(self._h, B, _ptr(dd), _ptr(xw), _ptr(yw), _ptr(ww),
                                        int(warm_mode), int(mem)))
        self.B = B

    def solve(self, tol: float = 1e-4, max_iters: int = 100000):
        self._check(lib.pdlpb_solve(self._h, float(tol), int(max_iters)))

    def get(self, j: int, want_x=True, want_y=True):
        x = np.empty(self.n) if want_x else None
        y = np.empty(self.m) if want_y else None
        st = C.c_int32()
        kkt = (C.c_double * 4)()
        obj = C.c_double()
        it = C.c_int64()
        self._check(lib.pdlpb_get(self._h, int(j), _ptr(x), _ptr(y), C.byref(st), kkt,
                                  C.byref(obj), C.byref(it), MEM_HOST))
        return dict(x=x, y=y, status=st.value, kkt=list(kkt), obj=obj.value, iters=it.value)

    def set_result_buffers(self, X=None, Y=None, capacity: int = 0):
        """x~ and y~ of the following batches go straight into the device
        tensors X (capacity x n) and Y (capacity x m), FP64; get_batch into
        them then copies nothing.  No arguments: the context's own blocks.
        Both must be contiguous float64 tensors on the context's device with
        room for capacity LPs; the context keeps them alive until they are
        replaced or cleared."""
        capacity = int(capacity)
        for name, t, cols in (("X", X, self.n), ("Y", Y, self.m)):
            if t is not None:       # one of the two alone is refused by the library
                _device_f64(name, t, max(capacity, 0) * cols, int(self.options.device))
        self._check(lib.pdlpb_set_result_buffers(self._h, _ptr(X), _ptr(Y), capacity))
        self._result_buffers = None if X is None else (X, Y)

    def get_batch(self, want_x=True, want_y=True, X=None, Y=None, mem: int = MEM_HOST):
        B = self.B
        if mem == MEM_HOST:
            X = np.empty((B, self.n)) if want_x else None
            Y = np.empty((B, self.m)) if want_y else None
        else:
            if X is not None:
                _device_f64("X", X, B * self.n, int(self.options.device))
            if Y is not None:
                _device_f64("Y", Y, B * self.m, int(self.options.device))
        status = np.empty(B, dtype=np.int32)
        kkt = np.empty((B, 4))
        obj = np.empty(B)
        iters = np.empty(B, dtype=np.int64)
        self._check(lib.pdlpb_get_batch(
            self._h, _ptr(X), _ptr(Y), status.ctypes.data_as(C.POINTER(C.c_int32)),
            kkt.ctypes.data_as(C.POINTER(C.c_double)), obj.ctypes.data_as(C.POINTER(C.c_double)),
            iters.ctypes.data_as(C.POINTER(C.c_int64)), int(mem)))
        return dict(X=X, Y=Y, status=status, kkt=kkt, obj=obj, iters=iters)

    def get_trace(self, j: int, log_cap: int = 64):
        x = np.empty(self.n)
        y = np.empty(self.m)
        w = C.c_double()
        nr = C.c_int32()
        log = (C.c_int32 * log_cap)()
        self._check(lib.pdlpb_get_trace(self._h, int(j), x.ctypes.data_as(C.POINTER(C.c_double)),
                                        y.ctypes.data_as(C.POINTER(C.c_double)), C.byref(w),
                                        C.byref(nr), log, log_cap))
        k = min(nr.value, log_cap)
        return dict(x_iter=x, y_iter=y, w=w.value, restarts=nr.value, restart_log=list(log[:k]))

    def dual_objective(self) -> np.ndarray:
        d = np.empty(self.B)
        self._check(lib.pdlpb_get_dual_objective(self._h, d.ctypes.data_as(C.POINTER(C.c_double))))
        return d

    def obbt_tighten(self, eps: float = 1e-8, min_improve: float = 1e-4):
        lo = np.empty(self.n)
        hi = np.empty(self.n)
        nch = C.c_int32()
        inf = C.c_int32()
        self._check(lib.pdlpb_obbt_tighten(self._h, float(eps), float(min_improve),
                                           lo.ctypes.data_as(C.POINTER(C.c_double)),
                                           hi.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(nch), C.byref(inf)))
        return dict(lo=lo, hi=hi, changed=nch.value, infeasible=bool(inf.value))

    def branch_scores(self, parent_obj: float, mu: float = 1.0 / 6.0):
        gain = np.empty(self.B)
        score = np.empty(self.B)
        self._check(lib.pdlpb_branch_scores(self._h, float(parent_obj), float(mu),
                                            gain.ctypes.data_as(C.POINTER(C.c_double)),
                                            score.ctypes.data_as(C.POINTER(C.c_double))))
        return dict(gain=gain, score=score)

    # ---- serving (continuous batching) ----
    def set_base_warm(self, x, y, w: float):
        xx, yy = _f64(x, self.n), _f64(y, self.m)
        self._check(lib.pdlpb_set_base_warm(self._h, _ptr(xx), _ptr(yy), float(w), MEM_HOST))

    def serve_begin(self, result_capacity: int):
        self._check(lib.pdlpb_serve_begin(self._h, int(result_capacity)))

    def submit(self, deltas, warm_mode: int = WARM_NONE, tol: float = 1e-4,
               max_iters: int = 100000) -> range:
        dd = np.ascontiguousarray(deltas)
        if dd.dtype.itemsize != 16:
            raise ValueError("deltas must have the 16-byte (kind, var, value) layout")
        first = C.c_int64()
        self._check(lib.pdlpb_submit(self._h, len(dd), _ptr(dd), int(warm_mode), float(tol),
                                     int(max_iters), MEM_HOST, C.byref(first)))
        return range(first.value, first.value + len(dd))

    def serve_launch(self):
        self._check(lib.pdlpb_serve_launch(self._h))

    def serve_wait(self):
        nr, nq = C.c_int32(), C.c_int32()
        self._check(lib.pdlpb_serve_wait(self._h, C.byref(nr), C.byref(nq)))
        return nr.value, nq.value

    def poll(self, cap: int = 4096):
        ids = np.empty(cap, dtype=np.int64)
        cnt = C.c_int32()
        self._check(lib.pdlpb_poll(self._h, ids.ctypes.data_as(C.POINTER(C.c_int64)), cap,
                                   C.byref(cnt)))
        return ids[:cnt.value].tolist()

    def result(self, lp_id: int, want_x=True, want_y=True):
        x = np.empty(self.n) if want_x else None
        y = np.empty(self.m) if want_y else None
        st = C.c_int32()
        kkt = (C.c_double * 4)()
        obj = C.c_double()
        it = C.c_int64()
        self._check(lib.pdlpb_result(self._h, int(lp_id), _ptr(x), _ptr(y), C.byref(st), kkt,
                                     C.byref(obj), C.byref(it), MEM_HOST))
        return dict(x=x, y=y, status=st.value, kkt=list(kkt), obj=obj.value, iters=it.value)

    def release(self, lp_id: int):
        self._check(lib.pdlpb_release(self._h, int(lp_id)))

    def serve_ready(self) -> bool:
        rc = lib.pdlpb_serve_ready(self._h)
        if rc < 0:
            self._check(rc)
        return rc == 1

    def serve_footprint(self, extra: int = 0) -> int:
        b = C.c_int64()
        self._check(lib.pdlpb_serve_footprint(self._h, int(extra), C.byref(b)))
        return b.value

    def serve_trim(self):
        self._check(lib.pdlpb_serve_trim(self._h))

    def estimate_batch(self, widths, reps: int = 10):
        w = np.ascontiguousarray(widths, dtype=np.int32)
        ms = np.empty(w.size)
        best = C.c_int32()
        self._check(lib.pdlpb_estimate_batch(self._h, w.ctypes.data_as(C.POINTER(C.c_int32)),
                                             int(w.size), int(reps),
                                             ms.ctypes.data_as(C.POINTER(C.c_double)),
                                             C.byref(best)))
        self.B = 0
        return best.value, ms

    def set_tile(self, lanes: int = 0, vec: int = 0):
        self._check(lib.pdlpb_set_tile(self._h, int(lanes), int(vec)))

    def set_kernel_timing(self, enable: bool):
        self._check(lib.pdlpb_set_kernel_timing(self._h, int(bool(enable))))

    def kernel_times(self):
        cnt = (C.c_int64 * 5)()
        ms = (C.c_double * 5)()
        self._check(lib.pdlpb_kernel_times(self._h, cnt, ms))
        return list(cnt), list(ms)

    def kernel_columns(self):
        cols = (C.c_int64 * 5)()
        self._check(lib.pdlpb_kernel_columns(self._h, cols))
        return list(cols)
