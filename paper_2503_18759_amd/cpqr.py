"""Python binding of libcpqr (ctypes): argument marshalling only.

Every step of the decomposition runs in the HIP library.  torch is used for
device memory and streams.  If the compiled library is missing the functions
here raise immediately; there is no CPU fallback.

Tensors are dense with mode 1 fastest (column-major), as in the paper's
unfolding convention (Section 2.1).  A torch tensor of shape (I_1, ..., I_N)
is accepted if its strides are Fortran-ordered (stride of mode 1 is 1), or a
1-D contiguous tensor together with ``dims``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpqr.so")

# status codes (include/cpqr.h)
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ERANKDEF, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
TREES = {"none": 0, "standard": 1, "restructured": 2}
EXTRAP = {"off": 0, "paper": 1, "learned": 2}
MLP_FEATURES, MLP_HIDDEN = 8, 64
MLP_PARAMS = MLP_HIDDEN * MLP_FEATURES + 2 * MLP_HIDDEN + 1
PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
FLAG_EXPLICIT_FIT, FLAG_TIME_KERNELS, FLAG_NO_GRAPH, FLAG_DENSE_ZQR = 0x1, 0x2, 0x4, 0x8
FLAG_TIME_PHASES = 0x10
FLAG_CLOSING_PLAIN = 0x20
PHASES = ("ttm", "qr", "q0", "apply_q0", "other")
ZQR = ("stair", "dense")


class CpqrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


class _Tensor(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("dtype", ctypes.c_int), ("data", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_int), ("extrapolate", ctypes.c_int), ("prec", ctypes.c_int),
                ("iters", ctypes.c_int), ("tol", ctypes.c_double), ("alpha", ctypes.c_double),
                ("switch_delta", ctypes.c_double), ("fixed_beta", ctypes.c_double),
                ("init_factors", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("flags", ctypes.c_uint), ("mlp_weights", ctypes.POINTER(ctypes.c_float)),
                ("beta_schedule", ctypes.POINTER(ctypes.c_double)),
                ("seed", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("factors", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("lambda_", ctypes.POINTER(ctypes.c_double)),
                ("fit_history", ctypes.POINTER(ctypes.c_double)),
                ("sweep_orders", ctypes.POINTER(ctypes.c_int)),
                ("fit", ctypes.c_double), ("fit_explicit", ctypes.c_double),
                ("sweeps_done", ctypes.c_int), ("beta", ctypes.c_double),
                ("beta_sweep", ctypes.c_int), ("ttm_flops", ctypes.c_double),
                ("ttm_bytes", ctypes.c_double), ("seconds", ctypes.c_double),
                ("l1_ttm_seconds", ctypes.c_double), ("l1_ttm_launches", ctypes.c_int),
                ("l1_ttm_bytes", ctypes.c_double), ("l1_ttm_flops", ctypes.c_double),
                ("beta_learned", ctypes.c_double), ("learned_fallback_sweep", ctypes.c_int),
                ("phase_seconds", ctypes.c_double * 5),
                ("q_factors", ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))]


EXPORTS = ["cpqr_create", "cpqr_destroy", "cpqr_last_error", "cpqr_status_string",
           "cpqr_check_args", "cpqr_als_qr", "cpqr_session_create", "cpqr_session_sweeps",
           "cpqr_session_sync", "cpqr_session_result", "cpqr_session_destroy",
           "cpqr_schedule", "cpqr_ttm", "cpqr_qr", "cpqr_als_qr_batched",
           "cpqr_mlp_forward", "cpqr_mlp_grad", "cpqr_mlp_train", "cpqr_qr_noalloc",
           "cpqr_tune_cache_check", "cpqr_tune_cache_path"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcpqr.so; raises if it has not been built.

    torch is imported first: it brings its own HIP runtime (libamdhip64), and
    loading it before libcpqr makes the library bind to that same runtime, so
    device memory, streams and events are shared with torch."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcpqr.so not found at {path}: build it with "
                           "`python -m paper_2503_18759_amd.build` (no CPU fallback exists)")
    import torch  # noqa: F401  (see above)
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.cpqr_create.argtypes = [ctypes.POINTER(vp), i32, vp]
    L.cpqr_destroy.argtypes = [vp]
    L.cpqr_last_error.argtypes = [vp]
    L.cpqr_last_error.restype = ctypes.c_char_p
    L.cpqr_status_string.argtypes = [i32]
    L.cpqr_status_string.restype = ctypes.c_char_p
    L.cpqr_als_qr.argtypes = [vp, ctypes.POINTER(_Tensor), i32, ctypes.POINTER(_Options),
                              ctypes.POINTER(_Result)]
    L.cpqr_session_create.argtypes = [vp, ctypes.POINTER(_Tensor), i32, ctypes.POINTER(_Options),
                                      ctypes.POINTER(vp)]
    L.cpqr_session_sweeps.argtypes = [vp, i32]
    L.cpqr_session_sync.argtypes = [vp]
    L.cpqr_session_result.argtypes = [vp, ctypes.POINTER(_Result)]
    L.cpqr_session_destroy.argtypes = [vp]
    L.cpqr_check_args.argtypes = [ctypes.POINTER(_Tensor), i32, ctypes.POINTER(_Options)]
    L.cpqr_schedule.argtypes = [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32,
                                ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.cpqr_ttm.argtypes = [vp, i32, i32, ctypes.POINTER(i64), i32, i32, vp, vp, vp]
    L.cpqr_qr.argtypes = [vp, i64, i32, vp, vp, vp]
    L.cpqr_qr_noalloc.argtypes = [i64, i32, vp, vp, vp, vp]
    L.cpqr_als_qr_batched.argtypes = [vp, i32, ctypes.POINTER(_Tensor), ctypes.POINTER(i32),
                                      ctypes.POINTER(_Options), ctypes.POINTER(_Result)]
    L.cpqr_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
    L.cpqr_mlp_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    L.cpqr_mlp_train.argtypes = [vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, vp]
    L.cpqr_tune_cache_check.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(i32)]
    L.cpqr_tune_cache_path.argtypes = [vp, ctypes.c_char_p, ctypes.c_char_p, i32]
    for f in ("cpqr_create", "cpqr_destroy", "cpqr_check_args", "cpqr_als_qr", "cpqr_schedule",
              "cpqr_ttm", "cpqr_qr", "cpqr_qr_noalloc", "cpqr_session_create", "cpqr_session_sweeps",
              "cpqr_session_sync", "cpqr_session_result", "cpqr_session_destroy",
              "cpqr_tune_cache_check", "cpqr_tune_cache_path"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _status_name(s: int) -> str:
    try:
        return load_library().cpqr_status_string(s).decode()
    except Exception:
        return str(s)


class Handle:
    """Owns a cpqr_handle bound to a device and a HIP stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        L = load_library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self._h = ctypes.c_void_p()
        st = L.cpqr_create(ctypes.byref(self._h), int(device), ctypes.c_void_p(stream or 0))
        if st != OK:
            raise CpqrError(st, "cpqr_create failed")
        self.device = device

    def check(self, st: int):
        if st != OK:
            msg = load_library().cpqr_last_error(self._h).decode()
            raise CpqrError(st, msg)

    def close(self):
        if self._h:
            load_library().cpqr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: Dict[int, Handle] = {}


def default_handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def _dims_and_ptr(x, dims: Optional[Sequence[int]]):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a torch tensor on a HIP device")
    if x.dim() == 1:
        if dims is None:
            raise ValueError("a flat tensor needs dims")
        if not x.is_contiguous():
            raise ValueError("flat tensor must be contiguous")
        dims = [int(d) for d in dims]
        if int(np.prod(dims)) != x.numel():
            raise ValueError("dims do not match the number of elements")
    else:
        d = [int(v) for v in x.shape]
        if dims is not None and [int(v) for v in dims] != d:
            raise ValueError("dims do not match x.shape")
        exp, s = [], 1
        for v in d:
            exp.append(s)
            s *= v
        if list(x.stride()) != exp:
            raise ValueError("x must be column-major (mode 1 fastest); use to_device()")
        dims = d
    if x.dtype == torch.float64:
        dt = 0
    elif x.dtype == torch.float32:
        dt = 1
    else:
        raise TypeError("x must be float32 or float64")
    return dims, dt, x.data_ptr()


def to_device(X: np.ndarray, dtype=None, device: int = 0):
    """Copy a numpy tensor to the GPU as a flat column-major buffer; returns
    (flat torch tensor, dims)."""
    import torch
    arr = np.asarray(X)
    if dtype is not None:
        arr = arr.astype(dtype)
    flat = np.ascontiguousarray(arr.ravel(order="F"))
    return torch.from_numpy(flat).to(f"cuda:{device}"), [int(d) for d in arr.shape]


def _prepare(x, rank, init, iters, dims, tree, extrapolate, prec, tol, alpha, switch_delta,
             fixed_beta, explicit_fit, time_kernels, use_graph, mlp_weights=None,
             beta_schedule=None, zqr="stair", seed=0, time_phases=False, closing_plain=False):
    if zqr not in ZQR:
        raise ValueError(f"zqr must be one of {ZQR}")
    dims, dt, ptr = _dims_and_ptr(x, dims)
    N = len(dims)
    keep = {"dims_c": (ctypes.c_int64 * N)(*dims)}
    keep["ten"] = _Tensor(N, keep["dims_c"], dt, ctypes.c_void_p(ptr))
    if init is None:
        # the library draws seeded N(0,1) factors (cpqr_options.seed)
        keep["init_ptrs"] = None
    else:
        inits = [np.asfortranarray(np.asarray(a, dtype=np.float64)) for a in init]
        if len(inits) != N:
            raise ValueError("need one initial factor per mode")
        for k, a in enumerate(inits):
            if a.shape != (dims[k], rank):
                raise ValueError(f"init factor {k} must be {dims[k]} x {rank}")
        keep["inits"] = inits
        keep["init_ptrs"] = (ctypes.POINTER(ctypes.c_double) * N)(
            *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in inits])
    flags = (FLAG_EXPLICIT_FIT if explicit_fit else 0) | (FLAG_TIME_KERNELS if time_kernels else 0) \
        | (0 if use_graph else FLAG_NO_GRAPH) | (FLAG_DENSE_ZQR if zqr == "dense" else 0) \
        | (FLAG_TIME_PHASES if time_phases else 0) | (FLAG_CLOSING_PLAIN if closing_plain else 0)
    wptr = None
    if mlp_weights is not None:
        w = np.ascontiguousarray(np.asarray(mlp_weights, dtype=np.float32).reshape(-1))
        if w.size != MLP_PARAMS:
            raise ValueError(f"mlp_weights must hold {MLP_PARAMS} floats")
        keep["mlp_w"] = w
        wptr = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    sptr = None
    if beta_schedule is not None:
        sch = np.ascontiguousarray(np.asarray(beta_schedule, dtype=np.float64).reshape(-1))
        if sch.size != iters:
            raise ValueError("beta_schedule must hold one value per sweep")
        keep["sched"] = sch
        sptr = sch.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    keep["opts"] = _Options(TREES[tree], EXTRAP[extrapolate], PRECS[prec], int(iters), float(tol),
                            float(alpha), float(switch_delta), float(fixed_beta),
                            keep["init_ptrs"], flags, wptr, sptr, int(seed) & 0xFFFFFFFFFFFFFFFF)
    return dims, keep


def _result_buffers(dims, rank, iters):
    N = len(dims)
    outs = [np.zeros((dims[k], rank), order="F") for k in range(N)]
    lam = np.zeros(rank)
    fits = np.full(max(iters, 1), np.nan)
    orders = np.zeros((max(iters, 1), N), dtype=np.int32)
    qs = [np.zeros((dims[k], rank), order="F") for k in range(N)]
    res = _Result()
    res.factors = (ctypes.POINTER(ctypes.c_double) * N)(
        *[o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in outs])
    res.q_factors = (ctypes.POINTER(ctypes.c_double) * N)(
        *[q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for q in qs])
    res.lambda_ = lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    res.fit_history = fits.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    res.sweep_orders = orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    return res, (outs, lam, fits, orders, qs)


def _result_dict(res, bufs):
    outs, lam, fits, orders, qs = bufs
    n = res.sweeps_done
    return {
        "factors": outs, "lam": lam, "fits": fits[:n].copy(), "fit": res.fit,
        "fit_explicit": res.fit_explicit, "orders": orders[:n].tolist(), "beta": res.beta,
        "beta_sweep": res.beta_sweep, "sweeps": n, "seconds": res.seconds,
        "ttm_flops": res.ttm_flops, "ttm_bytes": res.ttm_bytes,
        "l1_ttm_seconds": res.l1_ttm_seconds, "l1_ttm_launches": res.l1_ttm_launches,
        "l1_ttm_bytes": res.l1_ttm_bytes, "l1_ttm_flops": res.l1_ttm_flops,
        "beta_learned": res.beta_learned, "learned_fallback_sweep": res.learned_fallback_sweep,
        "phase_seconds": dict(zip(PHASES, list(res.phase_seconds))), "Q": qs,
    }


def cp_als_qr(x, rank: int, init: Optional[Sequence[np.ndarray]], iters: int = 100, *,
              dims: Optional[Sequence[int]] = None, tree: str = "restructured",
              extrapolate: str = "off", prec: str = "fp32", tol: float = 0.0,
              alpha: float = 0.1, switch_delta: float = 0.03, fixed_beta: float = 0.0,
              explicit_fit: bool = False, time_kernels: bool = False, use_graph: bool = True,
              mlp_weights=None, beta_schedule=None, zqr: str = "stair", seed: int = 0,
              time_phases: bool = False, closing_plain: bool = False,
              handle: Optional[Handle] = None) -> Dict:
    """CP-ALS-QR / ALS-QR-BR(E) on the GPU (Algorithms 2 and 3).

    ``zqr="dense"`` factors Z_n by the two-level TSQR even where the
    one-workgroup staircase QR applies (for comparison).  ``init=None`` lets
    the library draw seeded N(0,1) initial factors from ``seed``.
    ``time_phases`` fills ``phase_seconds`` (TTM, QR, computation and
    application of Q0, other) with kernels launched one by one.
    ``closing_plain`` runs the last sweep without extrapolation.

    Returns a dict with factors (list of I_n x R float64 arrays), lam, fits
    (per-sweep fit history), fit, fit_explicit, orders, beta, beta_sweep,
    sweeps, seconds, ttm_flops, ttm_bytes and the level-1 TTM timing fields.
    """
    L = load_library()
    dims, keep = _prepare(x, rank, init, iters, dims, tree, extrapolate, prec, tol, alpha,
                          switch_delta, fixed_beta, explicit_fit, time_kernels, use_graph,
                          mlp_weights, beta_schedule, zqr, seed, time_phases, closing_plain)
    h = handle or default_handle(x.device.index or 0)
    res, bufs = _result_buffers(dims, rank, iters)
    st = L.cpqr_als_qr(h._h, ctypes.byref(keep["ten"]), int(rank), ctypes.byref(keep["opts"]),
                       ctypes.byref(res))
    h.check(st)
    return _result_dict(res, bufs)


def cp_als_qr_batched(xs: Sequence, ranks: Sequence[int], inits: Sequence[Sequence[np.ndarray]],
                      iters: int = 50, *, dims: Optional[Sequence[Sequence[int]]] = None,
                      tree: str = "restructured", extrapolate: str = "off", prec: str = "fp32",
                      alpha: float = 0.1, switch_delta: float = 0.03, fixed_beta=0.0,
                      explicit_fit: bool = False, beta_schedules=None, zqr: str = "stair",
                      handle: Optional[Handle] = None) -> List[Dict]:
    """Independent decompositions run together (cpqr_als_qr_batched): every
    sweep of the whole batch is one HIP graph of batched kernels.  Returns one
    result dict per problem (as :func:`cp_als_qr`).  ``alpha``,
    ``switch_delta`` and ``fixed_beta`` may be one value or one per problem."""
    L = load_library()
    count = len(xs)
    if not (len(ranks) == len(inits) == count) or count < 1:
        raise ValueError("xs, ranks and inits must have the same non-zero length")
    keeps, bufs = [], []
    tens = (_Tensor * count)()
    optv = (_Options * count)()
    resv = (_Result * count)()
    def each(v, t):
        return v[t] if isinstance(v, (list, tuple, np.ndarray)) else v

    for t in range(count):
        d, keep = _prepare(xs[t], ranks[t], inits[t], iters, dims[t] if dims else None, tree,
                           extrapolate, prec, 0.0, each(alpha, t), each(switch_delta, t),
                           each(fixed_beta, t), explicit_fit,
                           False, True, None,
                           beta_schedules[t] if beta_schedules is not None else None, zqr)
        keeps.append(keep)
        tens[t] = keep["ten"]
        optv[t] = keep["opts"]
        r, b = _result_buffers(d, ranks[t], iters)
        resv[t] = r
        bufs.append(b)
    rk = (ctypes.c_int32 * count)(*[int(r) for r in ranks])
    h = handle or default_handle(xs[0].device.index or 0)
    st = L.cpqr_als_qr_batched(h._h, count, tens, rk, optv, resv)
    h.check(st)
    return [_result_dict(resv[t], bufs[t]) for t in range(count)]


class Session:
    """Step-wise decomposition: ``Session(x, R, init, max_sweeps, ...)``,
    then ``sweeps(n)`` (asynchronous), ``sync()``, ``result()``, ``close()``."""

    def __init__(self, x, rank: int, init: Sequence[np.ndarray], max_sweeps: int, *,
                 dims: Optional[Sequence[int]] = None, tree: str = "restructured",
                 extrapolate: str = "off", prec: str = "fp32", tol: float = 0.0,
                 alpha: float = 0.1, switch_delta: float = 0.03, fixed_beta: float = 0.0,
                 explicit_fit: bool = False, time_kernels: bool = False,
                 use_graph: bool = True, mlp_weights=None, zqr: str = "stair",
                 closing_plain: bool = False, handle: Optional[Handle] = None):
        L = load_library()
        self._x = x
        self.rank = rank
        self.max_sweeps = max_sweeps
        self.dims, self._keep = _prepare(x, rank, init, max_sweeps, dims, tree, extrapolate, prec,
                                         tol, alpha, switch_delta, fixed_beta, explicit_fit,
                                         time_kernels, use_graph, mlp_weights, None, zqr,
                                         closing_plain=closing_plain)
        self.h = handle or default_handle(x.device.index or 0)
        self._s = ctypes.c_void_p()
        self.h.check(L.cpqr_session_create(self.h._h, ctypes.byref(self._keep["ten"]), int(rank),
                                           ctypes.byref(self._keep["opts"]), ctypes.byref(self._s)))

    def sweeps(self, n: int):
        self.h.check(load_library().cpqr_session_sweeps(self._s, int(n)))

    def sync(self):
        self.h.check(load_library().cpqr_session_sync(self._s))

    def result(self) -> Dict:
        res, bufs = _result_buffers(self.dims, self.rank, self.max_sweeps)
        self.h.check(load_library().cpqr_session_result(self._s, ctypes.byref(res)))
        return _result_dict(res, bufs)

    def close(self):
        if self._s:
            load_library().cpqr_session_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_args(dims: Sequence[int], rank: int, *, dtype: str = "f32", iters: int = 1,
               tree: str = "restructured", extrapolate: str = "off", prec: str = "fp32",
               tol: float = 0.0, alpha: float = 0.1, switch_delta: float = 0.03,
               fixed_beta: float = 0.0, init: Optional[Sequence[np.ndarray]] = None,
               data_ptr: int = 1, mlp_weights=None, flags: int = 0,
               raw: Optional[dict] = None) -> int:
    """Host-only argument checks of cpqr_als_qr (no device needed); returns
    the status code.  ``raw`` overrides fields with raw integers/None to
    exercise invalid inputs."""
    L = load_library()
    raw = raw or {}
    N = len(dims)
    dims_c = (ctypes.c_int64 * max(N, 1))(*[int(d) for d in dims])
    ten = _Tensor(raw.get("order", N), None if raw.get("null_dims") else dims_c,
                  {"f64": 0, "f32": 1}.get(dtype, 7) if "dtype" not in raw else raw["dtype"],
                  ctypes.c_void_p(data_ptr))
    if init is None:
        init = [np.zeros((max(int(d), 1), max(rank, 1))) for d in dims]
    keep = [np.asfortranarray(a, dtype=np.float64) for a in init]
    ptrs = (ctypes.POINTER(ctypes.c_double) * max(N, 1))(
        *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in keep])
    if raw.get("null_init_k") is not None:
        ptrs[raw["null_init_k"]] = ctypes.POINTER(ctypes.c_double)()
    wbuf = None
    if mlp_weights is not None:
        wbuf = np.zeros(MLP_PARAMS, dtype=np.float32) if mlp_weights is True else \
            np.ascontiguousarray(np.asarray(mlp_weights, dtype=np.float32).reshape(-1))
    opts = _Options(raw.get("tree", TREES.get(tree, 9)), raw.get("extrapolate", EXTRAP.get(extrapolate, 9)),
                    raw.get("prec", PRECS.get(prec, 9)), int(iters), float(tol), float(alpha),
                    float(switch_delta), float(fixed_beta),
                    None if raw.get("null_init") else ptrs, int(flags),
                    None if wbuf is None else wbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return int(L.cpqr_check_args(ctypes.byref(ten), int(rank), ctypes.byref(opts)))


def ttm(x, q, mode: int, *, dims: Optional[Sequence[int]] = None, prec: str = "fp32",
        handle: Optional[Handle] = None):
    """One mode-`mode` product X x_mode Q^T; returns a flat column-major
    torch tensor and its dims.  ``q`` is a torch (I_mode x R) tensor stored
    column-major (pass ``q.t().contiguous().t()`` or a flat Fortran buffer)."""
    import torch
    L = load_library()
    dims, dt, ptr = _dims_and_ptr(x, dims)
    N = len(dims)
    R = int(q.shape[1])
    if q.stride() != (1, q.shape[0]):
        raise ValueError("q must be column-major")
    out_dims = list(dims)
    out_dims[mode] = R
    out = torch.empty(int(np.prod(out_dims)), dtype=x.dtype, device=x.device)
    h = handle or default_handle(x.device.index or 0)
    dims_c = (ctypes.c_int64 * N)(*dims)
    st = L.cpqr_ttm(h._h, PRECS[prec], N, dims_c, int(mode), R, ctypes.c_void_p(ptr),
                    ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    h.check(st)
    return out, out_dims


def qr(A, handle: Optional[Handle] = None):
    """Householder QR of a column-major float64 M x R torch tensor."""
    import torch
    L = load_library()
    M, R = int(A.shape[0]), int(A.shape[1])
    if A.dtype != torch.float64 or A.stride() != (1, M):
        raise ValueError("A must be a column-major float64 tensor")
    Q = torch.empty((R, M), dtype=torch.float64, device=A.device).t()
    Rm = torch.empty((R, R), dtype=torch.float64, device=A.device).t()
    h = handle or default_handle(A.device.index or 0)
    st = L.cpqr_qr(h._h, M, R, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(Q.data_ptr()),
                   ctypes.c_void_p(Rm.data_ptr()))
    h.check(st)
    return Q, Rm


def qr_noalloc(A, Q, Rm, stream=None) -> int:
    """Householder QR of a column-major float64 M x R torch tensor into the
    caller's Q (M x R) and Rm (R x R), both column-major float64 on A's
    device, through the entry point that allocates nothing.  Enqueued on
    `stream` (default: torch's current stream of A's device) without
    synchronising.  Returns the status code; raises on a malformed call."""
    import torch
    L = load_library()
    M, R = int(A.shape[0]), int(A.shape[1])
    for name, t, shape in (("A", A, (M, R)), ("Q", Q, (M, R)), ("Rm", Rm, (R, R))):
        if t.dtype != torch.float64 or tuple(t.shape) != shape or t.stride() != (1, shape[0]) \
                or t.device != A.device:
            raise ValueError(f"{name} must be a column-major float64 {shape[0]} x {shape[1]} tensor "
                             "on A's device")
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    with torch.cuda.device(A.device):
        return int(L.cpqr_qr_noalloc(M, R, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(Q.data_ptr()),
                                     ctypes.c_void_p(Rm.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))


def noalloc_last_error() -> str:
    """Message of the last failed cpqr_qr_noalloc call on this thread."""
    return load_library().cpqr_last_error(None).decode()


def schedule(order: int, tree: str, sweeps: int) -> Tuple[List[List[int]], List[Tuple[int, int, int]], Dict]:
    """Host-only: (orders per sweep, steps, TTM cost polynomial) of a tree.
    The polynomial maps (sorted free modes, power of R) to its coefficient."""
    L = load_library()
    n = ctypes.c_int(0)
    st = L.cpqr_schedule(order, TREES[tree], sweeps, None, None, 0, ctypes.byref(n), None)
    if st != OK:
        raise CpqrError(st, "cpqr_schedule failed")
    orders = (ctypes.c_int * (sweeps * order))()
    steps = (ctypes.c_int * (3 * n.value))()
    flops = (ctypes.c_double * ((1 << order) * order))()
    st = L.cpqr_schedule(order, TREES[tree], sweeps, orders, steps, n.value, ctypes.byref(n), flops)
    if st != OK:
        raise CpqrError(st, "cpqr_schedule failed")
    ords = [list(orders[k * order:(k + 1) * order]) for k in range(sweeps)]
    stp = [(steps[3 * i], steps[3 * i + 1], steps[3 * i + 2]) for i in range(n.value)]
    poly = {}
    for mask in range(1 << order):
        c = flops[mask * order]
        if c:
            modes = tuple(k for k in range(order) if mask >> k & 1)
            poly[(modes, order - len(modes) + 1)] = int(c)
    return ords, stp, poly


# ------------------------------------------------------------------ tuning table
def tune_cache_check(text: str, device: str) -> int:
    """Host-only: number of entries for `device` in the text of a TTM tuning
    file (include/cpqr.h); raises CpqrError for a malformed file."""
    L = load_library()
    n = ctypes.c_int(0)
    st = L.cpqr_tune_cache_check(text.encode(), device.encode(), ctypes.byref(n))
    if st != OK:
        raise CpqrError(st, "malformed tuning file")
    return n.value


def tune_cache_path(handle: Optional[Handle] = None) -> Tuple[str, str]:
    """(file the handle's TTM tuning results go to, '' when off; device signature)."""
    L = load_library()
    h = handle or default_handle()
    path = ctypes.create_string_buffer(4096)
    dev = ctypes.create_string_buffer(4096)
    h.check(L.cpqr_tune_cache_path(h._h, path, dev, 4096))
    return path.value.decode(), dev.value.decode()


# ------------------------------------------------------------------ MLP
def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None:
        a = a.reshape(shape)
    return a


def mlp_forward(w, x, handle: Optional[Handle] = None) -> np.ndarray:
    """Learned-extrapolation MLP outputs for the rows of x (n x 8), on the GPU."""
    L = load_library()
    w = _f32(w, (MLP_PARAMS,))
    x = _f32(x, (-1, MLP_FEATURES))
    y = np.zeros(x.shape[0], dtype=np.float32)
    h = handle or default_handle(0)
    h.check(L.cpqr_mlp_forward(h._h, w.ctypes.data, x.ctypes.data, x.shape[0], y.ctypes.data))
    return y


def mlp_grad(w, x, y, handle: Optional[Handle] = None) -> Tuple[float, np.ndarray]:
    """(loss, gradient) of the mean-squared error (1/2n) sum (yhat - y)^2, on the GPU."""
    L = load_library()
    w = _f32(w, (MLP_PARAMS,))
    x = _f32(x, (-1, MLP_FEATURES))
    y = _f32(y, (x.shape[0],))
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    h = handle or default_handle(0)
    h.check(L.cpqr_mlp_grad(h._h, w.ctypes.data, x.ctypes.data, y.ctypes.data, x.shape[0],
                            loss.ctypes.data, g.ctypes.data))
    return float(loss[0]), g


def mlp_train(w, x, y, *, epochs: int, batch: int = 64, lr: float = 1e-3, seed: int = 0,
              handle: Optional[Handle] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Adam training on the GPU; returns (weights, loss after each epoch)."""
    L = load_library()
    w = _f32(w, (MLP_PARAMS,)).copy()
    x = _f32(x, (-1, MLP_FEATURES))
    y = _f32(y, (x.shape[0],))
    hist = np.zeros(max(epochs, 1), dtype=np.float32)
    h = handle or default_handle(0)
    h.check(L.cpqr_mlp_train(h._h, w.ctypes.data, x.ctypes.data, y.ctypes.data, x.shape[0],
                             int(epochs), int(batch), float(lr), int(seed), hist.ctypes.data))
    return w, hist[:epochs]
