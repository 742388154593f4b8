"""ctypes binding of libfastsv.so (C ABI in include/fastsv.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the method runs in the library's HIP kernels.  There is
no fallback: if the library is missing or fails to load, every call raises.

torch is imported before the library is loaded so that the library binds to
the HIP runtime already in the process (the one torch uses for its tensors).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# FASTSV_LIBRARY selects another build of the same library (same C ABI)
LIB_PATH = os.environ.get("FASTSV_LIBRARY") or os.path.join(_HERE, "_lib", "libfastsv.so")

TRACE_ITERS = 64

FASTSV_OK = 0
FASTSV_EINVAL = -1
FASTSV_ERANGE = -2
FASTSV_EOVERFLOW = -3
FASTSV_ENOMEM = -4
FASTSV_EHIP = -5
FASTSV_ENOTCONVERGED = -6
FASTSV_EBUSY = -7
FASTSV_ESCRATCH = -8

NOALLOC_SCRATCH_BYTES = 64 << 20  # FASTSV_NOALLOC_SCRATCH_BYTES

__all__ = ["FastSVError", "Opts", "Stats", "cc_csr", "cc_csr_noalloc", "cc_edges", "cc_batch_csr", "workspace_bytes",
           "load_library", "make_opts", "default_opts", "context", "SV_FLAGS",
           "FASTSV_OK", "FASTSV_EINVAL", "FASTSV_ERANGE", "FASTSV_EOVERFLOW", "FASTSV_ENOMEM",
           "FASTSV_EHIP", "FASTSV_ENOTCONVERGED", "FASTSV_EBUSY", "FASTSV_ESCRATCH", "NOALLOC_SCRATCH_BYTES"]


class Opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("frontier_tau", ctypes.c_float),
                ("validate", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("binned", ctypes.c_int32), ("bin_shift", ctypes.c_int32), ("sv_flags", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("trace", ctypes.c_int32), ("bin_span", ctypes.c_int32),
                ("admit_mb", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("dense_iterations", ctypes.c_int32),
                ("sparse_iterations", ctypes.c_int32), ("num_tiles", ctypes.c_int32),
                ("binned_iterations", ctypes.c_int32), ("num_bins", ctypes.c_int32),
                ("bin_fused_first", ctypes.c_int32), ("bin_span", ctypes.c_int32), ("ms_bin_prepare", ctypes.c_float),
                ("frontier_edges", ctypes.c_int64), ("alg_bytes", ctypes.c_int64),
                ("atomics_issued", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("changed", ctypes.c_int64 * TRACE_ITERS), ("sparse", ctypes.c_int32 * TRACE_ITERS),
                ("pushed", ctypes.c_int64 * TRACE_ITERS), ("atomics", ctypes.c_int64 * TRACE_ITERS),
                ("alg_hook", ctypes.c_int64 * TRACE_ITERS),
                ("ms_hook", ctypes.c_float * TRACE_ITERS), ("ms_gp", ctypes.c_float * TRACE_ITERS)]

    def changed_list(self):
        return [int(self.changed[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def sparse_list(self):
        return [int(self.sparse[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def pushed_list(self):
        return [int(self.pushed[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def alg_hook_list(self):
        return [int(self.alg_hook[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def atomics_list(self):
        return [int(self.atomics[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def ms_hook_list(self):
        return [float(self.ms_hook[i]) for i in range(min(self.iterations, TRACE_ITERS))]

    def ms_gp_list(self):
        return [float(self.ms_gp[i]) for i in range(min(self.iterations, TRACE_ITERS))]


class FastSVError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} ({status})")


_lib = None
_lock = threading.Lock()
_ctx = {}


def load_library():
    """Load libfastsv.so (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with __graft_entry__.build()")
            lib = ctypes.CDLL(LIB_PATH)
            vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
            lib.fastsv_default_opts.restype = Opts
            lib.fastsv_default_opts.argtypes = []
            lib.fastsv_create.restype = ctypes.c_int
            lib.fastsv_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
            lib.fastsv_destroy.restype = None
            lib.fastsv_destroy.argtypes = [vp]
            lib.fastsv_strerror.restype = ctypes.c_char_p
            lib.fastsv_strerror.argtypes = [ctypes.c_int]
            lib.fastsv_workspace_bytes.restype = sz
            lib.fastsv_workspace_bytes.argtypes = [i32, i64]
            lib.fastsv_workspace_bytes_opts.restype = sz
            lib.fastsv_workspace_bytes_opts.argtypes = [i32, i64, ctypes.POINTER(Opts)]
            lib.fastsv_cc_csr.restype = ctypes.c_int
            lib.fastsv_cc_csr.argtypes = [vp, i32, i64, vp, vp, vp, vp, sz, vp,
                                          ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
            lib.fastsv_cc_csr_noalloc.restype = ctypes.c_int
            lib.fastsv_cc_csr_noalloc.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.POINTER(Opts),
                                                  ctypes.POINTER(Stats)]
            lib.fastsv_cc_csr_warm.restype = ctypes.c_int
            lib.fastsv_cc_csr_warm.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, sz, vp,
                                               ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
            lib.fastsv_edges_workspace_bytes.restype = sz
            lib.fastsv_edges_workspace_bytes.argtypes = [i32, i64]
            lib.fastsv_cc_edges.restype = ctypes.c_int
            lib.fastsv_cc_edges.argtypes = [vp, i32, i64, vp, vp, vp, vp, sz, vp,
                                            ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
            lib.fastsv_batch_workspace_bytes.restype = sz
            lib.fastsv_batch_workspace_bytes.argtypes = [i32, i64]
            lib.fastsv_cc_batch_csr.restype = ctypes.c_int
            lib.fastsv_cc_batch_csr.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                                ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
            _lib = lib
    return _lib


def _strerror(status: int) -> str:
    try:
        return load_library().fastsv_strerror(status).decode()
    except Exception:  # pragma: no cover - only when the library itself is missing
        return "unknown"


def context(device: int):
    """One library context per device (created on first use, kept for the process)."""
    lib = load_library()
    with _lock:
        c = _ctx.get(device)
        if c is None:
            h = ctypes.c_void_p()
            st = lib.fastsv_create(ctypes.byref(h), device)
            if st != FASTSV_OK:
                raise FastSVError(st, "fastsv_create")
            c = _ctx[device] = h
    return c


def default_opts() -> Opts:
    return load_library().fastsv_default_opts()


SV_FLAGS = {"sv1": 0, "sv2": 1, "sv3": 3, "sv4": 7, "sv5": 15}


def make_opts(max_iters=None, frontier_tau=None, validate=None, timing=None, binned=None, bin_shift=None,
              sv_flags=None, mode=None, trace=None, bin_span=None) -> Opts:
    """binned: None/"auto" -> automatic, False -> never, True -> always.
    sv_flags: 0..15 or one of SV_FLAGS' names (None: FastSV).
    mode: None/"jacobi"/0 or "async"/1.  trace: count the hooks' atomics."""
    o = default_opts()
    if mode is not None:
        o.mode = {"jacobi": 0, "async": 1}[mode] if isinstance(mode, str) else int(mode)
    if sv_flags is not None:
        o.sv_flags = SV_FLAGS[sv_flags] if isinstance(sv_flags, str) else int(sv_flags)
    if binned is not None and binned != "auto":
        o.binned = 1 if binned else 0
    if bin_shift is not None:
        o.bin_shift = int(bin_shift)
    if max_iters is not None:
        o.max_iters = int(max_iters)
    if frontier_tau is not None:
        o.frontier_tau = float(frontier_tau)
    if validate is not None:
        o.validate = int(bool(validate))
    if timing is not None:
        o.timing = int(bool(timing))
    if trace is not None:
        o.trace = int(bool(trace))
    if bin_span is not None:
        o.bin_span = int(bin_span)
    return o


def workspace_bytes(n: int, nnz: int, opts: Opts | None = None) -> int:
    if opts is None:
        return int(load_library().fastsv_workspace_bytes(int(n), int(nnz)))
    return int(load_library().fastsv_workspace_bytes_opts(int(n), int(nnz), ctypes.byref(opts)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_vec(t, name, n=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.int32:
        raise TypeError(f"{name} must be int32")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements")


def cc_csr(row_ptr: torch.Tensor, col: torch.Tensor, *, labels: torch.Tensor | None = None,
           workspace: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None,
           max_iters=None, frontier_tau=None, validate=None, timing=None, binned=None, bin_shift=None,
           sv_flags=None, mode=None, trace=None, bin_span=None, f_init=None, tuned=False, check=True):
    """Connected components of a symmetric int32 CSR graph resident on the GPU.

    Returns (labels, stats); labels[u] is the smallest vertex of u's component.
    ``f_init`` (int32[n] on the device, may be ``labels`` itself) starts the
    iteration from that parent vector (fastsv_cc_csr_warm).
    ``tuned=True`` takes the options the autotuner stored for this device and
    graph size (``tune.py``), where the call gives none.
    With ``check=False`` the status is returned instead of raising:
    (labels, stats, status)."""
    _check_vec(row_ptr, "row_ptr")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n+1 >= 1 entries")
    _check_vec(col, "col")
    dev = row_ptr.device
    if col.device != dev:
        raise ValueError("row_ptr and col must be on the same device")
    nnz = col.numel()
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    _check_vec(labels, "labels", n)
    if tuned:
        # options the autotuner picked for this device and graph size (explicit
        # arguments take precedence); none when nothing was tuned
        from . import tune
        t = tune.lookup(dev.index if dev.index is not None else torch.cuda.current_device(), n, nnz)
        frontier_tau = t.get("frontier_tau", frontier_tau) if frontier_tau is None else frontier_tau
        bin_shift = t.get("bin_shift", bin_shift) if bin_shift is None else bin_shift
        bin_span = t.get("bin_span", bin_span) if bin_span is None else bin_span
    opts = make_opts(max_iters, frontier_tau, validate, timing, binned, bin_shift, sv_flags, mode, trace, bin_span)
    if workspace is None:
        wsb = workspace_bytes(n, nnz, opts)
        if wsb == 0:
            raise ValueError("sizes do not fit the int32 layout, or invalid options")
        workspace = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) & ~255
    ws_bytes = workspace.numel() - (aligned - base)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    stats = Stats()
    lib = load_library()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    if f_init is None:
        st = lib.fastsv_cc_csr(ctx, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(labels),
                               ctypes.c_void_p(aligned), ws_bytes, ctypes.c_void_p(s.cuda_stream),
                               ctypes.byref(opts), ctypes.byref(stats))
    else:
        _check_vec(f_init, "f_init", n)
        if f_init.device != dev:
            raise ValueError("f_init must be on the graph's device")
        st = lib.fastsv_cc_csr_warm(ctx, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(f_init), _ptr(labels),
                                    ctypes.c_void_p(aligned), ws_bytes, ctypes.c_void_p(s.cuda_stream),
                                    ctypes.byref(opts), ctypes.byref(stats))
    if not check:
        return labels, stats, st
    if st != FASTSV_OK:
        raise FastSVError(st, "fastsv_cc_csr_warm" if f_init is not None else "fastsv_cc_csr")
    return labels, stats


def cc_csr_noalloc(row_ptr: torch.Tensor, col: torch.Tensor, *, labels: torch.Tensor | None = None,
                   stream: torch.cuda.Stream | None = None, max_iters=None, frontier_tau=None, validate=None,
                   timing=None, binned=None, bin_shift=None, sv_flags=None, mode=None, trace=None, check=True):
    """cc_csr through fastsv_cc_csr_noalloc: the library allocates no device
    memory during the call (its workspace is the library's fixed scratch
    array).  ``labels`` may be preallocated so that the whole call allocates
    nothing.  Returns (labels, stats), or (labels, stats, status) with
    ``check=False``."""
    _check_vec(row_ptr, "row_ptr")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n+1 >= 1 entries")
    _check_vec(col, "col")
    dev = row_ptr.device
    if col.device != dev:
        raise ValueError("row_ptr and col must be on the same device")
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    _check_vec(labels, "labels", n)
    opts = make_opts(max_iters, frontier_tau, validate, timing, binned, bin_shift, sv_flags, mode, trace)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    stats = Stats()
    lib = load_library()
    st = lib.fastsv_cc_csr_noalloc(context(_dev_index(dev)), n, col.numel(), _ptr(row_ptr), _ptr(col), _ptr(labels),
                                   ctypes.c_void_p(s.cuda_stream), ctypes.byref(opts), ctypes.byref(stats))
    if not check:
        return labels, stats, st
    if st != FASTSV_OK:
        raise FastSVError(st, "fastsv_cc_csr_noalloc")
    return labels, stats


def _workspace(nbytes, dev, workspace):
    if workspace is None:
        if nbytes == 0:
            raise ValueError("sizes do not fit the int32 layout, or invalid options")
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) & ~255
    return workspace, ctypes.c_void_p(aligned), workspace.numel() - (aligned - base)


def _dev_index(dev):
    return dev.index if dev.index is not None else torch.cuda.current_device()


def cc_edges(n: int, src: torch.Tensor, dst: torch.Tensor, *, labels=None, workspace=None, stream=None,
             max_iters=None, frontier_tau=None, validate=None, timing=None, sv_flags=None, mode=None, trace=None,
             check=True):
    """Connected components from an undirected edge list (each edge once, any
    orientation).  Returns (labels, stats)."""
    _check_vec(src, "src")
    _check_vec(dst, "dst", src.numel())
    dev = src.device
    m = src.numel()
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    _check_vec(labels, "labels", n)
    opts = make_opts(max_iters, frontier_tau, validate, timing, sv_flags=sv_flags, mode=mode, trace=trace)
    lib = load_library()
    workspace, ws, wsb = _workspace(int(lib.fastsv_edges_workspace_bytes(int(n), int(m))), dev, workspace)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    stats = Stats()
    st = lib.fastsv_cc_edges(context(_dev_index(dev)), int(n), int(m), _ptr(src), _ptr(dst), _ptr(labels), ws, wsb,
                             ctypes.c_void_p(s.cuda_stream), ctypes.byref(opts), ctypes.byref(stats))
    if not check:
        return labels, stats, st
    if st != FASTSV_OK:
        raise FastSVError(st, "fastsv_cc_edges")
    return labels, stats


def cc_batch_csr(vtx_off: torch.Tensor, edge_off: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, *,
                 labels=None, iters=None, workspace=None, stream=None, max_iters=None, frontier_tau=None,
                 validate=None, timing=None, trace=None, check=True):
    """Many graphs in one call.  row_ptr is global over the concatenation,
    column ids are local to each graph.  Returns (labels in local ids,
    per-graph iteration counts, stats)."""
    for t, name in ((vtx_off, "vtx_off"), (edge_off, "edge_off"), (row_ptr, "row_ptr"), (col, "col")):
        _check_vec(t, name)
    g = vtx_off.numel() - 1
    if g < 0 or edge_off.numel() != g + 1:
        raise ValueError("vtx_off and edge_off need G+1 entries")
    dev = row_ptr.device
    total_n = row_ptr.numel() - 1
    total_nnz = col.numel()
    if labels is None:
        labels = torch.empty(total_n, dtype=torch.int32, device=dev)
    if iters is None:
        iters = torch.empty(max(g, 1), dtype=torch.int32, device=dev)
    _check_vec(labels, "labels", total_n)
    opts = make_opts(max_iters, frontier_tau, validate, timing, trace=trace)
    lib = load_library()
    workspace, ws, wsb = _workspace(int(lib.fastsv_batch_workspace_bytes(int(total_n), int(total_nnz))), dev,
                                    workspace)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    stats = Stats()
    st = lib.fastsv_cc_batch_csr(context(_dev_index(dev)), int(g), int(total_n), int(total_nnz), _ptr(vtx_off),
                                 _ptr(edge_off), _ptr(row_ptr), _ptr(col), _ptr(labels), _ptr(iters), ws, wsb,
                                 ctypes.c_void_p(s.cuda_stream), ctypes.byref(opts), ctypes.byref(stats))
    if not check:
        return labels, iters[:g], stats, st
    if st != FASTSV_OK:
        raise FastSVError(st, "fastsv_cc_batch_csr")
    return labels, iters[:g], stats
