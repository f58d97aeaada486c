"""Thin Python binding of libaop's C ABI (include/aop.h).

Argument marshalling only: every pricing step runs in the gfx950 kernels of
``libaop.so``.  PyTorch provides device memory (workspace, outputs) and the
HIP stream.  Importing this module never falls back to anything else: if the
library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaop.so")

AOP_BINOMIAL_CALL, AOP_TRINOMIAL_CALL, AOP_BSM_PUT = 0, 1, 2
AOP_FP64, AOP_MIXED = 0, 1
AOP_EUROPEAN = 1  # aop_option.flags bit: exercise at expiry only
STATUS = {0: "ok", 1: "EINVAL", 2: "EPROB", 3: "ENOMEM", 4: "EDEVICE", 5: "ETOOBIG", 6: "ECANCELED",
          7: "ENOTIMPL"}
BSM_NONE = np.iinfo(np.int64).min

#: Every symbol include/aop.h declares.
EXPORTS = ["aop_twiddle_bytes", "aop_ctx_create", "aop_ctx_destroy", "aop_workspace_bytes", "aop_validate", "aop_price_batch",
           "aop_plain_workspace_bytes", "aop_price_batch_plain", "aop_batch_stats", "aop_price", "aop_sync",
           "aop_status_str", "aop_version", "aop_pool_stats", "aop_pool_abort_info", "aop_ctx_get_tuning", "aop_ctx_set_tuning",
           "aop_server_create", "aop_server_submit", "aop_server_poll", "aop_server_stats", "aop_server_destroy",
           "aop_graph_create", "aop_graph_launch", "aop_graph_destroy", "aop_batch_errors",
           "aop_price_batch_noalloc", "aop_noalloc_scratch_bytes", "aop_approx_workspace_bytes",
           "aop_european_approx"]

STATS_FIELDS = ["convs", "conv_in", "conv_out", "fft_points", "band_rows", "direct_cells", "max_depth",
                "trapezoids", "n_direct", "n_fft", "cyc_band", "cyc_tiles", "cyc_wait", "cyc_rows", "cyc_total",
                "n_published"]
POOL_FIELDS = ["workgroups", "helper_tiles", "helper_busy", "helper_idle", "options_done", "aborted"]


class AopTuning(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int32), ("pub_min_lg", ctypes.c_int32), ("pub_direct", ctypes.c_int32),
                ("direct_max_h", ctypes.c_int32), ("direct_max_n", ctypes.c_int32),
                ("helper_idle_us", ctypes.c_int32), ("late_pub_min_lg", ctypes.c_int32),
                ("late_after_pct", ctypes.c_int32), ("lds_max_lg", ctypes.c_int32), ("radix_lg", ctypes.c_int32),
                ("timeout_ms", ctypes.c_int64), ("timeout_us", ctypes.c_int64)]


class AopError(RuntimeError):
    pass


class AopClassTuning(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("log2T", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tuning", AopTuning)]


class AopServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tunings", ctypes.POINTER(AopClassTuning)), ("n_tunings", ctypes.c_int64),
                ("d_arena", ctypes.c_void_p)]


class AopResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("price", ctypes.c_double), ("status", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double)]


SERVER_STATS = ["submitted", "completed", "batches", "inflight", "pending", "peak_bytes", "arena_bytes",
                "workgroups_per_batch", "alg_bytes"]


class AopOption(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("flags", ctypes.c_int32), ("S0", ctypes.c_double),
                ("K", ctypes.c_double), ("r", ctypes.c_double), ("q", ctypes.c_double),
                ("sigma", ctypes.c_double), ("expiry", ctypes.c_double), ("T", ctypes.c_int64),
                ("exercise_every", ctypes.c_int64)]


_lib = None


def load():
    """Load libaop.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise AopError("libaop.so is not built (run __graft_entry__.build()); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "aop_twiddle_bytes": (SZ, []),
        "aop_ctx_create": (I32, [ctypes.c_int, D, P, SZ, ctypes.POINTER(P)]),
        "aop_ctx_destroy": (I32, [P]),
        "aop_workspace_bytes": (I32, [P, I64, I32, ctypes.POINTER(SZ)]),
        "aop_validate": (I32, [P, D]),
        "aop_price_batch": (I32, [P, P, I64, I32, P, SZ, P, P, P, I64, P]),
        "aop_plain_workspace_bytes": (I32, [P, I64, ctypes.POINTER(SZ)]),
        "aop_price_batch_plain": (I32, [P, P, I64, P, SZ, P, P, P, I64, P]),
        "aop_batch_stats": (I32, [P, I64, P]),
        "aop_price": (I32, [P, P, I32, ctypes.POINTER(D), P]),
        "aop_sync": (I32, [P]),
        "aop_status_str": (ctypes.c_char_p, [I32]),
        "aop_version": (ctypes.c_char_p, []),
        "aop_pool_stats": (I32, [P, I64, P]),
        "aop_pool_abort_info": (I32, [P, I64, P]),
        "aop_ctx_get_tuning": (I32, [P, ctypes.POINTER(AopTuning)]),
        "aop_ctx_set_tuning": (I32, [P, ctypes.POINTER(AopTuning)]),
        "aop_server_create": (I32, [P, ctypes.POINTER(AopServerConfig), ctypes.POINTER(P)]),
        "aop_server_submit": (I32, [P, P, P, I64]),
        "aop_server_poll": (I32, [P, P, I64, ctypes.POINTER(I64), I32]),
        "aop_server_stats": (I32, [P, P]),
        "aop_server_destroy": (I32, [P]),
        "aop_graph_create": (I32, [P, P, I64, I32, P, SZ, P, P, P, I64, ctypes.POINTER(P)]),
        "aop_graph_launch": (I32, [P, P]),
        "aop_graph_destroy": (I32, [P]),
        "aop_batch_errors": (I32, [P, I64, P]),
        "aop_price_batch_noalloc": (I32, [P, P, I64, I32, P, P, P, I64, P]),
        "aop_noalloc_scratch_bytes": (SZ, []),
        "aop_approx_workspace_bytes": (SZ, [I64]),
        "aop_european_approx": (I32, [P, P, I64, I32, P, SZ, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc, what):
    if rc != 0:
        raise AopError("%s failed: %s" % (what, load().aop_status_str(rc).decode()))


def options_array(opts) -> ctypes.Array:
    arr = (AopOption * max(1, len(opts)))()
    for i, o in enumerate(opts):
        flags = AOP_EUROPEAN if o.get("european", False) else 0
        arr[i] = AopOption(int(o["model"]), flags, float(o["S0"]), float(o["K"]), float(o["r"]), float(o["q"]),
                           float(o["sigma"]), float(o["expiry"]), int(o["T"]), int(o.get("exercise_every", 0)))
    return arr


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """An aop_ctx on one device.  The twiddle table is a torch tensor held here
    (the library fills and reads it); the context itself keeps a pinned
    staging buffer."""

    def __init__(self, device: int = 0, lam: float = 1.0 / 3.0):
        # PyTorch owns device memory and streams: bring its HIP state up
        # before the library touches the runtime.
        import torch

        torch.cuda.init()
        lib = load()
        nb = int(lib.aop_twiddle_bytes())
        self.twiddles = torch.empty(nb, dtype=torch.uint8, device=torch.device("cuda", device))
        self._h = ctypes.c_void_p()
        _check(lib.aop_ctx_create(int(device), float(lam), ctypes.c_void_p(self.twiddles.data_ptr()), nb,
                                  ctypes.byref(self._h)), "aop_ctx_create")
        self.device = device
        self.lam = lam

    @property
    def handle(self):
        return self._h

    def tuning(self) -> dict:
        t = AopTuning()
        _check(load().aop_ctx_get_tuning(self._h, ctypes.byref(t)), "aop_ctx_get_tuning")
        return {f: getattr(t, f) for f, _ in AopTuning._fields_}

    def set_tuning(self, **kw):
        """Change launch tuning fields (see aop_tuning); unknown fields raise."""
        cur = self.tuning()
        for k, v in kw.items():
            if k not in cur:
                raise KeyError(k)
            cur[k] = int(v)
        t = AopTuning(**cur)
        _check(load().aop_ctx_set_tuning(self._h, ctypes.byref(t)), "aop_ctx_set_tuning")

    def close(self):
        if self._h:
            load().aop_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.twiddles = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(opts, precision: int = AOP_FP64) -> int:
    arr = options_array(opts)
    n = ctypes.c_size_t()
    _check(load().aop_workspace_bytes(arr, len(opts), int(precision), ctypes.byref(n)), "aop_workspace_bytes")
    return n.value


def plain_workspace_bytes(opts) -> int:
    arr = options_array(opts)
    n = ctypes.c_size_t()
    _check(load().aop_plain_workspace_bytes(arr, len(opts), ctypes.byref(n)), "aop_plain_workspace_bytes")
    return n.value


def validate(opt, lam: float = 1.0 / 3.0) -> int:
    return int(load().aop_validate(options_array([opt]), float(lam)))


@dataclass
class Launch:
    """Device outputs of one asynchronous batch launch."""
    price: "object"      # torch float64 tensor [n] on the device
    status: np.ndarray   # host int32 [n]
    boundary: "object"   # torch int64 tensor [n, stride] or None
    workspace: "object"  # torch uint8 tensor (kept alive until the stream passes)


def launch_batch(ctx: Context, opts, precision: int = AOP_FP64, boundary: bool = False, stream=None,
                 workspace=None) -> Launch:
    """Enqueue pricing of ``opts`` on ``stream``; returns device tensors (no sync)."""
    import torch

    lib = load()
    n = len(opts)
    dev = torch.device("cuda", ctx.device)
    arr = options_array(opts)
    need = workspace_bytes(opts, precision)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    price = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    stride = max(int(o["T"]) for o in opts) + 1 if (boundary and n) else 0
    bnd = torch.empty((max(n, 1), max(stride, 1)), dtype=torch.int64, device=dev) if boundary else None
    status = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib.aop_price_batch(ctx.handle, arr, n, int(precision), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel(), ctypes.c_void_p(price.data_ptr()),
                             status.ctypes.data_as(ctypes.c_void_p),
                             ctypes.c_void_p(bnd.data_ptr()) if bnd is not None else None, stride,
                             _stream_handle(stream))
    _check(rc, "aop_price_batch")
    return Launch(price[:n], status[:n], bnd[:n] if bnd is not None else None, workspace)


def price_batch(ctx: Context, opts, precision: int = AOP_FP64, boundary: bool = False, stream=None):
    """Price a batch and wait: returns (prices, status, boundaries or None) as numpy arrays."""
    import torch

    L = launch_batch(ctx, opts, precision, boundary, stream)
    (stream or torch.cuda.current_stream()).synchronize()
    b = L.boundary.cpu().numpy() if L.boundary is not None else None
    return L.price.cpu().numpy(), L.status.copy(), b


def launch_batch_noalloc(ctx: Context, opts, precision: int = AOP_FP64, boundary: bool = False, stream=None,
                         price=None, bnd=None):
    """aop_price_batch_noalloc: the library's fixed scratch as workspace.  The
    outputs are the caller's (given, or made here as torch tensors); the call
    itself allocates nothing.  Returns (price, status, boundary) without sync."""
    import torch

    lib = load()
    n = len(opts)
    dev = torch.device("cuda", ctx.device)
    arr = options_array(opts)
    if price is None:
        price = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    stride = bnd.shape[1] if bnd is not None else 0
    if boundary and bnd is None:
        stride = max(int(o["T"]) for o in opts) + 1 if n else 0
        bnd = torch.empty((max(n, 1), max(stride, 1)), dtype=torch.int64, device=dev)
    status = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib.aop_price_batch_noalloc(ctx.handle, arr, n, int(precision), ctypes.c_void_p(price.data_ptr()),
                                     status.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.c_void_p(bnd.data_ptr()) if bnd is not None else None, stride,
                                     _stream_handle(stream))
    _check(rc, "aop_price_batch_noalloc")
    return price[:n], status[:n], (bnd[:n] if bnd is not None else None)


GAUSS_WINDOW, GAUSS_SUM, GAUSS_ERF = 0, 1, 2


def european_approx(ctx: Context, opts, method: int, stream=None):
    """aop_european_approx: Gaussian approximations of European binomial calls.
    Returns (prices as numpy, status) after synchronising the stream."""
    import torch

    lib = load()
    n = len(opts)
    dev = torch.device("cuda", ctx.device)
    ws = torch.empty(int(lib.aop_approx_workspace_bytes(n)), dtype=torch.uint8, device=dev)
    price = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    status = np.zeros(max(n, 1), dtype=np.int32)
    _check(lib.aop_european_approx(ctx.handle, options_array(opts), n, int(method), ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), ctypes.c_void_p(price.data_ptr()),
                                   status.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)),
           "aop_european_approx")
    (stream or torch.cuda.current_stream()).synchronize()
    return price[:n].cpu().numpy(), status[:n]


def launch_plain(ctx: Context, opts, stream=None, workspace=None, boundary: bool = False):
    """Enqueue the plain Theta(T^2) GPU stencil on ``opts`` (comparison path)."""
    import torch

    lib = load()
    n = len(opts)
    dev = torch.device("cuda", ctx.device)
    arr = options_array(opts)
    need = plain_workspace_bytes(opts)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    price = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    status = np.zeros(max(n, 1), dtype=np.int32)
    stride = max(int(o["T"]) for o in opts) + 1 if (boundary and n) else 0
    bnd = torch.empty((max(n, 1), max(stride, 1)), dtype=torch.int64, device=dev) if boundary else None
    rc = lib.aop_price_batch_plain(ctx.handle, arr, n, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   ctypes.c_void_p(price.data_ptr()), status.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(bnd.data_ptr()) if bnd is not None else None, stride,
                                   _stream_handle(stream))
    _check(rc, "aop_price_batch_plain")
    return Launch(price[:n], status[:n], bnd[:n] if bnd is not None else None, workspace)


def batch_stats(launch: "Launch", n: int) -> np.ndarray:
    """Work counters of a finished launch: int64 array [n, len(STATS_FIELDS)]."""
    out = np.zeros((max(n, 1), len(STATS_FIELDS)), dtype=np.int64)
    _check(load().aop_batch_stats(ctypes.c_void_p(launch.workspace.data_ptr()), n,
                                  out.ctypes.data_as(ctypes.c_void_p)), "aop_batch_stats")
    return out[:n]


def batch_errors(launch, n: int) -> np.ndarray:
    """Device error code of each option of a finished launch (0: none)."""
    out = np.zeros(max(n, 1), dtype=np.int32)
    _check(load().aop_batch_errors(ctypes.c_void_p(launch.workspace.data_ptr()), n,
                                   out.ctypes.data_as(ctypes.c_void_p)), "aop_batch_errors")
    return out[:n]


def pool_stats(launch: "Launch", n: int) -> dict:
    """Work-pool counters of a finished launch."""
    out = np.zeros(8, dtype=np.int64)
    _check(load().aop_pool_stats(ctypes.c_void_p(launch.workspace.data_ptr()), n,
                                 out.ctypes.data_as(ctypes.c_void_p)), "aop_pool_stats")
    return {f: int(out[i]) for i, f in enumerate(POOL_FIELDS)}


ABORT_FIELDS = ["reason", "slot", "phase_tile_or_ctl", "kind_sizes", "desc_nin_or_kind", "nout_or_wg", "ctl_or_slot", "unused"]


def pool_abort_info(launch: "Launch", n: int) -> dict:
    """First cause of an aborted launch (aop_pool_abort_info): reason 0 none, 1 refused job, 2/3 deadline."""
    out = np.zeros(8, dtype=np.int64)
    _check(load().aop_pool_abort_info(ctypes.c_void_p(launch.workspace.data_ptr()), n,
                                      out.ctypes.data_as(ctypes.c_void_p)), "aop_pool_abort_info")
    return {f: int(out[i]) for i, f in enumerate(ABORT_FIELDS)}


def price_one(ctx: Context, opt, precision: int = AOP_FP64, boundary: bool = False):
    """Synchronous single option through aop_price (the library allocates)."""
    lib = load()
    out = ctypes.c_double()
    b = np.empty(int(opt["T"]) + 1, dtype=np.int64) if boundary else None
    rc = lib.aop_price(ctx.handle, options_array([opt]), int(precision), ctypes.byref(out),
                       b.ctypes.data_as(ctypes.c_void_p) if b is not None else None)
    _check(rc, "aop_price")
    return (out.value, b) if boundary else out.value


class Server:
    """Continuous-batching server (aop_server_*): submit requests, poll results."""

    def __init__(self, ctx: Context, hbm_budget: int = 0, max_inflight: int = 4, max_batch: int = 64,
                 precision: int = AOP_FP64, tunings=None):
        """tunings: [(model, log2T, precision, schedule dict)] per size class (the autotuner's table).
        hbm_budget: bytes of the arena this object allocates as a torch tensor
        (0: a quarter of the device's free memory)."""
        import torch

        lib = load()
        dev = torch.device("cuda", ctx.device)
        if hbm_budget <= 0:
            free, _ = torch.cuda.mem_get_info(dev)
            hbm_budget = free // 4
        hbm_budget = int(hbm_budget) // 256 * 256
        self.arena = torch.empty(hbm_budget, dtype=torch.uint8, device=dev)
        self._h = ctypes.c_void_p()
        tab = list(tunings or [])
        base = ctx.tuning()
        arr = (AopClassTuning * max(1, len(tab)))()
        for i, (m, lg, p, sched) in enumerate(tab):
            arr[i] = AopClassTuning(int(m), int(lg), int(p), 0, AopTuning(**dict(base, **sched)))
        self._tab = arr
        cfg = AopServerConfig(int(hbm_budget), int(max_inflight), int(max_batch), int(precision), 0,
                              ctypes.cast(arr, ctypes.POINTER(AopClassTuning)) if tab else None, len(tab),
                              ctypes.c_void_p(self.arena.data_ptr()))
        _check(lib.aop_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(self._h)), "aop_server_create")
        self.ctx = ctx

    def submit(self, opts, ids):
        arr = options_array(opts)
        idv = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        _check(load().aop_server_submit(self._h, arr, idv.ctypes.data_as(ctypes.c_void_p), len(opts)),
               "aop_server_submit")

    def poll(self, max_results: int = 4096, wait_us: int = 1000):
        """Finished results as a list of dicts (any order)."""
        buf = (AopResult * max(1, max_results))()
        n = ctypes.c_int64()
        rc = load().aop_server_poll(self._h, buf, max_results, ctypes.byref(n), int(wait_us))
        out = [dict(id=int(buf[i].id), price=buf[i].price, status=buf[i].status, batch_size=buf[i].batch_size,
                    queue_s=buf[i].queue_s, latency_s=buf[i].latency_s) for i in range(n.value)]
        _check(rc, "aop_server_poll")
        return out

    def stats(self) -> dict:
        out = np.zeros(len(SERVER_STATS), dtype=np.int64)
        _check(load().aop_server_stats(self._h, out.ctypes.data_as(ctypes.c_void_p)), "aop_server_stats")
        return {f: int(out[i]) for i, f in enumerate(SERVER_STATS)}

    def close(self):
        if self._h:
            load().aop_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """A batch launch captured once in a hipGraph (aop_graph_*), replayed with launch()."""

    def __init__(self, ctx: Context, opts, precision: int = AOP_FP64, boundary: bool = False):
        import torch

        lib = load()
        n = len(opts)
        dev = torch.device("cuda", ctx.device)
        arr = options_array(opts)
        self.workspace = torch.empty(workspace_bytes(opts, precision), dtype=torch.uint8, device=dev)
        self.price = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        stride = max(int(o["T"]) for o in opts) + 1 if boundary else 0
        self.boundary = torch.empty((n, stride), dtype=torch.int64, device=dev) if boundary else None
        self.status = np.zeros(max(n, 1), dtype=np.int32)
        self.n = n
        self._h = ctypes.c_void_p()
        torch.cuda.synchronize(dev)
        _check(lib.aop_graph_create(ctx.handle, arr, n, int(precision), ctypes.c_void_p(self.workspace.data_ptr()),
                                    self.workspace.numel(), ctypes.c_void_p(self.price.data_ptr()),
                                    self.status.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.c_void_p(self.boundary.data_ptr()) if boundary else None, stride,
                                    ctypes.byref(self._h)), "aop_graph_create")

    def launch(self, stream=None):
        _check(load().aop_graph_launch(self._h, _stream_handle(stream)), "aop_graph_launch")
        return self.price[:self.n]

    def close(self):
        if self._h:
            load().aop_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
