"""MI355X (gfx950) NN-Descent K-NN graph construction, squared-l2 metric.

Thin ctypes binding of ``libknng.so`` (C ABI in ``include/knng.h``). It only
marshals arguments: torch provides the device memory (inputs, outputs and the
workspace) and the stream; every step of the method runs in the HIP kernels.
There is no CPU fallback: if the library is missing or fails to load, this
module raises on import.

Method: Kluser et al., "Fast single-core K-Nearest Neighbor Graph
computation" (arXiv 2112.06630), Sec. 2 (K-NNG, NN-Descent), Sec. 3.1
(sampling), Sec. 3.2 (reordering), Sec. 3.3 (squared-l2 distances).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = ["build", "build_noalloc", "Context", "Params", "workspace_bytes", "sample_cap", "KnngError", "LIB_PATH",
           "PATH_AUTO", "PATH_VALU", "PATH_MFMA", "PATH_MFMA_I8", "PATH_MFMA_BF16X3", "MAX_ITERS", "lib",
           "SAMPLING_WEIGHTED", "SAMPLING_TURBO"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknng.so")

PATH_AUTO, PATH_VALU, PATH_MFMA, PATH_MFMA_I8, PATH_MFMA_BF16X3 = 0, 1, 2, 3, 4
_PATHS = {"auto": PATH_AUTO, "valu": PATH_VALU, "mfma": PATH_MFMA, "mfma_i8": PATH_MFMA_I8,
          "bf16x3": PATH_MFMA_BF16X3}
SAMPLING_WEIGHTED, SAMPLING_TURBO = 0, 1
_SAMPLING = {"weighted": SAMPLING_WEIGHTED, "turbo": SAMPLING_TURBO}
MAX_ITERS = 64
MAX_NOALLOC_BYTES = 64 << 20   # KNNG_NOALLOC_MAX_BYTES

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV = 0, 1, 2, 3, 4


class KnngError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"knng status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("rho", ctypes.c_double), ("delta", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("path", ctypes.c_int32), ("sampling", ctypes.c_int32),
                ("blocks", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("path", ctypes.c_int32),
                ("dpad", ctypes.c_int32), ("precision", ctypes.c_int32), ("planes", ctypes.c_int32),
                ("accurate", ctypes.c_int32), ("u8", ctypes.c_int32),
                ("evals", ctypes.c_int64 * MAX_ITERS), ("changes", ctypes.c_int64 * MAX_ITERS),
                ("proposals", ctypes.c_int64 * MAX_ITERS), ("rescored", ctypes.c_int64 * MAX_ITERS),
                ("iter_ms", ctypes.c_float * MAX_ITERS), ("sample_ms", ctypes.c_float * MAX_ITERS),
                ("join_ms", ctypes.c_float * MAX_ITERS), ("merge_ms", ctypes.c_float * MAX_ITERS),
                ("init_ms", ctypes.c_float), ("reorder_ms", ctypes.c_float),
                ("finalize_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    PP = ctypes.POINTER(Params)
    L.knng_workspace_bytes.argtypes = [i64, i32, PP]
    L.knng_workspace_bytes.restype = sz
    L.knng_build.argtypes = [P, i64, i32, PP, P, P, P, sz, P, ctypes.POINTER(_Stats)]
    L.knng_build_noalloc.argtypes = [P, i64, i32, PP, P, P, P, ctypes.POINTER(_Stats)]
    L.knng_create.argtypes = [ctypes.POINTER(P), P, i64, i32, PP, P, sz, P]
    L.knng_init_graph.argtypes = [P]
    L.knng_load_graph.argtypes = [P, P, P, P, i32]
    L.knng_iterate.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.knng_export.argtypes = [P, P, P, P]
    L.knng_export_samples.argtypes = [P, P, P, P]
    L.knng_get_stats.argtypes = [P, ctypes.POINTER(_Stats)]
    L.knng_export_order.argtypes = [P, P]
    L.knng_destroy.argtypes = [P]
    L.knng_destroy.restype = None
    L.knng_sample_cap.argtypes = [i32, ctypes.c_double]
    L.knng_sample_cap.restype = i32
    L.knng_last_error.restype = ctypes.c_char_p
    for n in ("knng_build", "knng_create", "knng_init_graph", "knng_load_graph", "knng_iterate",
              "knng_export", "knng_export_samples", "knng_get_stats", "knng_export_order"):
        getattr(L, n).restype = ctypes.c_int
    return L


lib = _load()


def _err() -> str:
    return (lib.knng_last_error() or b"").decode()


def _check(st: int, allow=(OK,)):
    if st not in allow:
        raise KnngError(st, _err())
    return st


PRECISION_FP32, PRECISION_BF16_SCREEN = 0, 1
_PRECISIONS = {"fp32": PRECISION_FP32, "bf16": PRECISION_BF16_SCREEN}


def make_params(K: int, rho: float = 1.0, delta: float = 0.001, max_iters: int = 30, seed: int = 0,
                reorder: bool | int = False, path: str | int = "auto", precision: str | int = "fp32",
                sampling: str | int = "weighted", blocks: int = 0) -> Params:
    pth = _PATHS[path] if isinstance(path, str) else int(path)
    prc = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    smp = _SAMPLING[sampling] if isinstance(sampling, str) else int(sampling)
    # reorder: False/0 off, True/1 after iteration 1, an int t_p after iteration t_p
    return Params(int(K), float(rho), float(delta), int(max_iters), int(seed) & 0xFFFFFFFFFFFFFFFF, prc,
                  int(reorder), pth, smp, int(blocks))


def sample_cap(K: int, rho: float) -> int:
    return int(lib.knng_sample_cap(K, rho))


def workspace_bytes(N: int, d: int, params: Params) -> int:
    n = int(lib.knng_workspace_bytes(N, d, ctypes.byref(params)))
    if n == 0:
        raise KnngError(EINVAL, _err())
    return n


def _stream_ptr(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _check_x(X: torch.Tensor):
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
        raise ValueError("X must be a device tensor (ROCm)")
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous float32 [N, d] tensor")


def _stats_dict(s: _Stats) -> dict:
    it = s.iters
    return dict(iters=it, converged=bool(s.converged), path=s.path, dpad=s.dpad, precision=s.precision,
                planes=s.planes, accurate=s.accurate, u8=s.u8,
                evals=list(s.evals[:it]), changes=list(s.changes[:it]), proposals=list(s.proposals[:it]),
                rescored=list(s.rescored[:it]),
                iter_ms=list(s.iter_ms[:it]), sample_ms=list(s.sample_ms[:it]), join_ms=list(s.join_ms[:it]),
                merge_ms=list(s.merge_ms[:it]), init_ms=s.init_ms, reorder_ms=s.reorder_ms,
                finalize_ms=s.finalize_ms, total_ms=s.total_ms)


def build(X: torch.Tensor, K: int, rho: float = 1.0, delta: float = 0.001, max_iters: int = 30, seed: int = 0,
          reorder: bool | int = False, path: str | int = "auto", workspace: torch.Tensor | None = None,
          out: tuple | None = None, precision: str | int = "fp32", sampling: str | int = "weighted",
          blocks: int = 0):
    """K-NN graph of the rows of X (device float32 [N, d]).

    Returns (ids int32 [N, K], dists float32 [N, K] squared l2, stats dict);
    rows sorted by (distance, id). ``workspace`` (uint8 device tensor of at
    least ``workspace_bytes``) and ``out`` may be passed to reuse memory.
    """
    _check_x(X)
    N, d = X.shape
    p = make_params(K, rho, delta, max_iters, seed, reorder, path, precision, sampling, blocks)
    ws = workspace_bytes(N, d, p)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(ws, dtype=torch.uint8, device=X.device)
    if out is None:
        ids = torch.empty((N, K), dtype=torch.int32, device=X.device)
        dists = torch.empty((N, K), dtype=torch.float32, device=X.device)
    else:
        ids, dists = out
    st = _Stats()
    _check(lib.knng_build(ctypes.c_void_p(X.data_ptr()), N, d, ctypes.byref(p), ctypes.c_void_p(ids.data_ptr()),
                          ctypes.c_void_p(dists.data_ptr()), ctypes.c_void_p(workspace.data_ptr()), ws,
                          ctypes.c_void_p(_stream_ptr(X.device)), ctypes.byref(st)), allow=(OK, ENOTCONV))
    return ids, dists, _stats_dict(st)


def build_noalloc(X: torch.Tensor, K: int, ids: torch.Tensor, dists: torch.Tensor, rho: float = 1.0,
                  delta: float = 0.001, max_iters: int = 30, seed: int = 0, reorder: bool | int = False,
                  path: str | int = "auto", precision: str | int = "fp32", sampling: str | int = "weighted",
                  blocks: int = 0) -> dict:
    """knng_build_noalloc: the build with the library's static device scratch
    as workspace (nothing allocated). The caller passes the outputs ids
    (int32 [N, K]) and dists (float32 [N, K]); returns the stats dict (no
    timings). Raises KnngError (ENOMEM) when the build does not fit the
    scratch (MAX_NOALLOC_BYTES)."""
    _check_x(X)
    N, d = X.shape
    if tuple(ids.shape) != (N, K) or tuple(dists.shape) != (N, K) or ids.dtype != torch.int32 \
            or dists.dtype != torch.float32:
        raise ValueError("ids / dists must be int32 / float32 [N, K]")
    if not (ids.is_contiguous() and dists.is_contiguous()):
        raise ValueError("ids / dists must be contiguous")
    p = make_params(K, rho, delta, max_iters, seed, reorder, path, precision, sampling, blocks)
    st = _Stats()
    _check(lib.knng_build_noalloc(ctypes.c_void_p(X.data_ptr()), N, d, ctypes.byref(p),
                                  ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dists.data_ptr()),
                                  ctypes.c_void_p(_stream_ptr(X.device)), ctypes.byref(st)), allow=(OK, ENOTCONV))
    return _stats_dict(st)


@dataclass
class Graph:
    ids: torch.Tensor
    dists: torch.Tensor
    flags: torch.Tensor


class Context:
    """Step API: one build whose state lives in a caller-held workspace."""

    def __init__(self, X: torch.Tensor, K: int, rho: float = 1.0, delta: float = 0.001, max_iters: int = 30,
                 seed: int = 0, reorder: bool | int = False, path: str | int = "auto", precision: str | int = "fp32",
                 sampling: str | int = "weighted", blocks: int = 0):
        _check_x(X)
        self.X = X
        self.N, self.d = X.shape
        self.K = K
        self.params = make_params(K, rho, delta, max_iters, seed, reorder, path, precision, sampling, blocks)
        self.C = sample_cap(K, rho)
        self.ws_bytes = workspace_bytes(self.N, self.d, self.params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=X.device)
        h = ctypes.c_void_p()
        _check(lib.knng_create(ctypes.byref(h), ctypes.c_void_p(X.data_ptr()), self.N, self.d,
                               ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                               ctypes.c_void_p(_stream_ptr(X.device))))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.knng_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self):
        _check(lib.knng_init_graph(self._h))

    def load(self, ids: torch.Tensor, flags: torch.Tensor, t: int, dists: torch.Tensor | None = None):
        """Load a state; with ``dists`` (as exported) the keys are kept bit
        for bit, without them the distances are recomputed."""
        ids = ids.to(device=self.X.device, dtype=torch.int32).contiguous()
        flags = flags.to(device=self.X.device, dtype=torch.uint8).contiguous()
        dp = None
        if dists is not None:
            dists = dists.to(device=self.X.device, dtype=torch.float32).contiguous()
            dp = ctypes.c_void_p(dists.data_ptr())
        _check(lib.knng_load_graph(self._h, ctypes.c_void_p(ids.data_ptr()), dp, ctypes.c_void_p(flags.data_ptr()),
                                   t))
        torch.cuda.current_stream(self.X.device).synchronize()

    def iterate(self) -> tuple[int, int]:
        e, c = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib.knng_iterate(self._h, ctypes.byref(e), ctypes.byref(c)))
        return int(e.value), int(c.value)

    def export(self) -> Graph:
        dev = self.X.device
        ids = torch.empty((self.N, self.K), dtype=torch.int32, device=dev)
        dists = torch.empty((self.N, self.K), dtype=torch.float32, device=dev)
        flags = torch.empty((self.N, self.K), dtype=torch.uint8, device=dev)
        _check(lib.knng_export(self._h, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dists.data_ptr()),
                               ctypes.c_void_p(flags.data_ptr())))
        return Graph(ids, dists, flags)

    def samples(self):
        dev = self.X.device
        C = self.C
        nw = torch.empty((self.N, C), dtype=torch.int32, device=dev)
        od = torch.empty((self.N, C), dtype=torch.int32, device=dev)
        cnt = torch.empty((self.N, 2), dtype=torch.int32, device=dev)
        _check(lib.knng_export_samples(self._h, ctypes.c_void_p(nw.data_ptr()), ctypes.c_void_p(od.data_ptr()),
                                       ctypes.c_void_p(cnt.data_ptr())))
        return nw, od, cnt

    def order(self) -> torch.Tensor:
        """Original id stored at each position (the permutation, once applied)."""
        o = torch.empty(self.N, dtype=torch.int32, device=self.X.device)
        _check(lib.knng_export_order(self._h, ctypes.c_void_p(o.data_ptr())))
        return o

    def stats(self) -> dict:
        s = _Stats()
        _check(lib.knng_get_stats(self._h, ctypes.byref(s)))
        return _stats_dict(s)


# ----------------------------------------------------------------------------- batched form

class _Dataset(ctypes.Structure):
    _fields_ = [("dX", ctypes.c_void_p), ("N", ctypes.c_int64), ("d", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64), ("d_ids", ctypes.c_void_p),
                ("d_dists", ctypes.c_void_p)]


def _load_batch(L):
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    PD, PP = ctypes.POINTER(_Dataset), ctypes.POINTER(Params)
    L.knng_batch_workspace_bytes.argtypes = [PD, i32, PP]
    L.knng_batch_workspace_bytes.restype = ctypes.c_size_t
    L.knng_batch_plan.argtypes = [ctypes.POINTER(P), PD, i32, PP, P, ctypes.c_size_t, ctypes.c_char_p, P]
    L.knng_batch_tuning.argtypes = [P]
    L.knng_batch_tuning.restype = ctypes.c_char_p
    L.knng_batch_execute.argtypes = [P, P]
    L.knng_batch_capture.argtypes = [P, P]
    L.knng_batch_launch.argtypes = [P, P]
    L.knng_batch_stats.argtypes = [P, P, P, P, P, P]
    L.knng_batch_destroy.argtypes = [P]
    L.knng_batch_destroy.restype = None
    for n in ("knng_batch_plan", "knng_batch_execute", "knng_batch_capture", "knng_batch_launch",
              "knng_batch_stats"):
        getattr(L, n).restype = ctypes.c_int


_load_batch(lib)


class Batch:
    """Many independent datasets built together (one graph launch once captured).

    ``Xs``: list of device float32 [N_i, d_i] tensors; ``seeds``: one seed per
    dataset. ``tuning``: None/"auto" runs the autotuner, or a table such as
    "16:valu,64:mfma@2048,128:mfma" (join path per d, optional workgroup cap
    of the select and join passes). Work is ordered on ``stream`` (a non-default
    torch stream; one is created when not given).
    """

    def __init__(self, Xs, seeds, K: int, rho: float = 1.0, delta: float = 0.001, max_iters: int = 30,
                 path: str | int = "auto", tuning: str | None = None, stream=None,
                 sampling: str | int = "weighted"):
        if len(Xs) != len(seeds) or not Xs:
            raise ValueError("one seed per dataset")
        for X in Xs:
            _check_x(X)
        dev = Xs[0].device
        self.Xs = Xs
        self.K = K
        self.max_iters = max_iters
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.ids = [torch.empty((X.shape[0], K), dtype=torch.int32, device=dev) for X in Xs]
        self.dists = [torch.empty((X.shape[0], K), dtype=torch.float32, device=dev) for X in Xs]
        n = len(Xs)
        self._descs = (_Dataset * n)()
        for i, (X, s) in enumerate(zip(Xs, seeds)):
            self._descs[i] = _Dataset(X.data_ptr(), X.shape[0], X.shape[1], 0, int(s) & 0xFFFFFFFFFFFFFFFF,
                                      self.ids[i].data_ptr(), self.dists[i].data_ptr())
        self.params = make_params(K, rho, delta, max_iters, 0, False, path, sampling=sampling)
        nb = int(lib.knng_batch_workspace_bytes(self._descs, n, ctypes.byref(self.params)))
        if nb == 0:
            raise KnngError(EINVAL, _err())
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        torch.cuda.current_stream(dev).synchronize()
        _check(lib.knng_batch_plan(ctypes.byref(h), self._descs, n, ctypes.byref(self.params),
                                   ctypes.c_void_p(self.ws.data_ptr()), nb,
                                   (tuning or "auto").encode(), ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self.captured = False
        # the kernels use these buffers on self.stream: the caching allocator
        # must not hand their memory out again before that work is done
        for t in (self.ws, *self.ids, *self.dists, *self.Xs):
            t.record_stream(self.stream)

    @property
    def tuning(self) -> str:
        return lib.knng_batch_tuning(self._h).decode()

    def _order_after(self):
        # work the caller queues next on its current stream (reading ids and
        # dists, say) runs after the build
        ev = torch.cuda.Event()
        ev.record(self.stream)
        torch.cuda.current_stream(self.ws.device).wait_event(ev)

    def execute(self):
        _check(lib.knng_batch_execute(self._h, ctypes.c_void_p(self.stream.cuda_stream)))
        self._order_after()

    def capture(self):
        _check(lib.knng_batch_capture(self._h, ctypes.c_void_p(self.stream.cuda_stream)))
        self.captured = True

    def launch(self):
        _check(lib.knng_batch_launch(self._h, ctypes.c_void_p(self.stream.cuda_stream)))
        self._order_after()

    def synchronize(self):
        self.stream.synchronize()

    def stats(self) -> dict:
        import numpy as np
        n, T = len(self.Xs), self.max_iters
        it = np.zeros(n, np.int32)
        cv = np.zeros(n, np.int32)
        ev = np.zeros((n, T), np.int64)
        ch = np.zeros((n, T), np.int64)
        _check(lib.knng_batch_stats(self._h, it.ctypes.data, cv.ctypes.data, ev.ctypes.data, ch.ctypes.data,
                                    ctypes.c_void_p(self.stream.cuda_stream)))
        return dict(iters=it, converged=cv, evals=[list(ev[i, :it[i]]) for i in range(n)],
                    changes=[list(ch[i, :it[i]]) for i in range(n)])

    def close(self):
        if getattr(self, "_h", None):
            self.stream.synchronize()   # no launch of the plan's graph is still running
            lib.knng_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
