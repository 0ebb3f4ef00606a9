"""Python binding of the C ABI in ``include/stiles.h`` (argument marshalling only).

Every step of the factorization and of the selected inversion runs in the HIP
kernels of ``libstiles.so``; PyTorch only provides device memory and the
stream.  The library must have been built (``__graft_entry__.build()``):
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libstiles.so")

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t

STILES_EHIP = -100
STILES_ETIMEOUT = -101
STILES_EBADL = -102

EXPORTED = (
    "stiles_layout_init",
    "stiles_selection_closure",
    "stiles_pack",
    "stiles_factor_workspace_bytes",
    "stiles_selinv_workspace_bytes",
    "stiles_factor",
    "stiles_selinv",
    "stiles_strerror",
    "stiles_version",
    "stiles_timing_enable",
    "stiles_timing_collect",
    "stiles_batch_workspace_bytes",
    "stiles_factor_batched",
    "stiles_selinv_batched",
    "stiles_trace_workspace_bytes",
    "stiles_trace_product",
    "stiles_inverse_workspace_bytes",
    "stiles_inverse",
    "stiles_selinv_range",
    "stiles_gather",
    "stiles_mfma_peak",
    "stiles_batch_upload",
    "stiles_factor_batched_enqueue",
    "stiles_selinv_batched_enqueue",
)

TIMING_KINDS = ("potrf", "trsm", "update", "phase1", "phase2", "factor", "other")


class _CLayout(ctypes.Structure):
    _fields_ = [
        ("n", _i64), ("bandwidth", _i64), ("arrow", _i64),
        ("tile", _i32), ("bt", _i32),
        ("nb", _i64), ("w", _i64), ("nt", _i64),
        ("arrow_ld", _i32), ("reserved", _i32),
        ("off_band", _i64), ("off_arrow", _i64), ("off_corner", _i64),
        ("total_doubles", _i64),
    ]


class _CBatchItem(ctypes.Structure):
    _fields_ = [
        ("n", _i64), ("bandwidth", _i64), ("arrow", _i64),
        ("tile", _i32), ("reserved", _i32),
        ("A", _vp), ("L", _vp), ("Sigma", _vp), ("logdet", _vp), ("info", _vp),
    ]


_lib = None


class StilesError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


def load(path: Optional[str] = None):
    """Load libstiles.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBPATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    lib.stiles_layout_init.argtypes = [_i64, _i64, _i64, _i32, ctypes.POINTER(_CLayout)]
    lib.stiles_layout_init.restype = ctypes.c_int
    lib.stiles_pack.argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i32, _vp]
    lib.stiles_pack.restype = ctypes.c_int
    lib.stiles_factor_workspace_bytes.argtypes = [ctypes.POINTER(_CLayout)]
    lib.stiles_factor_workspace_bytes.restype = _sz
    lib.stiles_selinv_workspace_bytes.argtypes = [ctypes.POINTER(_CLayout)]
    lib.stiles_selinv_workspace_bytes.restype = _sz
    lib.stiles_factor.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, _vp, _vp, _vp, _sz, _vp]
    lib.stiles_factor.restype = ctypes.c_int
    lib.stiles_selinv.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, _vp, _vp, _sz, _vp]
    lib.stiles_selinv.restype = ctypes.c_int
    lib.stiles_strerror.argtypes = [ctypes.c_int]
    lib.stiles_strerror.restype = ctypes.c_char_p
    lib.stiles_timing_enable.argtypes = [ctypes.c_int]
    lib.stiles_timing_enable.restype = ctypes.c_int
    lib.stiles_timing_collect.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    lib.stiles_timing_collect.restype = ctypes.c_int
    lib.stiles_version.argtypes = []
    lib.stiles_version.restype = ctypes.c_int
    lib.stiles_inverse_workspace_bytes.argtypes = [ctypes.POINTER(_CLayout)]
    lib.stiles_inverse_workspace_bytes.restype = _sz
    lib.stiles_inverse.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, _vp, _vp, _sz, _vp]
    lib.stiles_inverse.restype = ctypes.c_int
    lib.stiles_selinv_range.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, _i64, _vp, _vp, _sz, _vp]
    lib.stiles_selinv_range.restype = ctypes.c_int
    lib.stiles_gather.argtypes = [_vp, _i64, _i64, _i64, _i32, _vp, _i64, _vp, _vp]
    lib.stiles_gather.restype = ctypes.c_int
    lib.stiles_trace_workspace_bytes.argtypes = []
    lib.stiles_trace_workspace_bytes.restype = _sz
    lib.stiles_trace_product.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, _vp, _vp, _sz, _vp]
    lib.stiles_trace_product.restype = ctypes.c_int
    lib.stiles_mfma_peak.argtypes = [_vp, _i64, _i32, ctypes.POINTER(ctypes.c_double), _vp]
    lib.stiles_mfma_peak.restype = ctypes.c_int
    lib.stiles_batch_workspace_bytes.argtypes = [ctypes.POINTER(_CBatchItem), _i32]
    lib.stiles_batch_workspace_bytes.restype = _sz
    lib.stiles_factor_batched.argtypes = [ctypes.POINTER(_CBatchItem), _i32, _vp, _sz, _vp]
    lib.stiles_factor_batched.restype = ctypes.c_int
    lib.stiles_selinv_batched.argtypes = [ctypes.POINTER(_CBatchItem), _i32, _vp, _sz, _vp]
    lib.stiles_selinv_batched.restype = ctypes.c_int
    for name in ("stiles_batch_upload", "stiles_factor_batched_enqueue", "stiles_selinv_batched_enqueue"):
        getattr(lib, name).argtypes = [ctypes.POINTER(_CBatchItem), _i32, _vp, _sz, _vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.stiles_selection_closure.argtypes = [_i64, _i64, _i64, _i32, _vp, _i64, ctypes.POINTER(_i32),
                                             ctypes.POINTER(_i64)]
    lib.stiles_selection_closure.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().stiles_strerror(int(code)).decode()


@dataclass(frozen=True)
class Layout:
    """Tile layout of one matrix (mirror of ``stiles_layout``)."""
    n: int
    bandwidth: int
    arrow: int
    tile: int
    bt: int
    nb: int
    w: int
    nt: int
    arrow_ld: int
    off_band: int
    off_arrow: int
    off_corner: int
    total_doubles: int

    def _c(self) -> _CLayout:
        c = _CLayout()
        rc = load().stiles_layout_init(self.n, self.bandwidth, self.arrow, self.tile, ctypes.byref(c))
        assert rc == 0
        return c

    @property
    def factor_workspace_bytes(self) -> int:
        return int(load().stiles_factor_workspace_bytes(ctypes.byref(self._c())))

    @property
    def selinv_workspace_bytes(self) -> int:
        return int(load().stiles_selinv_workspace_bytes(ctypes.byref(self._c())))


def layout(n: int, bandwidth: int, arrow: int, tile: int) -> Layout:
    c = _CLayout()
    rc = load().stiles_layout_init(int(n), int(bandwidth), int(arrow), int(tile), ctypes.byref(c))
    if rc != 0:
        raise StilesError(rc, "stiles_layout_init")
    return Layout(c.n, c.bandwidth, c.arrow, c.tile, c.bt, c.nb, c.w, c.nt, c.arrow_ld,
                  c.off_band, c.off_arrow, c.off_corner, c.total_doubles)


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _on(stream):
    """Context in which the wrappers allocate their outputs and temporaries:
    the stream the kernels are enqueued on, so the caching allocator never hands
    a temporary's memory to other work while those kernels may still use it."""
    import contextlib
    import torch
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _dev_f64(x, name: str):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return x


def pack(ab, arrow_rows, corner, lay: Layout, out=None, stream=None):
    """Pack device arrays in canonical band form into a new tile buffer."""
    with _on(stream):
        import torch
        ab = _dev_f64(ab, "ab")
        dev = ab.device
        if out is None:
            out = torch.empty(lay.total_doubles, dtype=torch.float64, device=dev)
        P = _dev_f64(arrow_rows, "arrow_rows").data_ptr() if lay.arrow else None
        C = _dev_f64(corner, "corner").data_ptr() if lay.arrow else None
        rc = load().stiles_pack(ab.data_ptr(), P, C, out.data_ptr(), lay.n, lay.bandwidth, lay.arrow,
                                lay.tile, _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_pack")
        return out


def factor(A, lay: Layout, out=None, workspace=None, stream=None) -> Tuple[object, object, object]:
    """Cholesky factor (tile layout) of A; returns (L, logdet, info) on the device.

    ``out`` may be ``A`` itself (in place).  logdet is a 1-element float64
    tensor and info a 1-element int32 tensor; neither is synchronised.
    """
    with _on(stream):
        import torch
        A = _dev_f64(A, "A")
        dev = A.device
        L = out if out is not None else torch.empty_like(A)
        ws = workspace
        if ws is None:
            ws = torch.empty(lay.factor_workspace_bytes, dtype=torch.uint8, device=dev)
        logdet = torch.empty(1, dtype=torch.float64, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        rc = load().stiles_factor(A.data_ptr(), L.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                  logdet.data_ptr(), info.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_factor")
        return L, logdet, info


def selinv(L, lay: Layout, out=None, workspace=None, stream=None):
    """Sigma = A^{-1} on the tile pattern of L; returns (Sigma, info) on the device."""
    with _on(stream):
        import torch
        L = _dev_f64(L, "L")
        dev = L.device
        S = out if out is not None else torch.empty_like(L)
        ws = workspace
        if ws is None:
            ws = torch.empty(lay.selinv_workspace_bytes, dtype=torch.uint8, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        rc = load().stiles_selinv(L.data_ptr(), S.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                  info.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_selinv")
        return S, info


def mfma_peak(iters: int = 4096, stream=None) -> Tuple[float, float]:
    """Launch the FP64 matrix-core throughput probe on the current device;
    returns (flops, elapsed ms) measured with events on the launch's stream."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    with _on(stream):
        n = 512 * torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        sink = torch.empty(n, dtype=torch.float64, device="cuda")
        flops = ctypes.c_double(0.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        rc = load().stiles_mfma_peak(sink.data_ptr(), n, int(iters), ctypes.byref(flops), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_mfma_peak")
        e1.record(s)
        e1.synchronize()
        return flops.value, e0.elapsed_time(e1)


def timing_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events (per-kernel timing)."""
    load().stiles_timing_enable(1 if on else 0)


def timing_collect() -> dict:
    """{kind: (total_ms, launches)} since the last collect (waits for the events)."""
    n = len(TIMING_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (_i64 * n)()
    rc = load().stiles_timing_collect(ms, cnt)
    if rc != 0:
        raise StilesError(rc, "stiles_timing_collect")
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(TIMING_KINDS)}


# ---------------------------------------------------------------------------
# Batched form (stiles_factor_batched / stiles_selinv_batched)
# ---------------------------------------------------------------------------

def _batch_items(lays, As=None, Ls=None, Sigmas=None, logdet=None, info=None):
    items = (_CBatchItem * len(lays))()
    for k, lay in enumerate(lays):
        it = items[k]
        it.n, it.bandwidth, it.arrow, it.tile, it.reserved = lay.n, lay.bandwidth, lay.arrow, lay.tile, 0
        L = Ls[k] if Ls is not None else None
        it.A = (As[k] if As is not None else L).data_ptr() if (As is not None or L is not None) else None
        it.L = L.data_ptr() if L is not None else it.A
        it.Sigma = Sigmas[k].data_ptr() if Sigmas is not None else None
        it.logdet = logdet.data_ptr() + 8 * k if logdet is not None else None
        it.info = info.data_ptr() + 8 * k if info is not None else None
    return items


def batch_workspace_bytes(lays) -> int:
    """Workspace bytes for a batch of matrices with these layouts (factor and selinv)."""
    items = (_CBatchItem * len(lays))()
    for k, lay in enumerate(lays):
        it = items[k]
        it.n, it.bandwidth, it.arrow, it.tile, it.reserved = lay.n, lay.bandwidth, lay.arrow, lay.tile, 0
        it.A = it.L = it.Sigma = it.logdet = it.info = 1   # only the layouts are read
    nbytes = int(load().stiles_batch_workspace_bytes(items, len(lays)))
    if nbytes == 0:
        raise ValueError("invalid batch")
    return nbytes


def factor_batched(As, lays, outs=None, workspace=None, info=None, stream=None, logdet=None, enqueue_only=False):
    """Cholesky factors of a batch; returns (Ls, logdet[count], info[count, 2]) on the device.

    ``outs[k]`` may be ``As[k]`` (in place).  ``info[:, 0]`` is each matrix's
    factor info (as :func:`factor`); column 1 is left for :func:`selinv_batched`.
    enqueue_only: device work only, from the tables :func:`batch_upload` wrote
    for the same matrices (``stiles_factor_batched_enqueue``; capturable).
    """
    with _on(stream):
        import torch
        As = [_dev_f64(x, "A") for x in As]
        dev = As[0].device
        Ls = outs if outs is not None else [torch.empty_like(x) for x in As]
        ws = workspace if workspace is not None else torch.empty(batch_workspace_bytes(lays), dtype=torch.uint8,
                                                                 device=dev)
        if logdet is None:
            logdet = torch.empty(len(As), dtype=torch.float64, device=dev)
        if info is None:
            info = torch.zeros((len(As), 2), dtype=torch.int32, device=dev)
        items = _batch_items(lays, As=As, Ls=Ls, logdet=logdet, info=info)
        fn = load().stiles_factor_batched_enqueue if enqueue_only else load().stiles_factor_batched
        rc = fn(items, len(As), ws.data_ptr(), ws.numel(), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_factor_batched")
        return Ls, logdet, info


def batch_upload(lays, As, Ls, Ss, logdet, info, workspace, stream=None):
    """Copy the tables of both batched calls for these matrices into the
    workspace (``stiles_batch_upload``), ahead of enqueue-only calls."""
    with _on(stream):
        items = _batch_items(lays, As=As, Ls=Ls, Sigmas=Ss, logdet=logdet, info=info)
        rc = load().stiles_batch_upload(items, len(lays), workspace.data_ptr(), workspace.numel(),
                                        _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_batch_upload")


def selinv_batched(Ls, lays, outs=None, workspace=None, info=None, stream=None, As=None, logdet=None,
                   enqueue_only=False):
    """Sigma on the tile pattern of every L of a batch; returns (Sigmas, info[count, 2]).

    ``info[:, 1]`` receives each matrix's selinv info (as :func:`selinv`).
    enqueue_only: device work only (``stiles_selinv_batched_enqueue``), from
    the tables :func:`batch_upload` wrote; the tensors must then be those given
    to that upload.
    """
    with _on(stream):
        import torch
        Ls = [_dev_f64(x, "L") for x in Ls]
        dev = Ls[0].device
        Ss = outs if outs is not None else [torch.empty_like(x) for x in Ls]
        ws = workspace if workspace is not None else torch.empty(batch_workspace_bytes(lays), dtype=torch.uint8,
                                                                 device=dev)
        if info is None:
            info = torch.zeros((len(Ls), 2), dtype=torch.int32, device=dev)
        dummy = logdet if logdet is not None else torch.empty(len(Ls), dtype=torch.float64, device=dev)
        items = _batch_items(lays, As=As, Ls=Ls, Sigmas=Ss, logdet=dummy, info=info)
        fn = load().stiles_selinv_batched_enqueue if enqueue_only else load().stiles_selinv_batched
        rc = fn(items, len(Ls), ws.data_ptr(), ws.numel(), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_selinv_batched")
        return Ss, info


def trace_product(Sigma, B, lay: Layout, out=None, workspace=None, stream=None):
    """sum_ij Sigma_ij B_ij over the real entries of the tile pattern (a
    1-element device tensor): tr(A^{-1} B) for Sigma from :func:`selinv` and B
    packed by :func:`pack` with its pattern inside L's."""
    with _on(stream):
        import torch
        Sigma = _dev_f64(Sigma, "Sigma")
        B = _dev_f64(B, "B")
        dev = Sigma.device
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=dev)
        ws = workspace if workspace is not None else torch.empty(int(load().stiles_trace_workspace_bytes()),
                                                                 dtype=torch.uint8, device=dev)
        rc = load().stiles_trace_product(Sigma.data_ptr(), B.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                         out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_trace_product")
        return out


def inverse(L, lay: Layout, out=None, workspace=None, stream=None):
    """Every entry of A^{-1} (n x n, column-major, full symmetric) from the factor L;
    returns (Ainv, info) on the device."""
    with _on(stream):
        import torch
        L = _dev_f64(L, "L")
        dev = L.device
        n = lay.n
        Ainv = out if out is not None else torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = workspace
        if ws is None:
            ws = torch.empty(int(load().stiles_inverse_workspace_bytes(ctypes.byref(lay._c()))), dtype=torch.uint8,
                             device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        rc = load().stiles_inverse(L.data_ptr(), Ainv.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                   info.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_inverse")
        return Ainv, info


def selinv_range(L, lay: Layout, first_column: int, out=None, workspace=None, stream=None):
    """:func:`selinv` restricted to the tile columns >= first_column (and the corner)."""
    with _on(stream):
        import torch
        L = _dev_f64(L, "L")
        S = out if out is not None else torch.empty_like(L)
        ws = workspace if workspace is not None else torch.empty(lay.selinv_workspace_bytes, dtype=torch.uint8,
                                                                 device=L.device)
        info = torch.empty(1, dtype=torch.int32, device=L.device)
        rc = load().stiles_selinv_range(L.data_ptr(), S.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                        int(first_column), info.data_ptr(), ws.data_ptr(), ws.numel(),
                                        _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_selinv_range")
        return S, info


def gather(Sigma, lay: Layout, ij, out=None, stream=None):
    """Sigma(i, j) for the pairs ij (a (k, 2) int64 device tensor) read off the tile layout."""
    with _on(stream):
        import torch
        Sigma = _dev_f64(Sigma, "Sigma")
        ij = ij.contiguous()
        if ij.dtype != torch.int64 or not ij.is_cuda or ij.dim() != 2 or ij.shape[1] != 2:
            raise TypeError("ij must be a (k, 2) int64 CUDA tensor")
        k = ij.shape[0]
        if out is None:
            out = torch.empty(k, dtype=torch.float64, device=Sigma.device)
        rc = load().stiles_gather(Sigma.data_ptr(), lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                  ij.data_ptr() if k else None, k, out.data_ptr() if k else None, _stream_handle(stream))
        if rc != 0:
            raise StilesError(rc, "stiles_gather")
        return out


def selection_closure(lay: Layout, pairs):
    """Symbolic step of a selection (Sec. III-B) through stiles_selection_closure:
    for pairs (i, j) -> (whether every pair lies in the tile pattern of L, the
    first tile column of the closure; N when only the corner is selected)."""
    import numpy as np
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    inside = _i32(0)
    first = _i64(0)
    rc = load().stiles_selection_closure(lay.n, lay.bandwidth, lay.arrow, lay.tile,
                                         p.ctypes.data if len(p) else None, len(p),
                                         ctypes.byref(inside), ctypes.byref(first))
    if rc == -5:
        raise ValueError("pair outside the matrix")
    if rc != 0:
        raise StilesError(rc, "stiles_selection_closure")
    return bool(inside.value), int(first.value)


def select(L, lay: Layout, pairs, stream=None):
    """Sigma(i, j) for a list of pairs: when they all lie in the tile pattern of L,
    the selected inverse of their closure only (stiles_selinv_range) read with
    stiles_gather; otherwise the full inverse.  Returns (values, info) on the device."""
    with _on(stream):
        import numpy as np
        import torch
        inside, first = selection_closure(lay, pairs)
        ij = torch.as_tensor(np.asarray(pairs, dtype=np.int64).reshape(-1, 2), device=L.device)
        if inside:
            S, info = selinv_range(L, lay, first, stream=stream)
            return gather(S, lay, ij, stream=stream), info
        X, info = inverse(L, lay, stream=stream)
        return X.t()[ij[:, 0], ij[:, 1]], info
