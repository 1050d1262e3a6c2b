"""cmsvd: incremental concatenated-SVD merge-error engine for MI355X (gfx950).

Thin ctypes binding over ``libcmsvd.so`` (built from ``csrc/`` by ``build.py``).  The
functions mirror the C ABI in ``include/cmsvd.h``; they only marshal torch tensors
(device memory and the current HIP stream) into the C calls.  Every step of the
computation runs in the HIP kernels of the library; there is no CPU fallback, and
importing this package raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmsvd.so")

CMSVD_F32 = 0
CMSVD_BF16 = 1
CMSVD_F64 = 2
_STATUS = {0: "OK", 1: "EINVAL", 2: "ESHAPE", 3: "ENOMEM", 4: "EHIP", 5: "EUNSUPPORTED"}


class CmsvdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cmsvd {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Block(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2601_11626_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.cmsvd_create.argtypes = [ctypes.POINTER(vp), vp]
    lib.cmsvd_create_ex.argtypes = [ctypes.POINTER(vp), vp, vp, vp, vp, vp]
    lib.cmsvd_destroy.argtypes = [vp]
    lib.cmsvd_set_stream.argtypes = [vp, vp]
    lib.cmsvd_last_error.restype = ctypes.c_char_p
    lib.cmsvd_update.argtypes = [vp, i64, vp, i64, vp, i64, ctypes.POINTER(Block), i64, vp, i64, vp, vp, vp]
    lib.cmsvd_merge_errors.argtypes = [vp, ctypes.POINTER(Block), i64, vp, i64, i64, vp, vp]
    lib.cmsvd_cluster.argtypes = [vp, ctypes.POINTER(Block), i64, i64, d, i32, vp, ctypes.POINTER(i64), vp]
    lib.cmsvd_sym_eigvals.argtypes = [vp, vp, i64, i64, i64, i64, i64, vp]
    lib.cmsvd_sym_eigvals_noalloc.argtypes = [vp, vp, i64, i64, i64, i64, i64, vp]
    lib.cmsvd_gemm_f64.argtypes = [vp, i32, i32, i64, i64, i64, d, vp, i64, i32, vp, i64, i32, d, vp, i64]
    lib.cmsvd_gemm_bf16.argtypes = [vp, i32, i32, i32, i64, i64, i64, d, vp, i64, i32, vp, i64, i32, d, vp, i64]
    lib.cmsvd_gemm_f32.argtypes = [vp, i32, i32, i64, i64, i64, d, vp, i64, i32, vp, i64, i32, d, vp, i64]
    lib.cmsvd_set_projection.argtypes = [vp, i32]
    lib.cmsvd_profile.argtypes = [vp, i32]
    lib.cmsvd_profile_read.argtypes = [vp, vp, vp]
    lib.cmsvd_update_batch.argtypes = [vp, i64, i64, vp, i64, vp, i64, ctypes.POINTER(Block), i64, vp, i64, vp, vp, vp]
    lib.cmsvd_cluster_residual.argtypes = [vp, ctypes.POINTER(Block), i64, i64, d, i32, vp, ctypes.POINTER(i64), vp]
    lib.cmsvd_residual_bound.argtypes = [vp, ctypes.POINTER(Block), i64, i64, ctypes.POINTER(d), vp]
    lib.cmsvd_weyl_bound.argtypes = [vp, ctypes.POINTER(Block), i64, i64, ctypes.POINTER(d)]
    lib.cmsvd_cluster_weyl.argtypes = [vp, ctypes.POINTER(Block), i64, i64, d, vp, ctypes.POINTER(i64), vp]
    lib.cmsvd_exact_tail.argtypes = [vp, ctypes.POINTER(Block), i64, i64, ctypes.POINTER(d)]
    lib.cmsvd_compress.argtypes = [vp, ctypes.POINTER(Block), i64, i64, vp, i64, vp, i64, ctypes.POINTER(i64),
                                   ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.cmsvd_cluster_trace.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    lib.cmsvd_graph_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(d)]
    lib.cmsvd_autotune.argtypes = [vp, i64, i64, i64, ctypes.c_char_p, i32, ctypes.POINTER(i64)]
    lib.cmsvd_compress_partition.argtypes = [vp, ctypes.POINTER(Block), i64, vp, i64, vp, vp, vp, vp, vp, vp, vp,
                                             ctypes.POINTER(i64), ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.cmsvd_tail_energy_grad.argtypes = [vp, ctypes.POINTER(Block), i64, i64, i64, ctypes.POINTER(d), vp,
                                           ctypes.POINTER(d)]
    for f in ("cmsvd_create", "cmsvd_destroy", "cmsvd_set_stream", "cmsvd_update", "cmsvd_merge_errors",
              "cmsvd_cluster", "cmsvd_sym_eigvals", "cmsvd_gemm_f64", "cmsvd_profile", "cmsvd_profile_read",
              "cmsvd_tail_energy_grad", "cmsvd_update_batch", "cmsvd_cluster_residual", "cmsvd_residual_bound",
              "cmsvd_weyl_bound", "cmsvd_cluster_weyl", "cmsvd_exact_tail", "cmsvd_compress", "cmsvd_gemm_bf16",
              "cmsvd_set_projection", "cmsvd_sym_eigvals_noalloc", "cmsvd_gemm_f32", "cmsvd_create_ex",
              "cmsvd_compress_partition", "cmsvd_cluster_trace", "cmsvd_graph_stats", "cmsvd_autotune"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = _load()

EXPORTS = ("cmsvd_create", "cmsvd_destroy", "cmsvd_set_stream", "cmsvd_last_error", "cmsvd_update",
           "cmsvd_merge_errors", "cmsvd_cluster", "cmsvd_sym_eigvals", "cmsvd_gemm_f64", "cmsvd_profile",
           "cmsvd_profile_read", "cmsvd_tail_energy_grad", "cmsvd_update_batch", "cmsvd_cluster_residual",
           "cmsvd_residual_bound", "cmsvd_weyl_bound", "cmsvd_cluster_weyl", "cmsvd_exact_tail", "cmsvd_compress",
           "cmsvd_gemm_bf16", "cmsvd_set_projection", "cmsvd_sym_eigvals_noalloc", "cmsvd_gemm_f32",
           "cmsvd_create_ex", "cmsvd_compress_partition", "cmsvd_cluster_trace", "cmsvd_graph_stats",
           "cmsvd_autotune")

PROJECTIONS = {"f64": 0, "bf16": 1, "bf16x3": 2, "f32": 3}  # cmsvd_projection

STAGES = ("norms_grams", "commit", "projection", "core_eig", "core_bisect", "core_tail")


def _check(status: int):
    if status != 0:
        raise CmsvdError(status, _lib.cmsvd_last_error().decode(errors="replace"))


def _stream_ptr(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Options(ctypes.Structure):
    """cmsvd_options (zero = the defaults)."""
    _fields_ = [("projection", ctypes.c_int32), ("chol_tau", ctypes.c_double), ("panel_cols", ctypes.c_int64),
                ("graphs", ctypes.c_int32)]


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _torch_allocator(device_index: int, stream):
    """The allocator callbacks of cmsvd_create_ex on PyTorch's caching allocator (blocks
    tied to the handle's stream)."""

    def alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device_index, stream)
        except Exception:  # out of memory: the library reports CMSVD_ENOMEM
            return None

    def release(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return _ALLOC_T(alloc), _RELEASE_T(release)


class Handle:
    """Owns a cmsvd handle bound to the current torch stream of ``device``.

    ``projection``, ``chol_tau``, ``panel_cols`` and ``graphs`` are the handle options
    (cmsvd_options); with ``torch_allocator`` (the default) the library's device memory
    comes from PyTorch's caching allocator."""

    def __init__(self, device=None, projection: str = "f64", chol_tau: float = 0.0, panel_cols: int = 0,
                 graphs: bool = False, torch_allocator: bool = True):
        self._h = ctypes.c_void_p()
        self._cb = None
        self.projection = projection
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index)
        opts = Options(PROJECTIONS[projection], float(chol_tau), int(panel_cols), 1 if graphs else 0)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            if torch_allocator:
                self._cb = _torch_allocator(self.device.index, stream)
                alloc, release = self._cb
            else:
                alloc, release = _ALLOC_T(), _RELEASE_T()
            _check(_lib.cmsvd_create_ex(ctypes.byref(self._h), ctypes.c_void_p(stream.cuda_stream),
                                        ctypes.byref(opts), alloc, release, None))

    def sync_stream(self):
        _check(_lib.cmsvd_set_stream(self._h, _stream_ptr(self.device)))

    def close(self):
        if self._h:
            _lib.cmsvd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):  # pragma: no cover
        if _finalizing():  # the allocator callbacks cannot run any more: leave it to the process exit
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def set_projection(self, precision: str):
        """'f64' (default), 'bf16', 'bf16x3' or 'f32': precision of the candidate projections
        Y = U_r^T A_j."""
        _check(_lib.cmsvd_set_projection(self._h, PROJECTIONS[precision]))
        self.projection = precision

    def call_with_projection(self, precision, fn):
        """Runs fn() with the projection precision set to ``precision`` (None: as set)."""
        if precision is None or precision == self.projection:
            return fn()
        prev = self.projection
        self.set_projection(precision)
        try:
            return fn()
        finally:
            self.set_projection(prev)

    def graph_stats(self) -> dict:
        """Captured sequences, graph replays and the last capture's wall time (ms)."""
        c, rp, ms = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_double(0.0)
        _check(_lib.cmsvd_graph_stats(self._h, ctypes.byref(c), ctypes.byref(rp), ctypes.byref(ms)))
        return {"captures": c.value, "replays": rp.value, "last_capture_ms": ms.value}

    def autotune(self, m: int, k: int, r: int, cache_path: str | None = None, force: bool = False) -> int:
        """Tunes (or loads from cache_path) the first scan chunk of Algorithm 3 for
        width-k candidates on rank-r states of m rows; returns the chunk chosen."""
        c = ctypes.c_int64(0)
        _check(_lib.cmsvd_autotune(self._h, m, k, r, cache_path.encode() if cache_path else None,
                                   1 if force else 0, ctypes.byref(c)))
        return c.value

    def profile(self, enable: bool = True):
        _check(_lib.cmsvd_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """Per-stage (milliseconds, launches) since the last read; synchronises the stream."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(_lib.cmsvd_profile_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}


_default: dict = {}


def default_handle(device=None) -> Handle:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    h = _default.get(dev)
    if h is None:
        h = _default[dev] = Handle(dev)
    h.sync_stream()
    return h


def _block(t: torch.Tensor) -> Block:
    if not t.is_cuda:
        raise ValueError("blocks must be device tensors")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("blocks must be 2-D with unit column stride (row-major)")
    if t.dtype == torch.float32:
        dt = CMSVD_F32
    elif t.dtype == torch.float64:
        dt = CMSVD_F64
    elif t.dtype == torch.bfloat16:
        dt = CMSVD_BF16
    else:
        raise ValueError(f"unsupported dtype {t.dtype}")
    return Block(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0), dt)


def _blocks(ts):
    if isinstance(ts, BlockArray):
        return ts.arr
    arr = (Block * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _block(t)
    return arr


class BlockArray:
    """The descriptors of a list of device blocks, marshalled once: pass it wherever a
    list of blocks is taken, for calls repeated over the same collection.  It keeps the
    tensors alive; they must not be resized or freed while it is in use."""

    def __init__(self, ts: Sequence[torch.Tensor]):
        self.tensors = list(ts)
        self.arr = (Block * len(self.tensors))()
        for i, t in enumerate(self.tensors):
            self.arr[i] = _block(t)

    def __len__(self):
        return len(self.tensors)

    def __getitem__(self, i):
        return self.tensors[i]

    def __iter__(self):
        return iter(self.tensors)


class State:
    """Device state of the estimator: basis U (m x r, FP64), singular values S (r),
    accumulators acc = [E_tot hi, E_tot lo, D hi, D lo] and est = [Etilde, sqrt(D)]."""

    def __init__(self, m: int, r: int, device):
        self.m, self.r = m, r
        self.U = torch.zeros((m, r), dtype=torch.float64, device=device)
        self.S = torch.zeros(r, dtype=torch.float64, device=device)
        self.acc = torch.zeros(4, dtype=torch.float64, device=device)
        self.est = torch.zeros(2, dtype=torch.float64, device=device)
        self.width = 0  # 0 = empty state


def cmsvd_update(state: State, B: torch.Tensor, r: int | None = None, handle: Handle | None = None) -> State:
    """One incremental step; returns a new State (the input state is not modified)."""
    h = handle or default_handle(B.device)
    r = state.r if r is None else r
    out = State(state.m, r, B.device)
    out.acc.copy_(state.acc)
    blk = _block(B)
    U = state.U if state.width else None
    _check(_lib.cmsvd_update(
        h.ptr, state.m,
        ctypes.c_void_p(U.data_ptr() if U is not None else 0), state.U.stride(0),
        ctypes.c_void_p(state.S.data_ptr() if U is not None else 0), state.width,
        ctypes.byref(blk), r,
        ctypes.c_void_p(out.U.data_ptr()), out.U.stride(0), ctypes.c_void_p(out.S.data_ptr()),
        ctypes.c_void_p(out.acc.data_ptr()), ctypes.c_void_p(out.est.data_ptr())))
    out.width = r
    return out


def cmsvd_update_batch(states: Sequence[State], blocks: Sequence[torch.Tensor], r: int | None = None,
                       handle: Handle | None = None) -> list:
    """One incremental step for each (state, block) pair, in one batched call (states of
    equal m, width and r, e.g. chains advanced in lockstep).  Returns new States."""
    n = len(states)
    if n != len(blocks):
        raise ValueError("states and blocks differ in length")
    if n == 0:
        return []
    h = handle or default_handle(blocks[0].device)
    s0 = states[0]
    r = s0.r if r is None else r
    outs = []
    for st in states:
        if st.m != s0.m or st.width != s0.width or st.U.stride(0) != s0.U.stride(0):
            raise ValueError("states must share m, width and layout")
        o = State(st.m, r, blocks[0].device)
        o.acc.copy_(st.acc)
        outs.append(o)
    P = ctypes.c_void_p * n
    arr = _blocks(blocks)
    U = P(*[st.U.data_ptr() for st in states]) if s0.width else None
    S = P(*[st.S.data_ptr() for st in states]) if s0.width else None
    _check(_lib.cmsvd_update_batch(
        h.ptr, n, s0.m, U, s0.U.stride(0), S, s0.width, arr, r,
        P(*[o.U.data_ptr() for o in outs]), outs[0].U.stride(0), P(*[o.S.data_ptr() for o in outs]),
        P(*[o.acc.data_ptr() for o in outs]), P(*[o.est.data_ptr() for o in outs])))
    for o in outs:
        o.width = r
    return outs


def cmsvd_merge_errors(blocks: Sequence[torch.Tensor], pairs, r: int, handle: Handle | None = None,
                       projection: str | None = None, out=None):
    """Returns (err, rel) device FP64 tensors for the ordered pairs (i, j).  projection:
    'f64', 'bf16', 'bf16x3' or 'f32' for this call (None: the handle's setting).  out:
    an (err, rel) pair of FP64 device tensors to write (repeated calls with the same
    outputs can be replayed from a captured graph, Handle(graphs=True))."""
    dev = blocks[0].device
    h = handle or default_handle(dev)
    if isinstance(pairs, torch.Tensor):
        pr = pairs.detach().to("cpu", torch.int32).contiguous()
    else:
        import numpy as np

        pr = torch.from_numpy(np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2)))
    npairs = pr.shape[0]
    if out is not None:
        err, rel = out
        if err.numel() != npairs or rel.numel() != npairs or err.dtype != torch.float64 or \
                rel.dtype != torch.float64 or not err.is_contiguous() or not rel.is_contiguous():
            raise ValueError("out must be two contiguous float64 tensors of npairs entries")
    else:
        err = torch.empty(npairs, dtype=torch.float64, device=dev)
        rel = torch.empty(npairs, dtype=torch.float64, device=dev)
    arr = _blocks(blocks)
    h.call_with_projection(projection, lambda: _check(_lib.cmsvd_merge_errors(
        h.ptr, arr, len(blocks), ctypes.c_void_p(pr.data_ptr()), npairs, r, ctypes.c_void_p(err.data_ptr()),
        ctypes.c_void_p(rel.data_ptr()))))
    return err, rel


def cmsvd_cluster(blocks: Sequence[torch.Tensor], r: int, eps: float, sort_mode: str = "frobenius",
                  handle: Handle | None = None, projection: str | None = None):
    """Algorithm 3 on the device.  Returns (labels list, clusters list, cluster_rel list).
    projection: 'f64', 'bf16', 'bf16x3' or 'f32' for the candidate evaluations of this call
    (None: the handle's setting)."""
    dev = blocks[0].device
    h = handle or default_handle(dev)
    mode = {"frobenius": 0, "residual": 1}[sort_mode]
    n = len(blocks)
    labels = (ctypes.c_int32 * n)()
    ncl = ctypes.c_int64(0)
    crel = (ctypes.c_double * n)()
    arr = _blocks(blocks)
    h.call_with_projection(projection, lambda: _check(_lib.cmsvd_cluster(
        h.ptr, arr, n, r, float(eps), mode, labels, ctypes.byref(ncl), crel)))
    lab = list(labels)
    clusters = [[] for _ in range(ncl.value)]
    for i, c in enumerate(lab):
        clusters[c].append(i)
    return lab, clusters, list(crel)[: ncl.value]


def cmsvd_cluster_trace(handle: Handle | None = None) -> list:
    """Anchors and acceptances of the handle's last cmsvd_cluster call, in order."""
    h = handle or default_handle()
    n = ctypes.c_int64(0)
    _check(_lib.cmsvd_cluster_trace(h.ptr, None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * max(n.value, 1))()
    _check(_lib.cmsvd_cluster_trace(h.ptr, buf, n.value, ctypes.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


def cmsvd_cluster_residual(blocks: Sequence[torch.Tensor], r: int, eps: float, sort_mode: str = "frobenius",
                           handle: Handle | None = None):
    """Algorithm 2 on the device.  Returns (labels list, clusters list, certified ratio list)."""
    dev = blocks[0].device
    h = handle or default_handle(dev)
    mode = {"frobenius": 0, "residual": 1}[sort_mode]
    n = len(blocks)
    labels = (ctypes.c_int32 * n)()
    ncl = ctypes.c_int64(0)
    crel = (ctypes.c_double * n)()
    arr = _blocks(blocks)
    _check(_lib.cmsvd_cluster_residual(h.ptr, arr, n, r, float(eps), mode, labels, ctypes.byref(ncl), crel))
    lab = list(labels)
    clusters = [[] for _ in range(ncl.value)]
    for i, c in enumerate(lab):
        clusters[c].append(i)
    return lab, clusters, list(crel)[: ncl.value]


def cmsvd_residual_bound(blocks: Sequence[torch.Tensor], r: int, handle: Handle | None = None):
    """Corollary 1 for the blocks in order.  Returns (bound^2, mu: the r largest
    residual singular values, descending, as a list)."""
    h = handle or default_handle(blocks[0].device)
    arr = _blocks(blocks)
    b2 = ctypes.c_double(0.0)
    mu = (ctypes.c_double * r)()
    _check(_lib.cmsvd_residual_bound(h.ptr, arr, len(blocks), r, ctypes.byref(b2), mu))
    return b2.value, list(mu)


def cmsvd_weyl_bound(blocks: Sequence[torch.Tensor], r: int, handle: Handle | None = None) -> float:
    """Theorem 1: S - max_j (r-head energy of A_j), clamped at 0."""
    h = handle or default_handle(blocks[0].device)
    out = ctypes.c_double(0.0)
    _check(_lib.cmsvd_weyl_bound(h.ptr, _blocks(blocks), len(blocks), r, ctypes.byref(out)))
    return out.value


def cmsvd_cluster_weyl(blocks: Sequence[torch.Tensor], r: int, eps: float, handle: Handle | None = None):
    """Algorithm 1 on the device.  Returns (labels list, clusters list, certified ratio list)."""
    h = handle or default_handle(blocks[0].device)
    n = len(blocks)
    labels = (ctypes.c_int32 * n)()
    ncl = ctypes.c_int64(0)
    crel = (ctypes.c_double * n)()
    _check(_lib.cmsvd_cluster_weyl(h.ptr, _blocks(blocks), n, r, float(eps), labels, ctypes.byref(ncl), crel))
    lab = list(labels)
    clusters = [[] for _ in range(ncl.value)]
    for i, c in enumerate(lab):
        clusters[c].append(i)
    return lab, clusters, list(crel)[: ncl.value]


def cmsvd_exact_tail(blocks: Sequence[torch.Tensor], r: int, handle: Handle | None = None) -> float:
    """sum_{l>r} sigma_l^2 of the concatenation, from its explicit Gram."""
    h = handle or default_handle(blocks[0].device)
    out = ctypes.c_double(0.0)
    _check(_lib.cmsvd_exact_tail(h.ptr, _blocks(blocks), len(blocks), r, ctypes.byref(out)))
    return out.value


def cmsvd_compress(blocks: Sequence[torch.Tensor], r: int, handle: Handle | None = None, with_energy: bool = False):
    """Stored factors of one cluster: (Ut = U S (m x r_C), Vt = V^T (r_C x N_C), tail2),
    plus ||M_C||_F^2 as a fourth item when ``with_energy``."""
    h = handle or default_handle(blocks[0].device)
    m = blocks[0].shape[0]
    N = sum(int(b.shape[1]) for b in blocks)
    rc = min(r, m, N)
    Ut = torch.empty((m, rc), dtype=torch.float64, device=blocks[0].device)
    Vt = torch.empty((rc, N), dtype=torch.float64, device=blocks[0].device)
    rank = ctypes.c_int64(0)
    tail2 = ctypes.c_double(0.0)
    energy = ctypes.c_double(0.0)
    _check(_lib.cmsvd_compress(h.ptr, _blocks(blocks), len(blocks), r, ctypes.c_void_p(Ut.data_ptr()), rc,
                               ctypes.c_void_p(Vt.data_ptr()), N, ctypes.byref(rank), ctypes.byref(tail2),
                               ctypes.byref(energy)))
    if with_energy:
        return Ut, Vt, tail2.value, energy.value
    return Ut, Vt, tail2.value


def compress_partition(blocks: Sequence[torch.Tensor], labels, r: int, handle: Handle | None = None):
    """Factors of every cluster of a partition (labels as returned by the clustering
    calls) and the summary computed by cmsvd_compress_partition: compression ratio
    (stored entries of the blocks over those of the factors) and the relative error
    sqrt(sum of the cluster tails) / ||all blocks||_F.
    Returns (factors: list of (members, Ut, Vt, tail2), summary dict)."""
    h = handle or default_handle(blocks[0].device)
    m = blocks[0].shape[0]
    lab = [int(c) for c in labels]
    ncl = max(lab) + 1
    members = [[i for i, c in enumerate(lab) if c == k] for k in range(ncl)]
    uts, vts = [], []
    for mem in members:
        N = sum(int(blocks[i].shape[1]) for i in mem)
        rc = min(r, m, N)
        uts.append(torch.empty((m, rc), dtype=torch.float64, device=blocks[0].device))
        vts.append(torch.empty((rc, N), dtype=torch.float64, device=blocks[0].device))
    P = ctypes.c_void_p * ncl
    L = ctypes.c_int64 * ncl
    ranks, t2 = L(), (ctypes.c_double * ncl)()
    lab_c = (ctypes.c_int32 * len(lab))(*lab)
    k, ratio, rel = ctypes.c_int64(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(_lib.cmsvd_compress_partition(
        h.ptr, _blocks(blocks), len(blocks), lab_c, r, P(*[u.data_ptr() for u in uts]), L(*[u.shape[1] for u in uts]),
        P(*[v.data_ptr() for v in vts]), L(*[v.shape[1] for v in vts]), ranks, t2, None, ctypes.byref(k),
        ctypes.byref(ratio), ctypes.byref(rel)))
    factors = [(mem, uts[c], vts[c], t2[c]) for c, mem in enumerate(members)]
    return factors, {"compression_ratio": ratio.value, "rel_error": rel.value, "clusters": int(k.value)}


def cmsvd_tail_energy_grad(blocks: Sequence[torch.Tensor], r: int, checkpoint: int | None = None,
                           want_grad: bool = True, handle: Handle | None = None):
    """Tail energy f = E~_r^2 of the chain ``blocks`` (in order) and, if ``want_grad``,
    d f / d A_t for every block (FP64, the blocks' shapes).  ``checkpoint`` = steps between
    stored states (default about sqrt(len(blocks))).  Returns (f, grads or None, min_gap)."""
    h = handle or default_handle(blocks[0].device)
    T = len(blocks)
    if checkpoint is None:
        checkpoint = max(1, int(round(T ** 0.5)))
    arr = _blocks(blocks)
    f = ctypes.c_double(0.0)
    gap = ctypes.c_double(0.0)
    grads = None
    gptr = None
    if want_grad:
        grads = [torch.empty((b.shape[0], b.shape[1]), dtype=torch.float64, device=b.device) for b in blocks]
        gptr = (ctypes.c_void_p * T)(*[g.data_ptr() for g in grads])
    _check(_lib.cmsvd_tail_energy_grad(h.ptr, arr, T, r, checkpoint, ctypes.byref(f), gptr, ctypes.byref(gap)))
    return f.value, grads, gap.value


class TailEnergy(torch.autograd.Function):
    """f = E~_r^2([A_1 ... A_T]) as a differentiable function of the blocks.

    ``TailEnergy.apply(r, checkpoint, *blocks)`` returns a 0-d FP64 tensor.  The backward
    calls the library again with gradients requested: it re-runs the forward keeping only
    checkpointed states and recomputes every step's bases during the reverse sweep."""

    @staticmethod
    def forward(ctx, r, checkpoint, *blocks):
        f, _, _ = cmsvd_tail_energy_grad(blocks, r, checkpoint, want_grad=False)
        ctx.r = r
        ctx.checkpoint = checkpoint
        ctx.save_for_backward(*blocks)
        return torch.tensor(f, dtype=torch.float64, device=blocks[0].device)

    @staticmethod
    def backward(ctx, gout):
        blocks = ctx.saved_tensors
        _, grads, _ = cmsvd_tail_energy_grad(blocks, ctx.r, ctx.checkpoint, want_grad=True)
        out = [(g * gout).to(b.dtype) for g, b in zip(grads, blocks)]
        return (None, None, *out)


def tail_energy(blocks: Sequence[torch.Tensor], r: int, checkpoint: int | None = None) -> torch.Tensor:
    """Differentiable tail energy of the chain (see ``TailEnergy``)."""
    if checkpoint is None:
        checkpoint = max(1, int(round(len(blocks) ** 0.5)))
    return TailEnergy.apply(r, checkpoint, *blocks)


def cmsvd_sym_eigvals(A: torch.Tensor, nkeep: int, handle: Handle | None = None) -> torch.Tensor:
    """Largest nkeep eigenvalues (descending) of a batch of symmetric FP64 matrices (..., n, n)."""
    if A.dtype != torch.float64 or not A.is_cuda:
        raise ValueError("A must be a CUDA float64 tensor")
    h = handle or default_handle(A.device)
    n = A.shape[-1]
    batch = A.reshape(-1, n, n).contiguous()
    lam = torch.empty((batch.shape[0], nkeep), dtype=torch.float64, device=A.device)
    # column-major view of each matrix: symmetric, so the row-major buffer serves as is
    _check(_lib.cmsvd_sym_eigvals(h.ptr, ctypes.c_void_p(batch.data_ptr()), n, n, n * n, batch.shape[0], nkeep,
                                  ctypes.c_void_p(lam.data_ptr())))
    return lam.reshape(*A.shape[:-2], nkeep)


def cmsvd_sym_eigvals_noalloc(A: torch.Tensor, nkeep: int, lam: torch.Tensor,
                              handle: Handle | None = None) -> torch.Tensor:
    """cmsvd_sym_eigvals into a caller-provided output (lam, (..., nkeep) FP64) through
    the entry point that allocates nothing: A must already be a contiguous CUDA float64
    batch (..., n, n), so that no copy is made here either."""
    if A.dtype != torch.float64 or not A.is_cuda or not A.is_contiguous():
        raise ValueError("A must be a contiguous CUDA float64 tensor")
    n = A.shape[-1]
    count = A.numel() // (n * n) if n else 0
    if lam.dtype != torch.float64 or not lam.is_contiguous() or lam.numel() != count * nkeep:
        raise ValueError("lam must be a contiguous float64 tensor of count x nkeep entries")
    h = handle or default_handle(A.device)
    _check(_lib.cmsvd_sym_eigvals_noalloc(h.ptr, ctypes.c_void_p(A.data_ptr()), n, n, n * n, count, nkeep,
                                          ctypes.c_void_p(lam.data_ptr())))
    return lam


def cmsvd_gemm_f64(opA: torch.Tensor, opB: torch.Tensor, C: torch.Tensor | None = None, alpha: float = 1.0,
                   beta: float = 0.0, handle: Handle | None = None) -> torch.Tensor:
    """C = alpha opA @ opB + beta C on the matrix cores.  opA (M x K) and opB (K x N) may be
    transposed views of contiguous FP32/FP64 tensors; C is FP64."""
    return _gemm(_lib.cmsvd_gemm_f64, opA, opB, C, alpha, beta, handle)


def cmsvd_gemm_bf16(opA: torch.Tensor, opB: torch.Tensor, C: torch.Tensor | None = None, alpha: float = 1.0,
                    beta: float = 0.0, handle: Handle | None = None, passes: int = 1) -> torch.Tensor:
    """As cmsvd_gemm_f64 with the operands rounded to BF16 (passes = 3: split into two
    BF16 parts) and FP32 accumulation."""
    return _gemm(lambda *a: _lib.cmsvd_gemm_bf16(a[0], passes, *a[1:]), opA, opB, C, alpha, beta, handle)


def cmsvd_gemm_f32(opA: torch.Tensor, opB: torch.Tensor, C: torch.Tensor | None = None, alpha: float = 1.0,
                   beta: float = 0.0, handle: Handle | None = None) -> torch.Tensor:
    """As cmsvd_gemm_f64 with the operands rounded to FP32 and FP32 accumulation."""
    return _gemm(_lib.cmsvd_gemm_f32, opA, opB, C, alpha, beta, handle)


def _gemm(fn, opA, opB, C, alpha, beta, handle):
    h = handle or default_handle(opA.device)

    def desc(t):
        # column-major (ld, trans) description of a 2-D view
        if t.stride(0) == 1 and t.stride(1) >= max(t.shape[0], 1):
            return t, 0, t.stride(1)
        if t.stride(1) == 1 and t.stride(0) >= max(t.shape[1], 1):
            return t, 1, t.stride(0)
        t = t.contiguous()
        return t, 1, t.stride(0)

    M, K = opA.shape
    K2, N = opB.shape
    assert K == K2
    a, ta, lda = desc(opA)
    b, tb, ldb = desc(opB)
    if C is None:
        C = torch.zeros((N, M), dtype=torch.float64, device=opA.device).t()
    assert C.stride(0) == 1
    dt = {torch.float32: CMSVD_F32, torch.float64: CMSVD_F64}
    _check(fn(h.ptr, ta, tb, M, N, K, float(alpha), ctypes.c_void_p(a.data_ptr()), lda, dt[a.dtype],
              ctypes.c_void_p(b.data_ptr()), ldb, dt[b.dtype], float(beta), ctypes.c_void_p(C.data_ptr()),
              C.stride(1)))
    return C


__all__ = ["cmsvd_gemm_f64", "cmsvd_gemm_bf16", "cmsvd_gemm_f32", "PROJECTIONS", "BlockArray", "Handle", "State", "Block", "CmsvdError", "cmsvd_update", "cmsvd_update_batch",
           "cmsvd_merge_errors", "cmsvd_cluster", "cmsvd_cluster_trace", "cmsvd_cluster_residual", "cmsvd_residual_bound",
           "cmsvd_weyl_bound", "cmsvd_cluster_weyl", "cmsvd_exact_tail", "cmsvd_compress", "compress_partition",
           "cmsvd_sym_eigvals", "cmsvd_sym_eigvals_noalloc", "cmsvd_tail_energy_grad", "TailEnergy", "tail_energy", "default_handle",
           "LIB_PATH", "EXPORTS"]
