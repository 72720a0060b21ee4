"""ctypes binding of ``libhda.so`` (the gfx950 library declared in
``include/hda.h``).  Argument marshalling only: every allocator step runs in
the library's kernels.  PyTorch provides the device buffers and the stream,
and -- through ``hda_set_device_allocator``, installed when the library is
loaded -- the device memory the library keeps for itself (torch's caching
allocator).

Importing this module does not load the library; the first call does, and it
raises if ``libhda.so`` has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhda.so")

FIRST_FIT, NEXT_FIT, BEST_FIT, SEG_FIT, TLSF, BITMAP = 0, 1, 2, 3, 4, 5
HDA_OK, HDA_FAIL, HDA_E_INVAL, HDA_E_BADFREE = 0, -1, -2, -3
HDA_E_NOMETA, HDA_E_DEVICE, HDA_E_BUSY, HDA_E_RANGE = -4, -5, -6, -7


class HdaError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class hda_tuning(ctypes.Structure):
    _fields_ = [("heaps_per_group", ctypes.c_int32), ("reg_free", ctypes.c_int32),
                ("reg_live", ctypes.c_int32), ("lds_free", ctypes.c_int32),
                ("lds_live", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("heavy_heaps", ctypes.c_int32), ("heavy_kib", ctypes.c_int32)]


TUNING_FIELDS = ("heaps_per_group", "reg_free", "reg_live", "lds_free", "lds_live", "groups",
                 "heavy_heaps", "heavy_kib")


def tuning(**kw) -> tuple:
    """A tuning tuple with the named fields set (others 0 = default)."""
    bad = set(kw) - set(TUNING_FIELDS)
    if bad:
        raise ValueError(f"unknown tuning fields {bad}")
    return tuple(int(kw.get(f, 0)) for f in TUNING_FIELDS)


class hda_batch_desc(ctypes.Structure):
    _fields_ = [("n_heaps", ctypes.c_int64),
                ("arena", ctypes.c_void_p), ("align", ctypes.c_void_p),
                ("algo", ctypes.c_void_p), ("req_off", ctypes.c_void_p),
                ("req", ctypes.c_void_p), ("res", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("state", ctypes.c_void_p),
                ("state_off", ctypes.c_void_p), ("state_len", ctypes.c_void_p),
                ("status", ctypes.c_void_p),
                ("meta_free", ctypes.c_int64), ("meta_live", ctypes.c_int64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("tuning", hda_tuning)]


class hda_serve_config(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("max_heaps", ctypes.c_int32),
                ("slot_free", ctypes.c_int32), ("slot_live", ctypes.c_int32),
                ("ring_entries", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("meta_budget", ctypes.c_int64), ("max_seconds", ctypes.c_double)]


class hda_load_config(ctypes.Structure):
    _fields_ = [("clients", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("log_clients", ctypes.c_int32),
                ("log_cap", ctypes.c_int64), ("log", ctypes.c_void_p),
                ("log_len", ctypes.c_void_p),
                ("arena_lo", ctypes.c_uint64), ("arena_hi", ctypes.c_uint64),
                ("align", ctypes.c_uint64), ("rate", ctypes.c_double),
                ("warmup_s", ctypes.c_double), ("measure_s", ctypes.c_double),
                ("p_pow2", ctypes.c_double), ("pow2_lo", ctypes.c_int32),
                ("pow2_hi", ctypes.c_int32), ("size_lo", ctypes.c_uint64),
                ("size_hi", ctypes.c_uint64), ("lifetime_mean", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("close_heaps", ctypes.c_int32),
                ("session_len", ctypes.c_int32)]


class hda_load_report(ctypes.Structure):
    _fields_ = [("issued", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("measured", ctypes.c_int64), ("alloc_ok", ctypes.c_int64),
                ("alloc_fail", ctypes.c_int64), ("frees", ctypes.c_int64),
                ("errors", ctypes.c_int64), ("window_s", ctypes.c_double),
                ("throughput", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p90_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("p999_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("mean_us", ctypes.c_double),
                ("host_p50_us", ctypes.c_double), ("host_p99_us", ctypes.c_double),
                ("queue_p50_us", ctypes.c_double), ("queue_p99_us", ctypes.c_double),
                ("service_p50_us", ctypes.c_double), ("service_p99_us", ctypes.c_double),
                ("transit_p50_us", ctypes.c_double), ("transit_p99_us", ctypes.c_double),
                ("sessions", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
                ("max_open", ctypes.c_int64), ("slot_bytes", ctypes.c_int64)]


HDA_OP_ALLOC, HDA_OP_FREE = 1, 2

_lib = None

DEV_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
    except Exception:       # out of memory: the library reports HDA_E_DEVICE
        return None


def _torch_free(ptr, ctx):
    import torch
    torch.cuda.caching_allocator_delete(ptr)


# kept alive for as long as the library may call them
_TORCH_ALLOCATOR = (DEV_ALLOC(_torch_alloc), DEV_FREE(_torch_free))

EXPORTS = ["hda_set_device_allocator", "hda_heap_load",
           "hda_replay_workspace", "hda_replay_resolve", "hda_replay", "hda_replay_static", "hda_replay_per_heap", "hda_replay_autotune", "hda_replay_capture",
           "hda_graph_launch", "hda_graph_destroy", "hda_bitmap_workspace", "hda_bitmap_replay",
           "hda_heap_create", "hda_heap_destroy", "hda_alloc",
           "hda_free", "hda_free_partial", "hda_heap_state", "hda_set_meta_budget", "hda_strerror",
           "hda_serve_start", "hda_serve_open", "hda_serve_submit", "hda_serve_poll",
           "hda_serve_wait", "hda_serve_close", "hda_serve_stop", "hda_serve_load",
           "hda_serve_slot_bytes"]


def lib():
    """Load libhda.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2405_07079_amd/build.py "
                               "(the GPU library has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        D = ctypes.POINTER(hda_batch_desc)
        L.hda_replay_workspace.restype = ctypes.c_size_t
        L.hda_replay_workspace.argtypes = [D]
        L.hda_bitmap_workspace.restype = ctypes.c_size_t
        L.hda_bitmap_workspace.argtypes = [D, ctypes.c_uint64]
        L.hda_bitmap_replay.restype = ctypes.c_int
        L.hda_bitmap_replay.argtypes = [D, ctypes.c_uint64, vp]
        L.hda_replay_resolve.restype = ctypes.c_int
        L.hda_replay_resolve.argtypes = [D, ctypes.POINTER(hda_tuning)]
        L.hda_replay.restype = ctypes.c_int
        L.hda_replay.argtypes = [D, vp]
        L.hda_replay_static.restype = ctypes.c_int
        L.hda_replay_static.argtypes = [D, vp]
        L.hda_replay_per_heap.restype = ctypes.c_int
        L.hda_replay_per_heap.argtypes = [D, vp]
        L.hda_replay_autotune.restype = ctypes.c_int
        L.hda_replay_autotune.argtypes = [D, ctypes.c_int32, vp, ctypes.POINTER(hda_tuning)]
        L.hda_replay_capture.restype = ctypes.c_int
        L.hda_replay_capture.argtypes = [D, ctypes.POINTER(vp)]
        L.hda_graph_launch.restype = ctypes.c_int
        L.hda_graph_launch.argtypes = [vp, vp]
        L.hda_graph_destroy.restype = ctypes.c_int
        L.hda_graph_destroy.argtypes = [vp]
        L.hda_heap_create.restype = ctypes.c_int
        L.hda_heap_create.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_uint32, ctypes.POINTER(vp)]
        L.hda_heap_destroy.restype = ctypes.c_int
        L.hda_heap_destroy.argtypes = [vp]
        L.hda_alloc.restype = ctypes.c_int64
        L.hda_alloc.argtypes = [vp, ctypes.c_uint64]
        L.hda_free.restype = ctypes.c_int
        L.hda_free.argtypes = [vp, ctypes.c_int64]
        L.hda_free_partial.restype = ctypes.c_int
        L.hda_free_partial.argtypes = [vp, ctypes.c_int64]
        L.hda_heap_load.restype = ctypes.c_int
        L.hda_heap_load.argtypes = [vp, vp, ctypes.c_size_t]
        L.hda_set_device_allocator.restype = ctypes.c_int
        L.hda_set_device_allocator.argtypes = [DEV_ALLOC, DEV_FREE, vp]
        L.hda_heap_state.restype = ctypes.c_int
        L.hda_heap_state.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.hda_set_meta_budget.restype = ctypes.c_int64
        L.hda_set_meta_budget.argtypes = [ctypes.c_int64]
        L.hda_strerror.restype = ctypes.c_char_p
        L.hda_strerror.argtypes = [ctypes.c_int]
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        for name, args in (
                ("hda_serve_start", [ctypes.POINTER(hda_serve_config), ctypes.POINTER(vp)]),
                ("hda_serve_open", [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, i32p]),
                ("hda_serve_submit", [vp, ctypes.c_int32, ctypes.c_int, ctypes.c_int64, u64p]),
                ("hda_serve_poll", [vp, ctypes.c_uint64, i64p, ctypes.POINTER(ctypes.c_int)]),
                ("hda_serve_wait", [vp, ctypes.c_uint64, i64p]),
                ("hda_serve_close", [vp, ctypes.c_int32]),
                ("hda_serve_stop", [vp]),
                ("hda_serve_load", [vp, ctypes.POINTER(hda_load_config),
                                    ctypes.POINTER(hda_load_report)])):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.hda_serve_slot_bytes.restype = ctypes.c_int64
        L.hda_serve_slot_bytes.argtypes = [ctypes.POINTER(hda_serve_config)]
        _lib = L
        if torch_available():
            use_torch_allocator()
    return _lib


def torch_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def use_torch_allocator() -> None:
    """Route the library's own device buffers through torch's caching
    allocator (done when the library is loaded on a machine with a GPU).
    torch's device state is set up first: it cannot be brought up from
    inside the library's callback."""
    import torch
    torch.cuda.init()
    _check(lib().hda_set_device_allocator(*_TORCH_ALLOCATOR, None), "hda_set_device_allocator")


def use_hip_allocator() -> None:
    """Back to hipMalloc / hipFree for the library's own device buffers."""
    _check(lib().hda_set_device_allocator(DEV_ALLOC(), DEV_FREE(), None),
           "hda_set_device_allocator")


def strerror(code: int) -> str:
    try:
        return lib().hda_strerror(int(code)).decode()
    except Exception:  # library not loadable: still give a readable message
        return f"error {code}"


def _check(code, what):
    if code != HDA_OK:
        raise HdaError(code, what)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# Batched replay
# ---------------------------------------------------------------------------

@dataclass
class DeviceBatch:
    """A workloads.Batch resident in device memory, with output buffers."""
    n_heaps: int
    arena: "torch.Tensor"
    align: "torch.Tensor"
    algo: "torch.Tensor"
    req_off: "torch.Tensor"
    req: "torch.Tensor"
    res: "torch.Tensor"
    order: "torch.Tensor | None"
    state: "torch.Tensor | None"
    state_off: "torch.Tensor | None"
    state_len: "torch.Tensor | None"
    status: "torch.Tensor"
    meta_free: int
    meta_live: int
    workspace: "torch.Tensor | None" = None
    tuning: tuple = (0, 0, 0, 0, 0, 0)

    def desc(self) -> hda_batch_desc:
        d = hda_batch_desc()
        p = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        d.n_heaps = self.n_heaps
        d.arena, d.align, d.algo = p(self.arena), p(self.align), p(self.algo)
        d.req_off, d.req, d.res = p(self.req_off), p(self.req), p(self.res)
        d.order = p(self.order)
        d.state, d.state_off, d.state_len = p(self.state), p(self.state_off), p(self.state_len)
        d.status = p(self.status)
        d.meta_free, d.meta_live = self.meta_free, self.meta_live
        d.workspace = p(self.workspace)
        d.workspace_bytes = 0 if self.workspace is None else self.workspace.numel()
        d.tuning = hda_tuning(*self.tuning)
        return d


def state_words(algo, blocks):
    """Words of a canonical state dump with at most `blocks` free + live blocks."""
    algo = np.asarray(algo)
    blocks = np.asarray(blocks, dtype=np.int64)
    return 4 + 2 * blocks + np.where(algo == SEG_FIT, 64 + blocks,
                                     np.where(algo == TLSF, 2048 + blocks, 0))


def upload(batch, device="cuda", order="lpt", with_state=True, meta_free=4096,
           meta_live=8192, tuning=(0, 0, 0, 0, 0, 0), share=None) -> DeviceBatch:
    """Copy a workloads.Batch to the device and allocate results, states,
    status and the library's workspace (all torch-owned).  With `share` (a
    DeviceBatch of the same streams) its request, offset, arena, alignment
    and order tensors are reused instead of copied again."""
    import torch
    H = batch.heaps
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device)  # noqa: E731
    lens = np.diff(batch.req_off)
    if share is not None:
        order_t = share.order
    elif order == "lpt":      # longest trace first; ties keep heap order
        ordv = np.argsort(-lens, kind="stable").astype(np.int32)
        order_t = t(ordv, np.int32)
    elif order is None:
        order_t = None
    else:
        order_t = t(order, np.int32)
    state = state_off = state_len = None
    if with_state:
        # a request adds at most one block to the tables -- two for the
        # bitmask allocator, which may cut from the middle of a free run, and
        # whose free runs are separated by live blocks
        blocks = np.where(np.asarray(batch.algo) == BITMAP,
                          np.minimum(2 * lens + 1, 2 * meta_live + 1),
                          np.minimum(lens + 1, meta_free + meta_live))
        caps = state_words(batch.algo, blocks).astype(np.int64)
        so = np.zeros(H + 1, np.int64)
        np.cumsum(caps, out=so[1:])
        state = torch.empty(int(so[-1]), dtype=torch.int64, device=device)
        state_off = t(so, np.int64)
        state_len = torch.zeros(H, dtype=torch.int64, device=device)
    # the library wants non-null request/result buffers even when empty
    if share is not None:
        arena_t, align_t, off_t, req_t = share.arena, share.align, share.req_off, share.req
    else:
        req = batch.req if batch.requests else np.zeros(1, np.int64)
        arena_t, align_t = t(batch.arena, np.int64), t(batch.align, np.int64)
        off_t, req_t = t(batch.req_off, np.int64), t(req, np.int64)
    db = DeviceBatch(H, arena_t, align_t, t(batch.algo, np.int32), off_t, req_t,
                     torch.empty(max(1, batch.requests), dtype=torch.int64, device=device),
                     order_t, state, state_off, state_len,
                     torch.zeros(H, dtype=torch.int32, device=device),
                     int(meta_free), int(meta_live), None, tuple(tuning))
    ws = hda_replay_workspace(db)
    db.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
    return db


def hda_replay_workspace(db: DeviceBatch) -> int:
    n = lib().hda_replay_workspace(ctypes.byref(db.desc()))
    if n == 0:
        raise HdaError(HDA_E_INVAL, "hda_replay_workspace")
    return int(n)


def hda_replay_resolve(db: DeviceBatch) -> dict:
    out = hda_tuning()
    _check(lib().hda_replay_resolve(ctypes.byref(db.desc()), ctypes.byref(out)),
           "hda_replay_resolve")
    return {f: getattr(out, f) for f in TUNING_FIELDS}


def hda_replay(db: DeviceBatch, stream=None) -> None:
    """Enqueue the batched replay on `stream` (default: torch's current)."""
    _check(lib().hda_replay(ctypes.byref(db.desc()), _stream_ptr(stream)), "hda_replay")


# bytes of the library's own per-GPU scratch behind hda_replay_static
STATIC_SCRATCH_BYTES = 64 << 20


def hda_replay_static(db: DeviceBatch, stream=None) -> None:
    """Enqueue the batched replay on `stream` with the library's static
    per-GPU scratch instead of the batch's workspace (no allocation)."""
    _check(lib().hda_replay_static(ctypes.byref(db.desc()), _stream_ptr(stream)),
           "hda_replay_static")


def max_granules(batch) -> int:
    """The largest arena of a workloads.Batch in granules."""
    return int((np.asarray(batch.arena) // np.asarray(batch.align)).max()) if batch.heaps else 1


def hda_bitmap_replay(db: DeviceBatch, max_gran: int, stream=None) -> None:
    """Enqueue the bitmask-allocator replay (every heap HDA_BITMAP, arenas of
    at most `max_gran` granules) on `stream`; the batch gets a workspace of
    hda_bitmap_workspace bytes the first time."""
    import torch
    d = db.desc()
    n = lib().hda_bitmap_workspace(ctypes.byref(d), int(max_gran))
    if n == 0:
        raise HdaError(HDA_E_INVAL, "hda_bitmap_workspace")
    ws = getattr(db, "bitmap_ws", None)
    if ws is None or ws.numel() < n:
        ws = torch.empty(n, dtype=torch.uint8, device=db.res.device)
        db.bitmap_ws = ws
    d.workspace, d.workspace_bytes = ws.data_ptr(), ws.numel()
    _check(lib().hda_bitmap_replay(ctypes.byref(d), int(max_gran), _stream_ptr(stream)),
           "hda_bitmap_replay")


def hda_replay_per_heap(db: DeviceBatch, stream=None) -> None:
    """Enqueue one launch per heap (the per-heap baseline) on `stream`."""
    _check(lib().hda_replay_per_heap(ctypes.byref(db.desc()), _stream_ptr(stream)),
           "hda_replay_per_heap")


def hda_replay_autotune(db: DeviceBatch, sample_heaps: int = 0, stream=None) -> tuple:
    """Time candidate tunings on a copy of the batch's longest heaps (traces
    cut to 65,536 requests); returns the fastest as a tuning tuple."""
    out = hda_tuning()
    _check(lib().hda_replay_autotune(ctypes.byref(db.desc()), int(sample_heaps),
                                     _stream_ptr(stream), ctypes.byref(out)),
           "hda_replay_autotune")
    return tuple(getattr(out, f) for f in TUNING_FIELDS)


def retune(db: DeviceBatch, tuning) -> DeviceBatch:
    """Set a batch's tuning and give it a workspace large enough for it."""
    import torch
    db.tuning = tuple(tuning)
    ws = hda_replay_workspace(db)
    if db.workspace is None or db.workspace.numel() < ws:
        db.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=db.res.device)
    return db


class ReplayGraph:
    """One hda_replay call on a DeviceBatch recorded as a hipGraph."""

    def __init__(self, db: DeviceBatch):
        self._db = db            # the graph points into its buffers
        h = ctypes.c_void_p()
        _check(lib().hda_replay_capture(ctypes.byref(db.desc()), ctypes.byref(h)),
               "hda_replay_capture")
        self._g = h

    def launch(self, stream=None) -> None:
        _check(lib().hda_graph_launch(self._g, _stream_ptr(stream)), "hda_graph_launch")

    def close(self) -> None:
        if self._g:
            _check(lib().hda_graph_destroy(self._g), "hda_graph_destroy")
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def states_to_host(db: DeviceBatch, heaps=None):
    """Per-heap canonical states as numpy arrays (a list; heaps=None: all)."""
    so = db.state_off.cpu().numpy()
    sl = db.state_len.cpu().numpy()
    heaps = range(db.n_heaps) if heaps is None else heaps
    out = []
    for h in heaps:
        n = min(int(sl[h]), int(so[h + 1] - so[h]))
        out.append(db.state[int(so[h]):int(so[h]) + n].cpu().numpy())
    return out


# ---------------------------------------------------------------------------
# Single heaps, call by call
# ---------------------------------------------------------------------------

class Heap:
    """A device-resident heap driven call by call (synchronous calls)."""

    def __init__(self, arena: int, align: int, algo: int, meta_cap: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hda_heap_create(int(arena), int(align), int(algo), int(meta_cap),
                                     ctypes.byref(h)), "hda_heap_create")
        self._h = h
        self.algo = int(algo)

    def close(self):
        if self._h:
            _check(lib().hda_heap_destroy(self._h), "hda_heap_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, size: int) -> int:
        r = int(lib().hda_alloc(self._h, int(size)))
        if r < -1:
            raise HdaError(r, "hda_alloc")
        return r

    def free(self, offset: int) -> int:
        return int(lib().hda_free(self._h, int(offset)))

    def free_partial(self, offset: int) -> int:
        return int(lib().hda_free_partial(self._h, int(offset)))

    def load(self, state) -> int:
        """Resume from a canonical state; returns the status code."""
        st = np.ascontiguousarray(state, np.int64)
        return int(lib().hda_heap_load(self._h, st.ctypes.data if st.size else None, st.size))

    def state(self) -> np.ndarray:
        n = ctypes.c_size_t(0)
        rc = lib().hda_heap_state(self._h, None, 0, ctypes.byref(n))
        if rc not in (HDA_OK, HDA_E_RANGE):
            raise HdaError(rc, "hda_heap_state")
        buf = np.empty(n.value, np.int64)
        _check(lib().hda_heap_state(self._h, buf.ctypes.data, n.value, ctypes.byref(n)),
               "hda_heap_state")
        return buf


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

class Server:
    """The device-resident allocator service (a persistent kernel)."""

    def __init__(self, max_heaps: int, waves: int = 0, slot_free: int = 0,
                 slot_live: int = 0, ring_entries: int = 0, meta_budget: int = 0,
                 max_seconds: float = 0.0):
        cfg = hda_serve_config(int(waves), int(max_heaps), int(slot_free), int(slot_live),
                               int(ring_entries), 0, int(meta_budget), float(max_seconds))
        h = ctypes.c_void_p()
        _check(lib().hda_serve_start(ctypes.byref(cfg), ctypes.byref(h)), "hda_serve_start")
        self._s = h

    @staticmethod
    def slot_bytes(slot_free: int = 0, slot_live: int = 0) -> int:
        """Metadata bytes one admitted heap holds (the budget's unit)."""
        cfg = hda_serve_config(0, 1, int(slot_free), int(slot_live), 0, 0, 0, 0.0)
        n = lib().hda_serve_slot_bytes(ctypes.byref(cfg))
        if n < 0:
            raise HdaError(int(n), "hda_serve_slot_bytes")
        return int(n)

    def open(self, arena: int, align: int, algo: int) -> int:
        heap = ctypes.c_int32()
        _check(lib().hda_serve_open(self._s, int(arena), int(align), int(algo),
                                    ctypes.byref(heap)), "hda_serve_open")
        return heap.value

    def submit(self, heap: int, op: int, arg: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().hda_serve_submit(self._s, int(heap), int(op), int(arg), ctypes.byref(t)),
               "hda_serve_submit")
        return t.value

    def poll(self, ticket: int):
        r, done = ctypes.c_int64(), ctypes.c_int()
        _check(lib().hda_serve_poll(self._s, int(ticket), ctypes.byref(r), ctypes.byref(done)),
               "hda_serve_poll")
        return (r.value if done.value else None)

    def wait(self, ticket: int) -> int:
        r = ctypes.c_int64()
        _check(lib().hda_serve_wait(self._s, int(ticket), ctypes.byref(r)), "hda_serve_wait")
        return r.value

    def alloc(self, heap: int, size: int) -> int:
        return self.wait(self.submit(heap, HDA_OP_ALLOC, size))

    def free(self, heap: int, offset: int) -> int:
        return self.wait(self.submit(heap, HDA_OP_FREE, offset))

    def close_heap(self, heap: int) -> None:
        _check(lib().hda_serve_close(self._s, int(heap)), "hda_serve_close")

    def load(self, clients: int, rate: float, warmup_s: float, measure_s: float,
             algo: int = SEG_FIT, threads: int = 0, log_clients: int = 0, log_cap: int = 0,
             arena=(64 << 20, 4 << 30), align: int = 512, p_pow2: float = 0.7,
             pow2=(9, 28), size=(512, 256 << 20), lifetime_mean: float = 500.0,
             seed: int = 4, close_heaps: bool = True, session_len: int = 0):
        """Run the open-loop client load; returns (report dict, logs or None).
        logs[c] is an array of (op, arg, result) rows for client c, with a
        (0, arena, align) row where each of its heaps (sessions) begins."""
        log = log_len = None
        if log_clients:
            log = np.zeros((log_clients, log_cap, 3), np.int64)
            log_len = np.zeros(log_clients, np.int64)
        cfg = hda_load_config(
            int(clients), int(algo), int(threads), int(log_clients), int(log_cap),
            None if log is None else log.ctypes.data,
            None if log_len is None else log_len.ctypes.data,
            int(arena[0]), int(arena[1]), int(align), float(rate), float(warmup_s),
            float(measure_s), float(p_pow2), int(pow2[0]), int(pow2[1]), int(size[0]),
            int(size[1]), float(lifetime_mean), int(seed), int(bool(close_heaps)),
            int(session_len))
        rep = hda_load_report()
        _check(lib().hda_serve_load(self._s, ctypes.byref(cfg), ctypes.byref(rep)),
               "hda_serve_load")
        out = {f: getattr(rep, f) for f, _ in hda_load_report._fields_}
        logs = None if log is None else [log[c, :log_len[c]] for c in range(log_clients)]
        return out, logs

    def stop(self) -> None:
        if self._s:
            _check(lib().hda_serve_stop(self._s), "hda_serve_stop")
            self._s = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
