"""LearnedSort 2.0 on AMD Instinct MI355X: Python binding of liblsort.so.

Argument marshalling only: every step of the sort runs in the HIP kernels of
the library (paper_2107_03290_amd/csrc).  PyTorch provides device memory and
the current stream.  If the library has not been built the import of a sort
function fails loudly; there is no CPU fallback.

    import torch, paper_2107_03290_amd as ls
    x = torch.rand(1 << 20, dtype=torch.float64, device="cuda")
    ls.sort_(x)                      # in place, bit-exact totalOrder
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblsort.so")

F64, U64 = 1, 2

FLAG_DEBUG_TOUCHUP = 0x1
FLAG_SYNC = 0x2
FLAG_NONMONOTONE = 0x4
FLAG_PROFILE = 0x8
FLAG_GRAPH = 0x10
FLAG_INPLACE = 0x20


def FLAG_PROFILE_ONLY(k: int) -> int:
    """With FLAG_PROFILE: time only kernel class k (an index of KERNEL_CLASSES)."""
    return (k + 1) << 8

KERNEL_CLASSES = ("train", "hist", "scan", "classify", "scatter", "base", "fill", "touchup")

NOALLOC_MAX_KEYS = 1 << 20

DEV_SEAM_REPAIRED = 0x1
DEV_FALLBACK = 0x2
DEV_DEEP = 0x4

STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error",
          4: "unsupported parameters", 5: "request exceeds the memory budget", 6: "timed out",
          7: "unknown ticket"}

# C-ABI entry points declared in include/lsort.h
EXPORTS = (
    "ls_create", "ls_destroy", "ls_default_params", "ls_workspace_size", "ls_reserve", "ls_device_bytes", "ls_trim",
    "ls_sort_f64", "ls_sort_u64", "ls_sort_noalloc", "ls_sort_segments", "ls_sort_segments_device",
    "ls_sort_arrays", "ls_sort_ls1",
    "ls_autotune", "ls_sync",
    "ls_last_stats", "ls_last_profile", "ls_profile_reset", "ls_status_string", "ls_last_error",
    "ls_model_train", "ls_stage_hist",
    "ls_server_create", "ls_server_submit", "ls_server_wait", "ls_server_stats",
    "ls_server_last_error", "ls_server_destroy",
)


class LsortError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__("%s%s" % (STATUS.get(status, "status %d" % status), (": " + msg) if msg else ""))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("fanout", ctypes.c_uint32),
        ("leaves", ctypes.c_uint32),
        ("tile", ctypes.c_uint32),
        ("base_threshold", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("sample_rate", ctypes.c_double),
        ("sample_cap", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
    ]


class Array(ctypes.Structure):
    _fields_ = [("d_keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("dtype", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("fanout", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("base_threshold", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("ms", ctypes.c_double)]


_lib = None
_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it was not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("liblsort.so is not built: run `python -c 'import __graft_entry__ as g; "
                                  "g.build()'` (no CPU fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            vp, u64, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t
            P = ctypes.POINTER
            L.ls_create.argtypes = [P(vp), ctypes.c_int]
            L.ls_destroy.argtypes = [vp]
            L.ls_default_params.argtypes = [P(Params)]
            L.ls_default_params.restype = None
            L.ls_workspace_size.argtypes = [vp, ctypes.c_int, sz, P(Params), P(sz)]
            L.ls_reserve.argtypes = [vp, sz, P(Params)]
            L.ls_device_bytes.argtypes = [vp, P(sz)]
            L.ls_trim.argtypes = [vp]
            L.ls_sort_f64.argtypes = [vp, vp, sz, vp, P(Params)]
            L.ls_sort_u64.argtypes = [vp, vp, sz, vp, P(Params)]
            L.ls_sort_noalloc.argtypes = [vp, ctypes.c_int, vp, sz, vp, P(Params)]
            L.ls_sort_segments.argtypes = [vp, ctypes.c_int, vp, P(u64), sz, P(ctypes.c_uint8), vp, P(Params)]
            L.ls_sort_arrays.argtypes = [vp, P(Array), sz, vp, P(Params)]
            L.ls_sort_segments_device.argtypes = [vp, ctypes.c_int, vp, vp, sz, vp, vp, P(Params)]
            L.ls_sort_ls1.argtypes = [vp, ctypes.c_int, vp, sz, ctypes.c_double, vp, P(Params),
                                      P(ctypes.c_double)]
            L.ls_autotune.argtypes = [vp, P(Array), sz, vp, P(Params), ctypes.c_uint32, P(Params),
                                      P(TuneResult), sz, P(sz)]
            L.ls_sync.argtypes = [vp, P(ctypes.c_uint32)]
            L.ls_last_stats.argtypes = [vp, P(u64)]
            L.ls_last_profile.argtypes = [vp, P(ctypes.c_double), sz]
            L.ls_profile_reset.argtypes = [vp]
            L.ls_status_string.argtypes = [ctypes.c_int]
            L.ls_status_string.restype = ctypes.c_char_p
            L.ls_last_error.argtypes = [vp]
            L.ls_last_error.restype = ctypes.c_char_p
            L.ls_model_train.argtypes = [vp, ctypes.c_int, vp, sz, P(Params), P(ctypes.c_double), sz]
            L.ls_stage_hist.argtypes = [vp, ctypes.c_int, vp, sz, P(ctypes.c_double), ctypes.c_uint32,
                                        ctypes.c_double, ctypes.c_int64, ctypes.c_uint32, P(u64), P(u64), P(u64)]
            L.ls_server_create.argtypes = [P(vp), ctypes.c_int, sz, ctypes.c_uint32, P(Params)]
            L.ls_server_submit.argtypes = [vp, ctypes.c_int, vp, sz, P(u64)]
            L.ls_server_wait.argtypes = [vp, u64, ctypes.c_int, P(ctypes.c_double)]
            L.ls_server_stats.argtypes = [vp, P(u64)]
            L.ls_server_last_error.argtypes = [vp, ctypes.c_char_p, sz]
            L.ls_server_destroy.argtypes = [vp]
            _lib = L
        return _lib


def params(**kw) -> Params:
    """Default parameters (see include/lsort.h) overridden by keywords."""
    p = Params()
    lib().ls_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _pp(p: Params | None):
    return ctypes.byref(p) if p is not None else None


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)):
        return U64
    raise TypeError("keys must be float64, or uint64 / int64 holding unsigned 64-bit words")


def _check_tensor(t):
    if not t.is_cuda:
        raise ValueError("keys must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("keys must be contiguous")


def _stream_handle(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


class Sorter:
    """A library context bound to one device (not thread-safe)."""

    def __init__(self, device: int = 0):
        self._ctx = ctypes.c_void_p()
        st = lib().ls_create(ctypes.byref(self._ctx), int(device))
        if st != 0:
            raise LsortError(st, "ls_create(device=%d)" % device)
        self.device = int(device)

    def close(self):
        if self._ctx:
            lib().ls_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise LsortError(st, lib().ls_last_error(self._ctx).decode())

    def sort_(self, t, p: Params | None = None):
        """Sort a float64 or u64 (int64 words) device tensor in place."""
        _check_tensor(t)
        code = _dtype_code(t)
        fn = lib().ls_sort_f64 if code == F64 else lib().ls_sort_u64
        self._check(fn(self._ctx, t.data_ptr(), t.numel(), _stream_handle(t), _pp(p)))

    def sort_noalloc_(self, t, p: Params | None = None):
        """The same sort out of the library's static per-device array, with no
        allocation (at most NOALLOC_MAX_KEYS keys; synchronous)."""
        _check_tensor(t)
        self._check(lib().ls_sort_noalloc(self._ctx, _dtype_code(t), t.data_ptr(), t.numel(), _stream_handle(t),
                                          _pp(p)))
        return t

    def sort_segments_(self, t, offsets: Sequence[int], dtypes: Sequence[int] | None = None,
                       p: Params | None = None):
        """Sort each segment t[offsets[i]:offsets[i+1]] in place."""
        _check_tensor(t)
        code = _dtype_code(t)
        n = len(offsets) - 1
        off = (ctypes.c_uint64 * (n + 1))(*[int(x) for x in offsets])
        dt = (ctypes.c_uint8 * n)(*[int(x) for x in dtypes]) if dtypes is not None else None
        self._check(lib().ls_sort_segments(self._ctx, code, t.data_ptr(), off, n, dt, _stream_handle(t), _pp(p)))
        return t

    def sort_segments_device_(self, t, d_offsets, d_dtypes=None, p: Params | None = None):
        """sort_segments_ with the batch described by device tensors:
        d_offsets (int64, num_segments + 1 entries) and d_dtypes (uint8
        ls_dtype codes, or None for t's type), both on t's device."""
        _check_tensor(t)
        if not d_offsets.is_cuda or d_offsets.dtype.itemsize != 8 or not d_offsets.is_contiguous():
            raise ValueError("d_offsets must be a contiguous 64-bit device tensor")
        if d_dtypes is not None and (not d_dtypes.is_cuda or d_dtypes.element_size() != 1 or
                                     not d_dtypes.is_contiguous()):
            raise ValueError("d_dtypes must be a contiguous 8-bit device tensor")
        n = d_offsets.numel() - 1
        dt = d_dtypes.data_ptr() if d_dtypes is not None else None
        self._check(lib().ls_sort_segments_device(self._ctx, _dtype_code(t), t.data_ptr(), d_offsets.data_ptr(),
                                                  max(n, 0), dt, _stream_handle(t), _pp(p)))
        return t

    def sort_arrays_(self, tensors: Sequence, p: Params | None = None):
        """Sort separate device tensors together in one batched pipeline."""
        arr = (Array * len(tensors))()
        for i, t in enumerate(tensors):
            _check_tensor(t)
            arr[i] = Array(t.data_ptr(), t.numel(), _dtype_code(t), 0)
        st = _stream_handle(tensors[0]) if len(tensors) else None
        self._check(lib().ls_sort_arrays(self._ctx, arr, len(tensors), st, _pp(p)))
        return tensors

    def autotune(self, tensors: Sequence, offsets: Sequence[int] | None = None, p: Params | None = None,
                 reps: int = 2):
        """Time the candidate (fanout, tile, base_threshold) settings on a
        copy of the keys (left unmodified) and return (best Params, results).
        `tensors` is a list of device tensors, or one tensor split by
        `offsets` into segments."""
        if offsets is not None:
            (t,) = tensors if isinstance(tensors, (list, tuple)) else (tensors,)
            _check_tensor(t)
            code, base = _dtype_code(t), t.data_ptr()
            arr = (Array * (len(offsets) - 1))()
            for i in range(len(offsets) - 1):
                arr[i] = Array(base + 8 * int(offsets[i]), int(offsets[i + 1]) - int(offsets[i]), code, 0)
            st = _stream_handle(t)
        else:
            arr = (Array * len(tensors))()
            for i, t in enumerate(tensors):
                _check_tensor(t)
                arr[i] = Array(t.data_ptr(), t.numel(), _dtype_code(t), 0)
            st = _stream_handle(tensors[0]) if len(tensors) else None
        best = Params()
        res = (TuneResult * 64)()
        cnt = ctypes.c_size_t()
        self._check(lib().ls_autotune(self._ctx, arr, len(arr), st, _pp(p), reps, ctypes.byref(best), res, 64,
                                      ctypes.byref(cnt)))
        out = [dict(fanout=r.fanout, tile=r.tile, base_threshold=r.base_threshold, ms=r.ms)
               for r in res[:min(cnt.value, 64)]]
        return best, out

    def sync(self) -> int:
        s = ctypes.c_uint32()
        self._check(lib().ls_sync(self._ctx, ctypes.byref(s)))
        return s.value

    def last_stats(self) -> dict:
        a = (ctypes.c_uint64 * 8)()
        self._check(lib().ls_last_stats(self._ctx, a))
        keys = ("rounds", "tasks", "groups", "fill_buckets", "fill_keys", "fallbacks", "seams_repaired",
                "max_level")
        return dict(zip(keys, [int(x) for x in a]))

    def profile(self) -> dict:
        """{class: (ms, launches, algorithmic bytes)} accumulated by sorts run
        with FLAG_PROFILE since the last profile_reset()."""
        a = (ctypes.c_double * 24)()
        self._check(lib().ls_last_profile(self._ctx, a, 24))
        return {k: (a[3 * i], int(a[3 * i + 1]), a[3 * i + 2]) for i, k in enumerate(KERNEL_CLASSES)}

    def profile_reset(self):
        self._check(lib().ls_profile_reset(self._ctx))

    def sort_ls1_(self, t, slack: float = 0.1, p: Params | None = None) -> dict:
        """LearnedSort 1.0's spill-bucket sort of t in place (the ablation of
        ls_sort_ls1; the same result as sort_).  Returns its counters and
        per-phase milliseconds."""
        _check_tensor(t)
        out = (ctypes.c_double * 8)()
        self._check(lib().ls_sort_ls1(self._ctx, _dtype_code(t), t.data_ptr(), t.numel(), slack,
                                      _stream_handle(t), _pp(p), out))
        keys = ("spilled", "capacity", "ms_partition", "ms_bucket_sorts", "ms_spill_sort", "ms_merge", "ms_total",
                "fanout")
        return dict(zip(keys, [float(x) for x in out]))

    def device_bytes(self) -> int:
        """Device memory the context's work buffers hold now."""
        b = ctypes.c_size_t()
        self._check(lib().ls_device_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    def trim(self):
        """Free the context's work buffers (after its queued work ends)."""
        self._check(lib().ls_trim(self._ctx))

    def workspace_size(self, n: int, dtype: int = F64, p: Params | None = None) -> int:
        b = ctypes.c_size_t()
        self._check(lib().ls_workspace_size(self._ctx, dtype, n, _pp(p), ctypes.byref(b)))
        return b.value

    def reserve(self, n: int, p: Params | None = None):
        self._check(lib().ls_reserve(self._ctx, n, _pp(p)))

    # --- stage hooks -------------------------------------------------------
    def model_train(self, t, p: Params | None = None):
        """Global model trained on the device (export layout, numpy f64)."""
        import numpy as np
        _check_tensor(t)
        leaves = (p.leaves if p is not None and p.leaves else 1024)
        out = np.zeros(4 + 7 * (leaves + 1), dtype=np.float64)
        self._check(lib().ls_model_train(self._ctx, _dtype_code(t), t.data_ptr(), t.numel(), _pp(p),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
        return out

    def stage_hist(self, t, model, leaves: int, scale: float, offset: int, fanout: int):
        """(counts, min, max) of one partition histogram on the device."""
        import numpy as np
        _check_tensor(t)
        m = np.ascontiguousarray(model, dtype=np.float64)
        c = np.zeros(fanout, np.uint64)
        lo = np.zeros(fanout, np.uint64)
        hi = np.zeros(fanout, np.uint64)
        u = ctypes.POINTER(ctypes.c_uint64)
        self._check(lib().ls_stage_hist(self._ctx, _dtype_code(t), t.data_ptr(), t.numel(),
                                        m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), leaves, float(scale),
                                        int(offset), fanout, c.ctypes.data_as(u), lo.ctypes.data_as(u),
                                        hi.ctypes.data_as(u)))
        return c, lo, hi


_default: dict[int, Sorter] = {}


def _sorter(device: int) -> Sorter:
    s = _default.get(device)
    if s is None:
        s = _default[device] = Sorter(device)
    return s


def sort_(t, p: Params | None = None):
    """Sort a device tensor in place with the default context of its device."""
    return _sorter(t.device.index or 0).sort_(t, p)


def sort_segments_(t, offsets, dtypes=None, p: Params | None = None):
    return _sorter(t.device.index or 0).sort_segments_(t, offsets, dtypes, p)


def sort_arrays_(tensors, p: Params | None = None):
    return _sorter(tensors[0].device.index or 0).sort_arrays_(tensors, p)


class TuneCache:
    """Autotuned parameters per size class, kept in a JSON file.

    The class of a batch is (key type, log2 of its total keys, log2 of its
    mean array size), so one measurement serves every batch of that shape.
    Tuned parameters never change a sorted result, only its speed."""

    def __init__(self, path: str):
        import json
        self.path = path
        self.table = {}
        if os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    @staticmethod
    def size_class(dtype: int, total: int, count: int) -> str:
        mean = total // max(count, 1)
        return "%s:t%d:m%d" % ("f64" if dtype == F64 else "u64", max(total, 1).bit_length() - 1,
                               max(mean, 1).bit_length() - 1)

    def lookup(self, key: str) -> Params | None:
        e = self.table.get(key)
        if e is None:
            return None
        return params(fanout=e["fanout"], tile=e["tile"], base_threshold=e["base_threshold"])

    def tuned(self, sorter: Sorter, tensors: Sequence, offsets: Sequence[int] | None = None,
              p: Params | None = None, reps: int = 2) -> Params:
        """Cached parameters for this batch's class, tuning (and saving) on a miss."""
        import json
        if offsets is not None:
            t = tensors[0] if isinstance(tensors, (list, tuple)) else tensors
            dt, total, count = _dtype_code(t), int(offsets[-1]), len(offsets) - 1
        else:
            dt, total, count = _dtype_code(tensors[0]), sum(int(t.numel()) for t in tensors), len(tensors)
        key = self.size_class(dt, total, count)
        got = self.lookup(key)
        if got is not None:
            return got
        best, results = sorter.autotune(tensors, offsets, p, reps)
        self.table[key] = {"fanout": best.fanout, "tile": best.tile, "base_threshold": best.base_threshold,
                           "results": results}
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        with open(self.path, "w") as f:
            json.dump(self.table, f, indent=1)
        return self.lookup(key)


class Server:
    """Continuous-batching sort server (ls_server_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 200 << 30, max_inflight: int = 2,
                 p: Params | None = None):
        self._s = ctypes.c_void_p()
        st = lib().ls_server_create(ctypes.byref(self._s), device, hbm_budget, max_inflight, _pp(p))
        if st != 0:
            raise LsortError(st, "ls_server_create")

    def submit(self, t) -> int:
        _check_tensor(t)
        tk = ctypes.c_uint64()
        st = lib().ls_server_submit(self._s, _dtype_code(t), t.data_ptr(), t.numel(), ctypes.byref(tk))
        if st != 0:
            raise LsortError(st, "submit")
        return tk.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> float:
        lat = ctypes.c_double()
        st = lib().ls_server_wait(self._s, ticket, timeout_ms, ctypes.byref(lat))
        if st != 0:
            buf = ctypes.create_string_buffer(512)
            lib().ls_server_last_error(self._s, buf, 512)
            raise LsortError(st, "wait: " + buf.value.decode(errors="replace"))
        return lat.value

    def stats(self) -> dict:
        a = (ctypes.c_uint64 * 6)()
        lib().ls_server_stats(self._s, a)
        return dict(zip(("submitted", "completed", "batches", "peak_bytes", "accounted_bytes", "queued"),
                        [int(x) for x in a]))

    def close(self):
        if self._s:
            st = lib().ls_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            if st != 0:
                raise LsortError(st, "destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
