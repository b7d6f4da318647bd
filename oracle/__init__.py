"""LearnedSort 2.0 oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``lsort_oracle.c``: a plain, single-threaded CPU
implementation of LearnedSort 2.0 (arXiv 2107.03290, Alg. 1 and Alg. 2,
Sec. 6.1 parameters).  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this module; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsort_oracle.c")
LIB = os.path.join(HERE, "liblsort_oracle.so")

F64, U64 = 1, 2


class Params(ctypes.Structure):
    _fields_ = [
        ("fanout", ctypes.c_uint32),
        ("frag_cap", ctypes.c_uint32),
        ("leaves", ctypes.c_uint32),
        ("small_n", ctypes.c_uint32),
        ("s_max", ctypes.c_uint64),
        ("sample_rate", ctypes.c_double),
        ("sample_cap", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("local_min_sample", ctypes.c_uint32),
        ("dtype", ctypes.c_uint32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("touchup_moves", ctypes.c_uint64),
        ("fragments", ctypes.c_uint64),
        ("partitions", ctypes.c_uint64),
        ("homogeneous", ctypes.c_uint64),
        ("counting_sorts", ctypes.c_uint64),
        ("fallbacks", ctypes.c_uint64),
        ("max_depth", ctypes.c_uint32),
        ("status", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no floating-point contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = os.environ.get("LSORT_ORACLE_LIB", LIB)   # mutation tests load a planted copy
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        u64p, dp = P(ctypes.c_uint64), P(ctypes.c_double)
        L.orc_default_params.argtypes = [P(Params), ctypes.c_uint32]
        L.orc_sort.argtypes = [u64p, ctypes.c_size_t, P(Params), P(Stats)]
        L.orc_sample_size.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64]
        L.orc_sample_size.restype = ctypes.c_uint64
        L.orc_sample_index.argtypes = [ctypes.c_uint64] * 3
        L.orc_sample_index.restype = ctypes.c_uint64
        L.orc_splitmix64_at.argtypes = [ctypes.c_uint64] * 2
        L.orc_splitmix64_at.restype = ctypes.c_uint64
        L.orc_train.argtypes = [u64p, ctypes.c_size_t, P(Params), dp, u64p]
        L.orc_train_sample.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.orc_model_eval.argtypes = [dp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_model_eval.restype = ctypes.c_double
        L.orc_bucket.argtypes = [dp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_double, ctypes.c_int64, ctypes.c_uint32]
        L.orc_bucket.restype = ctypes.c_uint32
        L.orc_stage_level0.argtypes = [u64p, ctypes.c_size_t, P(Params), dp, u64p, u64p,
                                       P(ctypes.c_uint8), u64p, u64p, u64p, ctypes.c_uint64, u64p]
        L.orc_partition.argtypes = [u64p, ctypes.c_size_t, dp, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32, u64p, u64p, ctypes.c_uint64, u64p]
        L.orc_defragment.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_uint32, u64p,
                                     ctypes.c_uint64]
        L.orc_counting_sort.argtypes = [u64p, ctypes.c_size_t, dp, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_double, ctypes.c_double]
        L.orc_split_stage.argtypes = [u64p, ctypes.c_size_t, P(Params), ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int, u64p, u64p, ctypes.c_uint32, P(ctypes.c_uint32),
                                      P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.orc_insertion_sort.argtypes = [u64p, ctypes.c_size_t, ctypes.c_uint32]
        L.orc_insertion_sort.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _u64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _f64(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(dtype: int = F64, **kw) -> Params:
    """Paper defaults (Sec. 6.1) overridden by keyword arguments."""
    p = Params()
    lib().orc_default_params(ctypes.byref(p), dtype)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def as_words(keys: np.ndarray) -> tuple[np.ndarray, int]:
    """Raw 64-bit words and the dtype code of a float64 / uint64 array."""
    if keys.dtype == np.float64:
        return np.ascontiguousarray(keys).view(np.uint64).copy(), F64
    if keys.dtype == np.uint64:
        return np.ascontiguousarray(keys).copy(), U64
    raise TypeError("oracle sorts float64 or uint64 keys")


def sort(keys: np.ndarray, **kw) -> tuple[np.ndarray, Stats]:
    """Return (sorted copy, stats) of a float64 / uint64 array."""
    w, dt = as_words(keys)
    p = params(dt, **kw)
    st = Stats()
    rc = lib().orc_sort(_u64(w), w.size, ctypes.byref(p), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("oracle sort failed: %d" % rc)
    return (w.view(np.float64) if dt == F64 else w), st


def sample_indices(n: int, **kw) -> np.ndarray:
    p = params(**kw)
    m = lib().orc_sample_size(n, p.sample_rate, p.sample_cap)
    return np.array([lib().orc_sample_index(p.seed, t, n) for t in range(m)], dtype=np.uint64)


def train(keys: np.ndarray, **kw) -> tuple[np.ndarray, np.ndarray]:
    """Global model in the export layout, and the sample indices used."""
    w, dt = as_words(keys)
    p = params(dt, **kw)
    m = lib().orc_sample_size(w.size, p.sample_rate, p.sample_cap)
    model = np.zeros(4 + 7 * (p.leaves + 1), dtype=np.float64)
    idx = np.zeros(m, dtype=np.uint64)
    rc = lib().orc_train(_u64(w), w.size, ctypes.byref(p), _f64(model), _u64(idx))
    if rc != 0:
        raise RuntimeError("oracle train failed: %d" % rc)
    return model, idx


def train_sample(sample: np.ndarray, leaves: int) -> np.ndarray:
    """Model trained on exactly these sample keys (no sampling step)."""
    w, dt = as_words(sample)
    model = np.zeros(4 + 7 * (leaves + 1), dtype=np.float64)
    rc = lib().orc_train_sample(_u64(w), w.size, leaves, dt, _f64(model))
    if rc != 0:
        raise RuntimeError("oracle train failed: %d" % rc)
    return model


def model_eval(model: np.ndarray, leaves: int, keys: np.ndarray) -> np.ndarray:
    w, dt = as_words(keys)
    L = lib()
    return np.array([L.orc_model_eval(_f64(model), leaves, int(k), dt) for k in w])


def bucket(model: np.ndarray, leaves: int, keys: np.ndarray, scale: float, offset: int,
           fanout: int) -> np.ndarray:
    w, dt = as_words(keys)
    L = lib()
    return np.array([L.orc_bucket(_f64(model), leaves, int(k), dt, scale, offset, fanout)
                     for k in w], dtype=np.int64)


def stage_level0(keys: np.ndarray, model: np.ndarray | None = None, with_sb1: bool = False,
                 **kw) -> dict:
    """Level-0 Partition + Defragment stage data (Alg. 2 first steps)."""
    w, dt = as_words(keys)
    p = params(dt, **kw)
    f = p.fanout
    sb = np.zeros(f, np.uint64)
    mm = np.zeros(2 * f, np.uint64)
    hom = np.zeros(f, np.uint8)
    sb1 = np.zeros(f * f, np.uint64) if with_sb1 else None
    out = np.zeros(w.size, np.uint64)
    cap = w.size // p.frag_cap + f + 1
    flog = np.zeros(2 * cap, np.uint64)
    nfrag = np.zeros(1, np.uint64)
    mp = _f64(np.ascontiguousarray(model, dtype=np.float64)) if model is not None else None
    rc = lib().orc_stage_level0(
        _u64(w), w.size, ctypes.byref(p), mp, _u64(sb), _u64(mm),
        hom.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
        _u64(sb1) if sb1 is not None else None, _u64(out), _u64(flog), cap, _u64(nfrag))
    if rc != 0:
        raise RuntimeError("oracle stage failed: %d" % rc)
    k = int(nfrag[0])
    return {"sb": sb, "min": mm[0::2], "max": mm[1::2], "homog": hom.astype(bool),
            "sb1": sb1.reshape(f, f) if sb1 is not None else None, "keys": out,
            "frag_log": flog[: 2 * k].reshape(k, 2)}


def partition(keys: np.ndarray, model: np.ndarray, leaves: int, fanout: int, frag_cap: int,
              level: int = 0, parent: int = 0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Alg. 1 on a copy: (array after copy-back, S_B, fragment log)."""
    w, dt = as_words(keys)
    sb = np.zeros(fanout, np.uint64)
    cap = w.size // frag_cap + fanout + 1
    flog = np.zeros(2 * cap, np.uint64)
    nfrag = np.zeros(1, np.uint64)
    rc = lib().orc_partition(_u64(w), w.size, _f64(np.ascontiguousarray(model)), leaves, dt,
                             fanout, frag_cap, level, parent, _u64(sb), _u64(flog), cap,
                             _u64(nfrag))
    if rc != 0:
        raise RuntimeError("oracle partition failed: %d" % rc)
    k = int(nfrag[0])
    out = w.view(np.float64) if dt == F64 else w
    return out, sb, flog[: 2 * k].reshape(k, 2)


def defragment(keys: np.ndarray, sb: np.ndarray, fanout: int, frag_log: np.ndarray) -> np.ndarray:
    w, dt = as_words(keys)
    fl = np.ascontiguousarray(frag_log.reshape(-1), dtype=np.uint64)
    rc = lib().orc_defragment(_u64(w), w.size, _u64(np.ascontiguousarray(sb, np.uint64)), fanout,
                              _u64(fl) if fl.size else None, frag_log.shape[0])
    if rc != 0:
        raise RuntimeError("oracle defragment failed: %d" % rc)
    return w.view(np.float64) if dt == F64 else w


def counting_sort(keys: np.ndarray, model: np.ndarray, leaves: int, scale: float,
                  offset: float) -> np.ndarray:
    w, dt = as_words(keys)
    rc = lib().orc_counting_sort(_u64(w), w.size, _f64(np.ascontiguousarray(model)), leaves, dt,
                                 scale, offset)
    if rc != 0:
        raise RuntimeError("oracle counting sort failed: %d" % rc)
    return w.view(np.float64) if dt == F64 else w


DEPTH_ERROR = -5


def split_stage(keys: np.ndarray, start: int = 0, depth: int = 2, force_msd: bool = False, **kw) -> dict:
    """One recursion split of reading R18 on a copy of keys (at least two
    distinct): {"keys": the range after the split, "sb": child sizes,
    "msd": whether the MSD digit split it, "shift": that digit's shift}."""
    w, dt = as_words(keys)
    p = params(dt, **kw)
    out = np.zeros(w.size, np.uint64)
    sb = np.zeros(p.fanout, np.uint64)
    fo, msd, sh = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib().orc_split_stage(_u64(w), w.size, ctypes.byref(p), start, depth, int(force_msd), _u64(out),
                               _u64(sb), p.fanout, ctypes.byref(fo), ctypes.byref(msd), ctypes.byref(sh))
    if rc != 0:
        raise RuntimeError("oracle split failed: %d" % rc)
    return {"keys": out.view(np.float64) if dt == F64 else out, "sb": sb[: fo.value], "msd": bool(msd.value),
            "shift": int(sh.value)}


def insertion_sort(keys: np.ndarray) -> tuple[np.ndarray, int]:
    w, dt = as_words(keys)
    moves = lib().orc_insertion_sort(_u64(w), w.size, dt)
    return (w.view(np.float64) if dt == F64 else w), int(moves)
