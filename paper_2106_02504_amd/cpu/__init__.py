"""The CPU baseline: RANLUX++ on the host in C++ (nine 64-bit words, products
with unsigned __int128, one std::thread per hardware thread), as the paper's
portable implementation computes it (section 3).  A ctypes binding over
numpy arrays; librlx_cpu.so is built by paper_2106_02504_amd.build.

It shares no code with the GPU kernels and is not the oracle: the tests
check it against the oracle, and bench.py times it beside the GPU."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlx_cpu.so")
_lib = None
_p = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int

_SIGS = {
    "rlx_cpu_seed": (None, [_p, _u64, _u64, _u32, _int]),
    "rlx_cpu_skip": (None, [_p, _u64, _p, _u32, _int]),
    "rlx_cpu_generate": (None, [_u64, _u64, _u64, _u32, _p, _p, _int]),
    "rlx_cpu_generate_split": (None, [_u64, _u64, _u32, _p, _int]),
    "rlx_cpu_generate_requests": (None, [_u64, _p, _p, _p, _p, _p, _p, _int]),
    "rlx_cpu_mulmod": (None, [_p, _p, _p]),
    "rlx_cpu_to_ranlux": (None, [_p, _p]),
    "rlx_cpu_threads": (_int, []),
}


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_02504_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous
    return a.ctypes.data


def threads() -> int:
    """Threads the calls use by default (one per hardware thread)."""
    return int(lib().rlx_cpu_threads())


def seed(n: int, id0: int, p: int, nthreads: int = 0) -> np.ndarray:
    """[n, 9] uint64 states A_p^(2^96 (id0 + i))."""
    x = np.empty((n, 9), dtype=np.uint64)
    lib().rlx_cpu_seed(_ptr(x), n, id0, p, nthreads)
    return x


def skip(x: np.ndarray, k, p: int, nthreads: int = 0) -> None:
    """x[i] <- A_p^(k[i]) x[i] in place (k: uint64 per state)."""
    k = np.ascontiguousarray(np.asarray(k, dtype=np.uint64).reshape(-1))
    assert x.dtype == np.uint64 and x.shape == (k.shape[0], 9)
    lib().rlx_cpu_skip(_ptr(x), x.shape[0], _ptr(k), p, nthreads)


def generate(n: int, id0: int, count: int, p: int, u48: bool = False, nthreads: int = 0) -> np.ndarray:
    """[n, count] doubles (or 48-bit integers) of the streams seeded with ids
    id0 .. id0 + n - 1, from position 0."""
    if u48:
        out = np.empty((n, count), dtype=np.uint64)
        lib().rlx_cpu_generate(n, id0, count, p, None, _ptr(out), nthreads)
    else:
        out = np.empty((n, count), dtype=np.float64)
        lib().rlx_cpu_generate(n, id0, count, p, _ptr(out), None, nthreads)
    return out


def generate_split(stream_id: int, count: int, p: int, nthreads: int = 0) -> np.ndarray:
    """One stream's `count` doubles, its steps split over the threads."""
    out = np.empty(count, dtype=np.float64)
    lib().rlx_cpu_generate_split(stream_id, count, p, _ptr(out), nthreads)
    return out


def generate_requests(ids, starts, counts, ps, nthreads: int = 0):
    """Flat doubles of the requests (stream ids[r], values starts[r] ..
    starts[r] + counts[r] at level ps[r]), at prefix-sum offsets."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    starts = np.ascontiguousarray(starts, dtype=np.uint64)
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    ps = np.ascontiguousarray(ps, dtype=np.uint32)
    offs = np.zeros(len(counts), dtype=np.uint64)
    offs[1:] = np.cumsum(counts)[:-1]
    out = np.empty(int(counts.sum()), dtype=np.float64)
    lib().rlx_cpu_generate_requests(len(counts), _ptr(ids), _ptr(starts), _ptr(counts), _ptr(ps), _ptr(offs),
                                    _ptr(out), nthreads)
    return out, offs


def mulmod(x: int, y: int) -> int:
    a = np.array([(x >> (64 * k)) & (2 ** 64 - 1) for k in range(9)], dtype=np.uint64)
    b = np.array([(y >> (64 * k)) & (2 ** 64 - 1) for k in range(9)], dtype=np.uint64)
    r = np.empty(9, dtype=np.uint64)
    lib().rlx_cpu_mulmod(_ptr(a), _ptr(b), _ptr(r))
    return sum(int(r[k]) << (64 * k) for k in range(9))


def to_ranlux(x: int) -> int:
    a = np.array([(x >> (64 * k)) & (2 ** 64 - 1) for k in range(9)], dtype=np.uint64)
    d = np.empty(9, dtype=np.uint64)
    lib().rlx_cpu_to_ranlux(_ptr(a), _ptr(d))
    return sum(int(d[k]) << (64 * k) for k in range(9))
