"""rlx -- RANLUX++ random numbers on an AMD MI355X (gfx950).

Thin ctypes binding over librlx.so (see include/rlx.h).  Every step of the
generator runs in the library's HIP kernels; this module only marshals
PyTorch tensors (device memory) and the current HIP stream into the C ABI.
There is no CPU implementation here: if the library is missing, every call
raises.

Stream records are ``int64`` tensors of shape ``[n, 10]`` on a CUDA (HIP)
device: words 0..8 hold the 576-bit LCG state X (least significant first),
word 9 holds ``pos | p << 32``.

Paper: Hahnfeld & Moneta, "A Portable Implementation of RANLUX++",
arXiv 2106.02504.  Seeding/skipping: section 2.4; generation: sections
2.1-2.3.
"""

from __future__ import annotations

import ctypes
import os

import torch  # load torch's HIP runtime first: librlx.so binds to the same one

__all__ = [
    "RlxError", "lib", "new_states", "prepare", "init_streams", "skip",
    "generate_f64", "generate_u64", "generate_normal_f64", "generate_f64_trace", "check_errors",
    "EngineTables", "get_tables", "build_tables_static", "table_words", "test_engine",
    "set_lanes_per_stream", "lanes_per_stream", "set_step_kernel", "step_kernel", "STEP_MFMA", "STEP_VALU",
    "skip_values", "export_ranlux", "import_ranlux", "REQUEST_DTYPE", "requests_array", "Plan", "plan_dry_run",
    "constants", "test_mulmod", "test_pow", "test_to_ranlux",
    "test_generate_u64_general", "test_step", "test_rates", "RATE_KINDS", "STATE_WORDS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlx.so")
STATE_WORDS = 10

_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p
_int = ctypes.c_int

_SIGS = {
    "rlx_strerror": (ctypes.c_char_p, [_int]),
    "rlx_version": (ctypes.c_char_p, []),
    "rlx_prepare": (_int, [_u32, _vp]),
    "rlx_init_streams": (_int, [_vp, _u64, _vp, _u64, _u32, _vp]),
    "rlx_skip": (_int, [_vp, _u64, _vp, _u64, _u32, _vp]),
    "rlx_skip_values": (_int, [_vp, _u64, _vp, _u64, _u32, _vp]),
    "rlx_export_ranlux": (_int, [_vp, _u64, _vp, _vp, _vp, _vp]),
    "rlx_import_ranlux": (_int, [_vp, _u64, _vp, _vp, _vp, _u32, _vp]),
    "rlx_generate_f64": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_generate_u64": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_generate_normal_f64": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_generate_f32": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_generate_f64_lcg52": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_get_tables": (_int, [_u32, _vp, _vp]),
    "rlx_build_tables_static": (_int, [_u32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "rlx_test_engine": (_int, [_vp, _u64, _u64, _vp, _u32, _u32, _vp]),
    "rlx_generate_f64_trace": (_int, [_vp, _u64, _u64, _vp, _vp, _u64, _u32, _vp]),
    "rlx_check_errors": (_int, [_vp, ctypes.POINTER(_u32)]),
    "rlx_set_lanes_per_stream": (_int, [_u32]),
    "rlx_lanes_per_stream": (_u32, [_u64, _u64]),
    "rlx_set_step_kernel": (_int, [_int]),
    "rlx_step_kernel": (_int, []),
    "rlx_constants": (None, [ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "rlx_plan_create": (_int, [ctypes.POINTER(_vp), _vp, _u64, _u32, _u64, _u64, _vp]),
    "rlx_plan_update": (_int, [_vp, _vp, _u64, _vp]),
    "rlx_plan_info": (_int, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "rlx_plan_generate_f64": (_int, [_vp, _vp, _vp, _vp]),
    "rlx_plan_generate_u64": (_int, [_vp, _vp, _vp, _vp]),
    "rlx_plan_generate_f32": (_int, [_vp, _vp, _vp, _vp]),
    "rlx_plan_destroy": (_int, [_vp]),
    "rlx_plan_dry_run": (_int, [_vp, _u64, _u32, _u64, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                ctypes.POINTER(_u64), _vp, _u64]),
    "rlx_test_mulmod": (_int, [_vp, _vp, _vp, _u64, _vp]),
    "rlx_test_pow": (_int, [_vp, _vp, _vp, _u64, _vp]),
    "rlx_test_to_ranlux": (_int, [_vp, _vp, _vp, _u64, _vp]),
    "rlx_test_generate_u64_general": (_int, [_vp, _u64, _u64, _vp, _u32, _vp]),
    "rlx_test_step": (_int, [_vp, _vp, _u64, _u32, _u32, _int, _int, _vp]),
    "rlx_test_rates": (_int, [_int, _u32, _vp, _u64, _vp]),
}

_lib = None

# struct rlx_request: state, start, count, out_offset (uint64), p, reserved (uint32)
import numpy as _np  # noqa: E402

REQUEST_DTYPE = _np.dtype([("state", "<u8"), ("start", "<u8"), ("count", "<u8"),
                           ("out_offset", "<u8"), ("p", "<u4"), ("reserved", "<u4")])
assert REQUEST_DTYPE.itemsize == 40


class RlxError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().rlx_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded librlx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2106_02504_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(code: int, where: str) -> None:
    if code != 0:
        raise RlxError(code, where)


def _stream(device: torch.device | None = None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _need_states(states: torch.Tensor) -> int:
    if states.dtype != torch.int64 or states.dim() != 2 or states.shape[1] != STATE_WORDS:
        raise ValueError("states must be an int64 tensor of shape [n, 10]")
    if not states.is_cuda or not states.is_contiguous():
        raise ValueError("states must be a contiguous device tensor")
    return states.shape[0]


def _need_u64_vector(t: torch.Tensor, n: int, what: str) -> None:
    if t.dtype not in (torch.int64, torch.uint64) or t.numel() != n or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous device int64/uint64 tensor with {n} elements")


def new_states(n: int, device: str | torch.device = "cuda") -> torch.Tensor:
    """Uninitialised-but-zeroed record array; fill it with init_streams()."""
    return torch.zeros((n, STATE_WORDS), dtype=torch.int64, device=device)


P_RECORD = 0   # p for skip/generate calls that use each record's own luxury level


def prepare(p: int) -> None:
    """Build the tables of luxury level p on the current device now."""
    _check(lib().rlx_prepare(p, _stream()), "rlx_prepare")


def init_streams(states: torch.Tensor, p: int, ids: torch.Tensor | None = None, id0: int = 0) -> torch.Tensor:
    """states[i] <- seed(ids[i] or id0 + i, p) (section 2.4)."""
    n = _need_states(states)
    if ids is not None:
        _need_u64_vector(ids, n, "ids")
    with torch.cuda.device(states.device):
        _check(lib().rlx_init_streams(states.data_ptr(), n, _ptr(ids), id0, p, _stream()), "rlx_init_streams")
    return states


def skip(states: torch.Tensor, steps, p: int) -> torch.Tensor:
    """Advance every record by `steps` generator steps (12 values each):
    an int for all, or a device tensor of n uint64/int64 (section 2.4).
    p = P_RECORD uses each record's own (prepared) level."""
    n = _need_states(states)
    if isinstance(steps, torch.Tensor):
        _need_u64_vector(steps, n, "steps")
        ptr, s0 = steps.data_ptr(), 0
    else:
        ptr, s0 = None, int(steps)
    with torch.cuda.device(states.device):
        _check(lib().rlx_skip(states.data_ptr(), n, ptr, s0, p, _stream()), "rlx_skip")
    return states


def skip_values(states: torch.Tensor, values, p: int) -> torch.Tensor:
    """Advance every record by `values` draws (an int, or a device tensor of
    n uint64/int64)."""
    n = _need_states(states)
    if isinstance(values, torch.Tensor):
        _need_u64_vector(values, n, "values")
        ptr, v0 = values.data_ptr(), 0
    else:
        ptr, v0 = None, int(values)
    with torch.cuda.device(states.device):
        _check(lib().rlx_skip_values(states.data_ptr(), n, ptr, v0, p, _stream()), "rlx_skip_values")
    return states


def export_ranlux(states: torch.Tensor):
    """(packed [n, 9] int64 = the 24 RANLUX numbers of the current step,
    carry [n] int32, pos [n] int32) of every record (section 2)."""
    n = _need_states(states)
    packed = torch.zeros((n, 9), dtype=torch.int64, device=states.device)
    carry = torch.zeros((n,), dtype=torch.int32, device=states.device)
    pos = torch.zeros((n,), dtype=torch.int32, device=states.device)
    with torch.cuda.device(states.device):
        _check(lib().rlx_export_ranlux(states.data_ptr(), n, packed.data_ptr(), carry.data_ptr(), pos.data_ptr(),
                                       _stream()), "rlx_export_ranlux")
    return packed, carry, pos


def import_ranlux(states: torch.Tensor, packed: torch.Tensor, carry: torch.Tensor, p: int,
                  pos: torch.Tensor | None = None) -> torch.Tensor:
    """Records from RANLUX-form states (canonical ones only; others are
    flagged in the error word and left unchanged): packed [n, 9] int64,
    carry [n] and pos [n] (optional) int32, on the states' device."""
    n = _need_states(states)

    def need(t, shape, dtypes, what):
        if (t.dtype not in dtypes or tuple(t.shape) != shape or not t.is_contiguous()
                or t.device != states.device):
            raise ValueError(f"{what} must be a contiguous {shape} tensor on the states' device")
    need(packed, (n, 9), (torch.int64, torch.uint64), "packed")
    need(carry, (n,), (torch.int32, torch.uint32), "carry")
    if pos is not None:
        need(pos, (n,), (torch.int32, torch.uint32), "pos")
    with torch.cuda.device(states.device):
        _check(lib().rlx_import_ranlux(states.data_ptr(), n, packed.data_ptr(), carry.data_ptr(), _ptr(pos), p,
                                       _stream()), "rlx_import_ranlux")
    return states


def _out(states: torch.Tensor, count: int, dtype: torch.dtype, out: torch.Tensor | None) -> torch.Tensor:
    n = states.shape[0]
    if out is None:
        return torch.empty((n, count), dtype=dtype, device=states.device)
    if out.dtype != dtype or out.numel() != n * count or not out.is_contiguous() or out.device != states.device:
        raise ValueError(f"out must be a contiguous {dtype} tensor with n*count elements on the states' device")
    return out


def generate_f64(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """`count` uniform doubles per record, shape [n, count] (section 2.3).
    p = P_RECORD draws each record at its own level (every level present
    prepared first); so do generate_u64, generate_f32 and
    generate_normal_f64."""
    n = _need_states(states)
    out = _out(states, count, torch.float64, out)
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_f64(states.data_ptr(), n, count, out.data_ptr(), p, _stream()), "rlx_generate_f64")
    return out


def generate_u64(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """The same draws as 48-bit integers (int64 tensor, values < 2^48)."""
    n = _need_states(states)
    out = _out(states, count, torch.int64, out)
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_u64(states.data_ptr(), n, count, out.data_ptr(), p, _stream()), "rlx_generate_u64")
    return out


def generate_normal_f64(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """`count` standard normal doubles per record, shape [n, count]: Box-Muller
    on the field pair of each position's step (include/rlx_gauss.hpp)."""
    n = _need_states(states)
    out = _out(states, count, torch.float64, out)
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_normal_f64(states.data_ptr(), n, count, out.data_ptr(), p, _stream()),
               "rlx_generate_normal_f64")
    return out


def generate_f32(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """`count` (even) float32 values per record, shape [n, count]: one RANLUX
    number v 2^-24 each, 24 per generator step (section 2.3); advances each
    record by count / 2 positions."""
    n = _need_states(states)
    out = _out(states, count, torch.float32, out)
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_f32(states.data_ptr(), n, count, out.data_ptr(), p, _stream()), "rlx_generate_f32")
    return out


def generate_f64_lcg52(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Legacy doubles from 52-bit slices of the LCG state (biased; for
    comparison only, section 2.3), shape [n, count], 11 per step; record
    positions count these values."""
    n = _need_states(states)
    out = _out(states, count, torch.float64, out)
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_f64_lcg52(states.data_ptr(), n, count, out.data_ptr(), p, _stream()),
               "rlx_generate_f64_lcg52")
    return out


class EngineTables(ctypes.Structure):
    """rlx_engine_tables: device addresses of a luxury level's tables, to be
    passed by value to kernels that use the device-side engine."""
    _fields_ = [("windows", ctypes.c_void_p), ("folded", ctypes.c_void_p), ("windows16", ctypes.c_void_p),
                ("p", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("mfma", ctypes.c_void_p)]


def get_tables(p: int, device=None) -> EngineTables:
    """The tables of level p on `device` (built on first use)."""
    t = EngineTables()
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        _check(lib().rlx_get_tables(p, ctypes.byref(t), _stream()), "rlx_get_tables")
    return t


def table_words(rows: int = 64) -> dict:
    """Sizes in 32-bit words of a level's tables (windows, folded, windows16,
    mfma) with `rows` step sizes."""
    return {"windows": 40 * 16 * 18, "folded": rows * 21 * 18, "windows16": 8 * 65536 * 18,
            "mfma": rows * 9 * 64 * 4}


def build_tables_static(p: int, rows: int, windows: torch.Tensor, folded: torch.Tensor,
                        windows16: torch.Tensor, mfma: torch.Tensor) -> None:
    """rlx_build_tables_static: build level p's tables into caller-owned
    int32 device tensors (sizes from table_words(rows)) on the current
    stream, allocating nothing; staging in the library's static array."""
    need = table_words(rows)
    for name, t in (("windows", windows), ("folded", folded), ("windows16", windows16), ("mfma", mfma)):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < need[name]:
            raise ValueError(f"{name}: contiguous int32 device tensor of >= {need[name]} words needed")
    with torch.cuda.device(windows.device):
        _check(lib().rlx_build_tables_static(p, rows, windows.data_ptr(), folded.data_ptr(), windows16.data_ptr(),
                                             mfma.data_ptr(), _stream()), "rlx_build_tables_static")


ENGINE_MODES = {"f64": 0, "seed": 1, "skip": 2, "normal": 3, "u48": 4, "sum": 5, "divergent": 6, "f32": 7}


def test_engine(states: torch.Tensor, count: int, p: int, mode: str) -> torch.Tensor:
    """Test hook: run the device-side engine (rlx_engine.h) from a kernel
    written as user code, one thread per record; returns [n, count] values
    (float64, or the u48 bits as int64 for mode "u48"; [n] sums for "sum";
    [n, 2 count] float32 for "f32")."""
    n = _need_states(states)
    m = ENGINE_MODES[mode]
    shape = (n,) if mode == "sum" else (n, count)
    out = torch.empty(shape, dtype=torch.float64, device=states.device)
    with torch.cuda.device(states.device):
        _check(lib().rlx_test_engine(states.data_ptr(), n, count, out.data_ptr(), m, p, _stream()),
               "rlx_test_engine")
    if mode == "u48":
        return out.view(torch.int64)
    if mode == "f32":
        return out.view(torch.float32)
    return out


def generate_f64_trace(states: torch.Tensor, count: int, p: int, out: torch.Tensor | None = None,
                       trace: torch.Tensor | None = None):
    """generate_f64 plus the LCG state of every step visited:
    returns (values [n, count], trace [n, steps, 9] int64), steps =
    (11 + count) // 12 + 1; `out` and `trace` may be given (trace rows past
    the last state visited are left as they are)."""
    n = _need_states(states)
    steps = (11 + count) // 12 + 1
    out = _out(states, count, torch.float64, out)
    if trace is None:
        trace = torch.zeros((n, steps, 9), dtype=torch.int64, device=states.device)
    elif (trace.dtype != torch.int64 or tuple(trace.shape) != (n, steps, 9) or not trace.is_contiguous()
          or trace.device != states.device):
        raise ValueError(f"trace must be a contiguous int64 tensor of shape {(n, steps, 9)} on {states.device}")
    with torch.cuda.device(states.device):
        _check(lib().rlx_generate_f64_trace(states.data_ptr(), n, count, out.data_ptr(), trace.data_ptr(),
                                            steps, p, _stream()), "rlx_generate_f64_trace")
    return out, trace


def set_lanes_per_stream(lanes: int) -> None:
    """Force G lanes per record for later generate calls (power of two
    <= 65536); 0 restores the automatic choice.  Values never depend on G."""
    _check(lib().rlx_set_lanes_per_stream(lanes), "rlx_set_lanes_per_stream")


def lanes_per_stream(n: int, count: int) -> int:
    """The G a generate call with n records and `count` values would use."""
    return int(lib().rlx_lanes_per_stream(n, count))


STEP_MFMA = 0   # generator step on the int8 matrix cores (default)
STEP_VALU = 1   # generator step as 32-bit multiply-adds on the vector ALU


def set_step_kernel(kind: int) -> None:
    """Choose how later generate calls multiply by A_p^G: STEP_MFMA or
    STEP_VALU (bit-identical values and records)."""
    _check(lib().rlx_set_step_kernel(kind), "rlx_set_step_kernel")


def step_kernel() -> int:
    """The current step kernel (STEP_MFMA or STEP_VALU)."""
    return int(lib().rlx_step_kernel())


def requests_array(state, start, count, p, out_offset=None) -> "_np.ndarray":
    """Build a host array of rlx_request from per-request sequences; output
    offsets default to the prefix sums of the counts."""
    state = _np.asarray(state, dtype=_np.uint64)
    n = state.shape[0]
    a = _np.zeros(n, dtype=REQUEST_DTYPE)
    a["state"] = state
    a["start"] = _np.broadcast_to(_np.asarray(start, dtype=_np.uint64), (n,))
    a["count"] = _np.asarray(count, dtype=_np.uint64)
    a["p"] = _np.broadcast_to(_np.asarray(p, dtype=_np.uint32), (n,))
    if out_offset is None:
        off = _np.zeros(n, dtype=_np.uint64)
        if n > 1:
            off[1:] = _np.cumsum(a["count"][:-1], dtype=_np.uint64)
        a["out_offset"] = off
    else:
        a["out_offset"] = _np.asarray(out_offset, dtype=_np.uint64)
    return a


class Plan:
    """A batch of requests planned for the batched kernel (rlx_plan_*).

    `requests` is a host array of REQUEST_DTYPE.  lanes: lanes per segment
    (power of two <= 64); seg_blocks: maximum generator steps per segment.
    """

    def __init__(self, requests, lanes: int = 8, seg_blocks: int = 2048, capacity_segments: int = 0,
                 device: torch.device | str | None = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        req = _np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        self._h = _vp()
        with torch.cuda.device(self.device):
            _check(lib().rlx_plan_create(ctypes.byref(self._h), req.ctypes.data, req.shape[0], lanes, seg_blocks,
                                         capacity_segments, _stream()), "rlx_plan_create")
        self.lanes, self.seg_blocks = lanes, seg_blocks
        self.extent, self.records = self._extent(req)

    @staticmethod
    def _extent(req) -> tuple[int, int]:
        """(output elements, records) the requests need: max of out_offset +
        count and of state + 1 over requests with count > 0 (the library
        accepted them, so these sums do not overflow)."""
        live = req[req["count"] > 0]
        if not live.shape[0]:
            return 0, 0
        return int((live["out_offset"] + live["count"]).max()), int(live["state"].max()) + 1

    def update(self, requests) -> None:
        req = _np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        with torch.cuda.device(self.device):
            _check(lib().rlx_plan_update(self._h, req.ctypes.data, req.shape[0], _stream()), "rlx_plan_update")
        self.extent, self.records = self._extent(req)

    def _check_out(self, states: torch.Tensor, out: torch.Tensor, dtype: torch.dtype, per_value: int) -> None:
        if _need_states(states) < self.records:
            raise ValueError(f"the requests read record {self.records - 1}; states holds {states.shape[0]}")
        if out.dtype != dtype or not out.is_contiguous() or out.device != states.device:
            raise ValueError(f"out must be a contiguous {dtype} tensor on the states' device")
        if out.numel() < per_value * self.extent:
            raise ValueError(f"out holds {out.numel()} elements; the requests need {per_value * self.extent}")

    def info(self) -> dict:
        a, b, c = _u64(0), _u64(0), _u64(0)
        _check(lib().rlx_plan_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "rlx_plan_info")
        return {"segments": a.value, "items": b.value, "values": c.value}

    def generate_f64(self, states: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        self._check_out(states, out, torch.float64, 1)
        with torch.cuda.device(states.device):
            _check(lib().rlx_plan_generate_f64(self._h, states.data_ptr(), out.data_ptr(), _stream()),
                   "rlx_plan_generate_f64")
        return out

    def generate_u64(self, states: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        self._check_out(states, out, torch.int64, 1)
        with torch.cuda.device(states.device):
            _check(lib().rlx_plan_generate_u64(self._h, states.data_ptr(), out.data_ptr(), _stream()),
                   "rlx_plan_generate_u64")
        return out

    def generate_f32(self, states: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """Two floats per requested position: value j of a request goes to
        out[2 (out_offset + j)] and out[2 (out_offset + j) + 1]."""
        self._check_out(states, out, torch.float32, 2)
        with torch.cuda.device(states.device):
            _check(lib().rlx_plan_generate_f32(self._h, states.data_ptr(), out.data_ptr(), _stream()),
                   "rlx_plan_generate_f32")
        return out

    def close(self) -> None:
        if self._h:
            _check(lib().rlx_plan_destroy(self._h), "rlx_plan_destroy")
            self._h = _vp()

    def __del__(self):
        try:
            if self._h:
                lib().rlx_plan_destroy(self._h)
        except Exception:
            pass


def batch(states: torch.Tensor, requests, out: torch.Tensor | None = None, lanes: int = 64,
          seg_blocks: int = 4096, dtype: torch.dtype = torch.float64) -> torch.Tensor:
    """One-shot batched generation: plan `requests` (REQUEST_DTYPE, e.g. from
    requests_array), run the batched launch and free the plan (which
    synchronises the device).  dtype float64, int64 (the 48-bit values) or
    float32 (two floats per position).  `out` is allocated to the requests'
    extent when None.  For repeated batches keep a Plan, whose launches can be
    captured in a HIP graph, or use serve.Server."""
    per = {torch.float64: 1, torch.int64: 1, torch.float32: 2}
    if dtype not in per:
        raise ValueError("dtype must be float64, int64 or float32")
    plan = Plan(requests, lanes=lanes, seg_blocks=seg_blocks, device=states.device)
    try:
        if out is None:
            out = torch.empty(per[dtype] * plan.extent, dtype=dtype, device=states.device)
        {torch.float64: plan.generate_f64, torch.int64: plan.generate_u64,
         torch.float32: plan.generate_f32}[dtype](states, out)
    finally:
        plan.close()
    return out


def plan_dry_run(requests, lanes: int = 8, seg_blocks: int = 2048):
    """Host-only planner run (no GPU): returns (segments [k, 6] uint64 array
    in launch order, n_items, total values); see rlx_plan_dry_run."""
    req = _np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
    ns, ni, tv = _u64(0), _u64(0), _u64(0)
    _check(lib().rlx_plan_dry_run(req.ctypes.data, req.shape[0], lanes, seg_blocks, ctypes.byref(ns),
                                  ctypes.byref(ni), ctypes.byref(tv), None, 0), "rlx_plan_dry_run")
    segs = _np.zeros((ns.value, 6), dtype=_np.uint64)
    if ns.value:
        _check(lib().rlx_plan_dry_run(req.ctypes.data, req.shape[0], lanes, seg_blocks, None, None, None,
                                      segs.ctypes.data, ns.value), "rlx_plan_dry_run")
    return segs, ni.value, tv.value


def check_errors() -> int:
    """Synchronise and return (and clear) the device error bits."""
    flags = _u32(0)
    code = lib().rlx_check_errors(_stream(), ctypes.byref(flags))
    if code not in (0, 4):
        _check(code, "rlx_check_errors")
    return flags.value


def constants() -> tuple[int, int]:
    """(m, a) as the library holds them (host-only call)."""
    m = (_u32 * 18)()
    a = (_u32 * 18)()
    lib().rlx_constants(m, a)
    return (sum(int(w) << (32 * k) for k, w in enumerate(m)),
            sum(int(w) << (32 * k) for k, w in enumerate(a)))


# ---- test-only entry points ------------------------------------------------

def _need_words(t: torch.Tensor, n: int | None, what: str, words: int = 9) -> int:
    """A contiguous device int64/uint64 tensor of shape [n, words]."""
    if (t.dtype not in (torch.int64, torch.uint64) or t.dim() != 2 or t.shape[1] != words or not t.is_cuda
            or not t.is_contiguous() or (n is not None and t.shape[0] != n)):
        raise ValueError(f"{what} must be a contiguous device int64 tensor of shape [n, {words}]")
    return t.shape[0]


def test_mulmod(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    n = _need_words(x, None, "x")
    _need_words(y, n, "y")
    out = torch.empty_like(x)
    _check(lib().rlx_test_mulmod(x.data_ptr(), y.data_ptr(), out.data_ptr(), n, _stream()), "rlx_test_mulmod")
    return out


def test_pow(base: torch.Tensor, exps: torch.Tensor) -> torch.Tensor:
    n = _need_words(base, None, "base")
    _need_words(exps, n, "exps", words=3)
    out = torch.empty_like(base)
    _check(lib().rlx_test_pow(base.data_ptr(), exps.data_ptr(), out.data_ptr(), n, _stream()), "rlx_test_pow")
    return out


def test_step(x: torch.Tensor, p: int, g: int, kind: int = STEP_MFMA, general: bool = False) -> torch.Tensor:
    """One generator step by 2^g steps (A_p^(2^g) x mod m) with the given
    step kernel, on int64 [n, 9] states x < m."""
    n = _need_words(x, None, "x")
    out = torch.empty_like(x)
    with torch.cuda.device(x.device):
        _check(lib().rlx_test_step(x.data_ptr(), out.data_ptr(), n, p, g, kind, int(general), _stream()),
               "rlx_test_step")
    return out


# rlx_test_rates kinds: (name, instructions per iteration per lane, unit)
RATE_KINDS = {0: ("v_mad_u64_u32", 64), 1: ("add_with_carry_valu", 80), 2: ("v_fma_f64", 64),
              3: ("v_mfma_i32_32x32x32_i8", 18)}


def test_rates(kind: int, iters: int, n_threads: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Launch the instruction-rate microbenchmark `kind` (see RATE_KINDS) on
    the current stream; returns the (meaningless) output words."""
    if out is None:
        out = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    _check(lib().rlx_test_rates(kind, iters, out.data_ptr(), n_threads, _stream()), "rlx_test_rates")
    return out


def test_to_ranlux(x: torch.Tensor):
    n = _need_words(x, None, "x")
    d = torch.empty_like(x)
    carry = torch.empty((n,), dtype=torch.int32, device=x.device)
    _check(lib().rlx_test_to_ranlux(x.data_ptr(), d.data_ptr(), carry.data_ptr(), n, _stream()),
           "rlx_test_to_ranlux")
    return d, carry


def test_generate_u64_general(states: torch.Tensor, count: int, p: int) -> torch.Tensor:
    n = _need_states(states)
    out = _out(states, count, torch.int64, None)
    _check(lib().rlx_test_generate_u64_general(states.data_ptr(), n, count, out.data_ptr(), p, _stream()),
           "rlx_test_generate_u64_general")
    return out
