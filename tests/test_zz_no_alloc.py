"""rlx_build_tables_static, the entry point for callers that cannot allocate:
it builds a luxury level's tables into caller-owned device memory with its
staging in the library's static device array.  Checked word for word
against the library-owned tables of rlx_get_tables (the existing entry
point), on two calls in a row, the second one smaller; the device's free
memory must not change across the calls."""
import ctypes

import pytest
import torch

import paper_2106_02504_amd as rlx

pytestmark = pytest.mark.gpu


def _hip():
    # the HIP runtime torch loaded (the library binds to the same one)
    for line in open("/proc/self/maps"):
        if "libamdhip64" in line:
            return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("HIP runtime not loaded")


HIP = None


def device_words(addr: int, nwords: int) -> torch.Tensor:
    """Copy nwords 32-bit words at device address addr into a new tensor."""
    global HIP
    HIP = HIP or _hip()
    t = torch.empty(nwords, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = HIP.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(addr), ctypes.c_size_t(4 * nwords), 3)
    assert rc == 0
    return t


def free_bytes() -> int:
    global HIP
    HIP = HIP or _hip()
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    torch.cuda.synchronize()
    assert HIP.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def library_tables(p, rows):
    t = rlx.get_tables(p)
    w = rlx.table_words(rows)
    return {"windows": device_words(t.windows, w["windows"]), "folded": device_words(t.folded, w["folded"]),
            "windows16": device_words(t.windows16, w["windows16"]), "mfma": device_words(t.mfma, w["mfma"])}


def test_static_table_build_matches_library_tables():
    full = rlx.table_words(64)
    sentinel = -0x21524111  # 0xDEADBEEF
    bufs = {k: torch.full((n,), sentinel, dtype=torch.int32, device="cuda") for k, n in full.items()}
    ref = {p: library_tables(p, 64) for p in (2048, 218)}   # the library's own build (allocates)
    # first call: every step size, p = 2048; the device's free memory is the
    # same before and after (measured around the call alone)
    before = free_bytes()
    rlx.build_tables_static(2048, 64, bufs["windows"], bufs["folded"], bufs["windows16"], bufs["mfma"])
    assert free_bytes() == before
    for k in full:
        assert torch.equal(bufs[k], ref[2048][k]), k
    # second call, smaller: five step sizes of p = 218 into the same buffers
    for b in bufs.values():
        b.fill_(sentinel)
    before = free_bytes()
    rlx.build_tables_static(218, 5, bufs["windows"], bufs["folded"], bufs["windows16"], bufs["mfma"])
    assert free_bytes() == before
    small = rlx.table_words(5)
    for k in full:
        assert torch.equal(bufs[k][:small[k]], ref[218][k][:small[k]]), k
        assert bool((bufs[k][small[k]:] == sentinel).all()), k     # rows past `rows` untouched


def test_static_table_build_rejects_oversize_and_bad_arguments():
    lib = rlx.lib()
    w = rlx.table_words(64)
    bufs = [torch.zeros(w[k], dtype=torch.int32, device="cuda") for k in ("windows", "folded", "windows16", "mfma")]
    ptrs = [b.data_ptr() for b in bufs]
    assert lib.rlx_build_tables_static(2048, 65, *ptrs, None) == 6          # RLX_ESCRATCH
    assert b"static device array" in lib.rlx_strerror(6)
    assert lib.rlx_build_tables_static(2048, 0, *ptrs, None) == 1
    assert lib.rlx_build_tables_static(23, 4, *ptrs, None) == 1
    assert lib.rlx_build_tables_static(2048, 4, None, *ptrs[1:], None) == 1
    assert lib.rlx_build_tables_static(2048, 4, *ptrs[:3], ptrs[3] + 4, None) == 1   # mfma not 16-byte aligned
    torch.cuda.synchronize()
    assert all(int(b.abs().sum()) == 0 for b in bufs)                     # nothing was enqueued
