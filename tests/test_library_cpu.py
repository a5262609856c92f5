"""Host-side checks of librlx.so that need no GPU: it loads, it exports every
symbol the public header declares, and its constants are the paper's."""
import ctypes
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rlx():
    import paper_2106_02504_amd as r
    return r


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("rlx_init_streams", "rlx_skip", "rlx_generate_f64", "rlx_generate_u64"):
        assert need in names


def test_library_exports_every_declared_symbol(rlx):
    lib = rlx.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    from paper_2106_02504_amd import _SIGS
    assert sorted(_SIGS) == declared_functions()


def test_library_constants_match_the_paper(rlx):
    m, a = rlx.constants()
    assert m == 2 ** 576 - 2 ** 240 + 1 == O.M
    assert a == O.A and (a << 24) % m == 1


def test_strerror_and_version(rlx):
    lib = rlx.lib()
    assert lib.rlx_strerror(0) == b"ok"
    assert b"invalid" in lib.rlx_strerror(1)
    assert lib.rlx_version().startswith(b"rlx")


def test_invalid_arguments_fail_before_any_device_work(rlx):
    lib = rlx.lib()
    # NULL states with n > 0, bad luxury levels, misaligned pointers
    assert lib.rlx_init_streams(None, 5, None, 0, 2048, None) == 1
    assert lib.rlx_generate_f64(None, 5, 10, None, 2048, None) == 1
    assert lib.rlx_skip(ctypes.c_void_p(16), 5, None, 0, 23, None) == 1
    assert lib.rlx_generate_u64(ctypes.c_void_p(8), 5, 10, ctypes.c_void_p(16), 2048, None) == 1
    assert lib.rlx_generate_f64(ctypes.c_void_p(16), 5, 10, ctypes.c_void_p(12), 2048, None) == 1
    assert lib.rlx_prepare(10, None) == 1
    # overflow of n * count
    assert lib.rlx_generate_f64(ctypes.c_void_p(16), 1 << 40, 1 << 40, ctypes.c_void_p(16), 2048, None) == 1
    # table accessor: bad level or NULL output
    assert lib.rlx_get_tables(23, ctypes.c_void_p(16), None) == 1
    assert lib.rlx_get_tables(2048, None, None) == 1
    assert lib.rlx_test_engine(ctypes.c_void_p(16), 5, 10, ctypes.c_void_p(16), 9, 2048, None) == 1
    # per-call size limits: n < 2^32 records, count <= 2^35 values
    assert lib.rlx_generate_f64(ctypes.c_void_p(16), 1 << 32, 1, ctypes.c_void_p(16), 2048, None) == 1
    assert lib.rlx_generate_u64(ctypes.c_void_p(16), 1, (1 << 35) + 1, ctypes.c_void_p(16), 2048, None) == 1
    # no-ops
    assert lib.rlx_generate_f64(None, 0, 10, None, 2048, None) == 0
    assert lib.rlx_generate_u64(None, 5, 0, None, 2048, None) == 0
    assert lib.rlx_skip(None, 0, None, 0, 2048, None) == 0


def test_other_widths_argument_checks(rlx):
    lib = rlx.lib()
    v = ctypes.c_void_p
    # float32 draws come in pairs: odd counts are rejected, even with n = 0
    assert lib.rlx_generate_f32(v(16), 5, 7, v(16), 2048, None) == 1
    assert lib.rlx_generate_f32(None, 0, 3, None, 2048, None) == 1
    assert lib.rlx_generate_f32(None, 0, 4, None, 2048, None) == 0
    assert lib.rlx_generate_f32(v(16), 5, 10, v(12), 2048, None) == 1      # out not 8-byte aligned
    assert lib.rlx_generate_f32(v(16), 1, 2 * ((1 << 35) + 1), v(16), 2048, None) == 1
    assert lib.rlx_generate_f32(v(16), 5, 10, v(16), 23, None) == 1
    # legacy doubles: same checks as the 48-bit doubles
    assert lib.rlx_generate_f64_lcg52(None, 5, 10, None, 2048, None) == 1
    assert lib.rlx_generate_f64_lcg52(v(16), 5, 10, v(12), 2048, None) == 1
    assert lib.rlx_generate_f64_lcg52(v(16), 1 << 32, 1, v(16), 2048, None) == 1
    assert lib.rlx_generate_f64_lcg52(None, 0, 10, None, 2048, None) == 0
    assert lib.rlx_plan_generate_f32(None, v(16), v(16), None) == 1
    assert lib.rlx_test_engine(v(16), 5, 10, v(16), 8, 2048, None) == 1


def test_record_level_argument_checks(rlx):
    lib = rlx.lib()
    v = ctypes.c_void_p
    assert rlx.P_RECORD == 0
    hdr = open(os.path.join(ROOT, "include", "rlx.h")).read()
    assert "#define RLX_P_RECORD 0u" in hdr and "#define RLX_MAX_RECORD_LEVELS 16" in hdr
    # one-level entry points refuse the per-record level
    assert lib.rlx_init_streams(v(16), 5, None, 0, 0, None) == 1
    assert lib.rlx_generate_f64_trace(v(16), 5, 10, v(16), v(16), 100, 0, None) == 1
    assert lib.rlx_generate_f64_lcg52(v(16), 5, 10, v(16), 0, None) == 1
    assert lib.rlx_test_generate_u64_general(v(16), 5, 10, v(16), 0, None) == 1
    # the per-record calls keep the argument checks of the others
    assert lib.rlx_generate_f64(v(16), 5, 10, v(12), 0, None) == 1
    assert lib.rlx_generate_u64(v(16), 1 << 32, 1, v(16), 0, None) == 1
    assert lib.rlx_generate_f32(v(16), 5, 7, v(16), 0, None) == 1
    assert lib.rlx_skip(v(16), 5, v(12), 0, 0, None) == 1
    assert lib.rlx_skip_values(None, 5, None, 0, 0, None) == 1
    # no-ops
    assert lib.rlx_generate_f64(None, 0, 10, None, 0, None) == 0
    assert lib.rlx_generate_normal_f64(None, 5, 0, None, 0, None) == 0
    assert lib.rlx_skip(None, 0, None, 0, 0, None) == 0


def test_automatic_lanes_per_stream(rlx):
    # host-only pick of lanes per record: powers of two within the launch
    # and step limits; more lanes for few streams, whole waves otherwise.
    # The limits depend on the step kernel: 2^21 lanes and 8 steps per lane
    # with the matrix-core step, 2^20 and 16 with the vector-ALU step.
    lib = rlx.lib()
    pick = rlx.lanes_per_stream
    try:
        for kind, target, min_steps, many in ((rlx.STEP_MFMA, 1 << 21, 8, 32), (rlx.STEP_VALU, 1 << 20, 16, 16)):
            assert lib.rlx_set_step_kernel(kind) == 0
            assert pick(65536, 4096) == many          # the many-streams shape
            assert pick(1, 1 << 20) == 65536          # one long stream fills the chip
            assert pick(1 << 21, 4096) == 1
            assert pick(1, 11) == 1 and pick(1, 12) == 2
            for n in (1, 3, 64, 100, 5000, 1 << 16, 1 << 21):
                for count in (1, 12, 1000, 1 << 16, 1 << 20, 1 << 22):
                    g = pick(n, count)
                    steps = count // 12 + 1
                    assert g & (g - 1) == 0 and 1 <= g <= 65536
                    assert g == 1 or (n * g <= target and steps // g >= 1)
                    assert g == 1 or steps // g >= min_steps or n * g <= 1 << 16
                    # the largest such power of two
                    g2 = 2 * g
                    assert (g2 > 65536 or n * g2 > target or steps // g2 == 0
                            or (steps // g2 < min_steps and n * g2 > 1 << 16))
        # the override: powers of two up to 65536, 0 restores the automatic pick
        assert lib.rlx_set_lanes_per_stream(65536) == 0 and pick(65536, 4096) == 65536
        assert lib.rlx_set_lanes_per_stream(131072) == 1 and lib.rlx_set_lanes_per_stream(48) == 1
        assert lib.rlx_set_lanes_per_stream(0) == 0 and pick(65536, 4096) == 16
    finally:
        lib.rlx_set_step_kernel(rlx.STEP_MFMA)
        lib.rlx_set_lanes_per_stream(0)


def test_ranlux_form_argument_checks(rlx):
    lib = rlx.lib()
    v = ctypes.c_void_p
    assert lib.rlx_export_ranlux(v(16), 3, v(16), v(2), None, None) == 1      # carry not 4-byte aligned
    assert lib.rlx_export_ranlux(v(16), 3, v(16), v(16), v(6), None) == 1     # pos not 4-byte aligned
    assert lib.rlx_import_ranlux(v(16), 3, v(16), v(2), None, 24, None) == 1
    assert lib.rlx_import_ranlux(v(16), 3, v(16), v(16), v(6), 24, None) == 1
    assert lib.rlx_import_ranlux(v(16), 3, v(12), v(16), None, 24, None) == 1  # packed not 8-byte aligned
    assert lib.rlx_import_ranlux(v(16), 3, v(16), v(16), None, 23, None) == 1
    assert lib.rlx_export_ranlux(None, 0, None, None, None, None) == 0


def test_plan_capacity_limit(rlx):
    # a capacity beyond 2^32 - 1 segments is rejected before any device work
    lib = rlx.lib()
    req = rlx.requests_array([0], [0], [10], 2048)
    h = ctypes.c_void_p()
    assert lib.rlx_plan_create(ctypes.byref(h), req.ctypes.data, 1, 8, 64, 1 << 33, None) == 1
    assert not h.value
    assert lib.rlx_plan_create(None, req.ctypes.data, 1, 8, 64, 0, None) == 1


def test_step_kernel_choice(rlx):
    # the step kernel switch: two kinds, anything else rejected, default MFMA
    lib = rlx.lib()
    assert lib.rlx_step_kernel() == rlx.STEP_MFMA == 0
    assert lib.rlx_set_step_kernel(2) == 1 and lib.rlx_set_step_kernel(-1) == 1
    assert lib.rlx_set_step_kernel(rlx.STEP_VALU) == 0 and lib.rlx_step_kernel() == rlx.STEP_VALU
    assert lib.rlx_set_step_kernel(rlx.STEP_MFMA) == 0 and lib.rlx_step_kernel() == rlx.STEP_MFMA
    # invalid arguments of the step test hook fail before any device work
    assert lib.rlx_test_step(None, None, 5, 2048, 0, 0, 0, None) == 1
    assert lib.rlx_test_step(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 2048, 64, 0, 0, None) == 1
    assert lib.rlx_test_step(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 2048, 0, 2, 0, None) == 1
