"""Register budget of the main kernels, from the gfx950 compiler's own
resource report (-Rpass-analysis=kernel-resource-usage on the library's
sources, built with the library's flags): the occupancy each kernel was
designed for, and no scratch spills.

- k_generate, staged, matrix-core step, every output kind (uniform doubles,
  48-bit integers, float32, normals): 4 waves per SIMD without spills.  For
  normals this relies on the scheduling barrier after each field pair's
  transform; without it the six transforms interleave and need 166 VGPRs.
- k_skip and k_init: at least 5 waves per SIMD without spills.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
OUT_KINDS = {"U64": 0, "F64": 1, "NORMAL": 2, "F32": 3}


@pytest.fixture(scope="module")
def resources(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_2106_02504_amd import build as b
    obj = str(tmp_path_factory.mktemp("res") / "rlx.o")
    flags = [f for f in b.FLAGS if f not in ("-shared", "-fPIC")]
    res = subprocess.run([HIPCC, *flags, "--cuda-device-only", "-c", "-o", obj,
                          os.path.join(ROOT, "paper_2106_02504_amd", "csrc", "rlx.hip"),
                          "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True, check=True)
    table, name = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            table[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and name:
            table[name][m.group(1).split()[0]] = int(m.group(2))
    assert table, res.stderr[-2000:]
    return table


def generate_kernel(table, kind, lgs, mf=True):
    tag = f"k_generateILN3rlx3OutE{OUT_KINDS[kind]}ELb0ELi{lgs}ELb{int(mf)}E"
    hits = [v for k, v in table.items() if tag in k]
    assert len(hits) == 1, tag
    return hits[0]


@pytest.mark.parametrize("kind", ("F64", "U64", "F32", "NORMAL"))
@pytest.mark.parametrize("lgs", (1, 5, 6))
def test_generate_kernels_four_waves_no_spills(resources, kind, lgs):
    r = generate_kernel(resources, kind, lgs)
    print(kind, lgs, r)
    assert r["ScratchSize"] == 0, r
    assert r["Occupancy"] == 4, r
    assert r["VGPRs"] + r.get("AGPRs", 0) <= 128, r


@pytest.mark.parametrize("kernel", ("k_skipEP9rlx_state", "k_initEP9rlx_state"))
def test_seed_and_skip_kernels(resources, kernel):
    hits = [v for k, v in resources.items() if kernel in k]
    assert len(hits) == 1, kernel
    r = hits[0]
    print(kernel, r)
    assert r["ScratchSize"] == 0, r
    assert r["Occupancy"] >= 5, r
