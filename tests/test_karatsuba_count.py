"""The one-level Karatsuba form of the generic 576-bit product (tests/
host_arith/karatsuba.hip), measured against the library's schoolbook
product: its products are checked exactly against Python integers on the
host, then both forms are compiled to gfx950 assembly and their vector
instructions counted.

Karatsuba removes 99 of the 441 digit products (section 2.1's product
written as three half-size products), but the recombination adds two
64-bit subtractions per middle column and a signed carry, and a
v_mad_u64_u32 issues at the same rate as the add-with-carry pairs it is
traded for.  The count shows no saving, which is why the library keeps the
schoolbook product."""
import os
import random
import re
import subprocess
from collections import Counter

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SRC = os.path.join(ROOT, "tests", "host_arith", "karatsuba.hip")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def built(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("karatsuba")
    exe, asm = str(d / "karatsuba"), str(d / "karatsuba.s")
    subprocess.run([HIPCC, *FLAGS, "-o", exe, SRC], check=True, capture_output=True)
    subprocess.run([HIPCC, *FLAGS, "--cuda-device-only", "-S", "-o", asm, SRC], check=True, capture_output=True)
    return exe, asm


def test_karatsuba_products_are_exact(built, tmp_path):
    rng = random.Random(9)
    top = (1 << 576) - 1
    pairs = [(top, top), (0, top), (1, top), (top, 1 << 575), ((1 << 308) - 1, (1 << 308) - 1),
             ((1 << 308) | 1, top)]
    for _ in range(3000):
        a, b = rng.getrandbits(576), rng.getrandbits(576)
        if rng.random() < 0.3:   # long runs of ones and zeros in the digits
            mask = rng.getrandbits(576)
            a, b = (a | mask) if rng.random() < 0.5 else (a & mask), b | mask
        pairs.append((a, b))
    src = tmp_path / "in.txt"
    with open(src, "w") as f:
        f.write(f"{len(pairs)}\n")
        for a, b in pairs:
            f.write(" ".join(f"{(v >> (32 * k)) & 0xFFFFFFFF:x}" for v in (a, b) for k in range(18)) + "\n")
    out = tmp_path / "out.txt"
    subprocess.run([built[0], str(src), str(out)], check=True)
    rows = open(out).read().split("\n")
    for (a, b), row in zip(pairs, rows):
        got = sum(int(w, 16) << (32 * k) for k, w in enumerate(row.split()))
        assert got == a * b, (hex(a), hex(b))


def vector_instructions(asm, kernel):
    body = asm.split(kernel + ":", 1)[1].split(".Lfunc_end", 1)[0]
    ops = [m.group(1) for m in re.finditer(r"^\s+(v_\w+)", body, re.M)]
    return len(ops), Counter(ops)["v_mad_u64_u32"]


def test_karatsuba_saves_no_vector_instructions(built):
    asm = open(built[1]).read()
    school, school_mads = vector_instructions(asm, "k_product_schoolbook")
    kara, kara_mads = vector_instructions(asm, "k_product_karatsuba")
    print(f"schoolbook: {school} vector instructions ({school_mads} v_mad_u64_u32); "
          f"Karatsuba: {kara} ({kara_mads})")
    assert school_mads - kara_mads >= 90         # the 99 digit products it removes
    assert kara >= 0.97 * school                 # but the total stays within 3% (or grows)
