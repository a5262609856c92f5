"""The library's Box-Muller evaluation (include/rlx_gauss.hpp) compiled for
the host and checked on the CPU against 40-digit values: ln(1 - u1),
cos(2 pi u2), sin(2 pi u2) and the two normals of a field pair, on pairs
crafted at the edges of both range reductions and on random pairs.

rlx_gauss.hpp uses only correctly rounded binary64 operations (basic
arithmetic, fma, rint, division, sqrt) with contraction off, so the host
build computes the device's bits; the device values themselves are compared
with the oracle in tests/test_gpu_normal.py.

Bounds: ln, cos and sin each within 1.5 ulp (a single final rounding of a
result whose other errors stay below an ulp), the normals within 4 ulp (the
radius carries half the log's error plus its own rounding, the product adds
half an ulp).  Results below 2^-60 in magnitude (the exact zeros of cos and
sin at quarter turns, which the 40-digit reference gives as tiny values) are
held to an absolute 2^-70."""
import math
import os
import random
import subprocess

import mpmath
import pytest

from oracle import gauss as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
M48 = (1 << 48) - 1


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("host_gauss")
    exe = str(d / "gauss_harness")
    src = os.path.join(ROOT, "tests", "host_arith", "gauss_harness.hip")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, src], check=True, capture_output=True)
    return exe


def crafted_pairs(rng):
    pairs = []
    # w = 1 - u1 = n 2^-48 around sqrt(1/2) 2^-k (where the log's reduction
    # switches binade) and around the powers of two
    for k in range(49):
        base = int(mpmath.floor(mpmath.sqrt(0.5) * mpmath.mpf(2) ** (48 - k)))
        for n in [base + d for d in (-2, -1, 0, 1, 2)] + [(1 << (48 - k)) + d for d in (-1, 0, 1)]:
            if 1 <= n <= 1 << 48:
                pairs.append(((1 << 48) - n, rng.getrandbits(48)))
    # t = 4 u2 at and around the quarter turns (j changes, phi = 0) and the
    # odd eighth turns (phi = +-pi/4)
    v2s = [0, 1, 2, M48, M48 - 1]
    for q in range(5):
        for d in (-3, -1, 0, 1, 3):
            v2s.append(q * (1 << 46) + d)
        for d in (-1, 0, 1):
            v2s.append(q * (1 << 46) + (1 << 45) + d)
    for v2 in (v for v in v2s if 0 <= v <= M48):
        pairs += [(rng.getrandbits(48), v2), (0, v2), (1, v2), (M48, v2)]
    return pairs


def run(harness, tmp_path, pairs):
    src = tmp_path / "in.txt"
    with open(src, "w") as f:
        f.write(f"{len(pairs)}\n")
        for v1, v2 in pairs:
            x = v1 | (v2 << 48)
            f.write(f"{x & 0xFFFFFFFF:x} {(x >> 32) & 0xFFFFFFFF:x} {x >> 64:x}\n")
    out = tmp_path / "out.txt"
    subprocess.run([harness, str(src), str(out)], check=True)
    return [[float.fromhex(v) for v in line.split()] for line in open(out)]


def err_ulp(got, want):
    if abs(want) < 2.0 ** -60:
        assert abs(got - want) <= 2.0 ** -70, (got, want)
        return 0.0
    return abs(got - want) / math.ulp(abs(want))


def test_box_muller_host_build_against_40_digits(harness, tmp_path):
    rng = random.Random(7)
    pairs = crafted_pairs(rng) + [(rng.getrandbits(48), rng.getrandbits(48)) for _ in range(4000)]
    rows = run(harness, tmp_path, pairs)
    assert len(rows) == len(pairs)
    worst = {"ln": 0.0, "cos": 0.0, "sin": 0.0, "normal": 0.0}
    with mpmath.workdps(40):
        for (v1, v2), (ln, c, s, zc, zs) in zip(pairs, rows):
            u1 = mpmath.mpf(v1) * mpmath.mpf(2) ** -48
            ang = 2 * mpmath.pi * mpmath.mpf(v2) * mpmath.mpf(2) ** -48
            worst["ln"] = max(worst["ln"], err_ulp(ln, float(mpmath.log(1 - u1))))
            worst["cos"] = max(worst["cos"], err_ulp(c, float(mpmath.cos(ang))))
            worst["sin"] = max(worst["sin"], err_ulp(s, float(mpmath.sin(ang))))
            for comp, z in ((0, zc), (1, zs)):
                worst["normal"] = max(worst["normal"], err_ulp(z, G.box_muller(v1, v2, comp)))
    print("max error (ulp):", {k: round(v, 3) for k, v in worst.items()})
    assert worst["ln"] <= 1.5 and worst["cos"] <= 1.5 and worst["sin"] <= 1.5, worst
    assert worst["normal"] <= 4.0, worst


def test_box_muller_exact_cases(harness, tmp_path):
    # u1 = 0 gives r = 0; quarter turns give exact +-1 and 0 factors;
    # u1 = 1 - 2^-48 gives the largest radius, sqrt(96 ln 2)
    pairs = [(0, 12345), (5, 0), (5, 1 << 46), (5, 2 << 46), (5, 3 << 46), (M48, 0)]
    rows = run(harness, tmp_path, pairs)
    assert rows[0][3] == 0.0 and rows[0][4] == 0.0
    for k, (c, s) in enumerate(((1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0))):
        assert rows[1 + k][1] == c and rows[1 + k][2] == s, k
    r = G.radius(M48)
    assert rows[5][3] == pytest.approx(r, rel=2.0 ** -51) and rows[5][4] == 0.0
    assert rows[5][0] == pytest.approx(-48 * math.log(2), rel=2.0 ** -52)


@pytest.mark.gpu
def test_device_normals_equal_host_build(harness, tmp_path):
    # the claim behind the bounds above: the device computes the host build's
    # bits (inputs are the oracle's field pairs; no GPU value feeds the host)
    import numpy as np
    import torch

    import oracle as O
    import paper_2106_02504_amd as rlx

    p, n, count = 2048, 48, 120
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=7)
    got = rlx.generate_normal_f64(st, count, p).cpu().numpy()
    pairs = []
    for i in range(n):
        v = O.draws(O.seed(7 + i, p), 0, p, count)[0]
        pairs += [(v[2 * k], v[2 * k + 1]) for k in range(count // 2)]
    rows = run(harness, tmp_path, pairs)
    want = np.array([[r[3], r[4]] for r in rows], dtype=np.float64).reshape(n, count)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert torch.cuda.is_available()
