"""The library's 576-bit arithmetic (include/rlx_arith.hpp) compiled for the
host and checked against the oracle on the CPU: generic mulmod, the folded
constant-multiplier step (fast path and forced general path), the conversion
to RANLUX numbers (both paths), the carry and the fields, on random operands
and on operands crafted to reach every rare branch."""
import os
import random
import shutil
import subprocess

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def words(v, n=18):
    return [(v >> (32 * k)) & 0xFFFFFFFF for k in range(n)]


def from_words(ws):
    return sum(int(w, 16) << (32 * k) for k, w in enumerate(ws))


def limb_offsets():
    """Bit offsets of the 21 limbs of the library's constant-multiplier step
    (ten 28-bit, ten 27-bit, one 26-bit limb): its table rows are
    A 2^offset mod m."""
    widths = [28] * 10 + [27] * 10 + [26]
    assert sum(widths) == 576 and sum(1 << w for w in widths) <= 1 << 32
    return [sum(widths[:j]) for j in range(21)]


def setw(x, k, v):
    return (x & ~(0xFFFFFFFF << (32 * k))) | (v << (32 * k))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("host_arith")
    exe = str(d / "harness")
    src = os.path.join(ROOT, "tests", "host_arith", "harness.hip")
    inc = os.path.join(ROOT, "include")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", inc, "-I",
                    os.path.join(ROOT, "include"), "-o", exe, src], check=True, capture_output=True)
    return exe


def cases(rng):
    m = O.M
    xs = [0, 1, 2, m - 1, m - 2, 2 ** 336 - 1, 2 ** 336, 2 ** 336 + 1, 2 ** 240 - 1, 2 ** 240,
          2 ** 576 - 2 ** 240, (m - 1) // 2, 2 ** 575, m - 2 ** 240]
    for _ in range(150):
        x = rng.randrange(m)
        xs.append(setw(x, 17, (x >> 304) & 0xFFFFFFFF))
        xs.append(setw(setw(setw(x, 7, 0xFFFFFFFF), 8, 0xFFFFFFFF), 9, 0xFFFFFFFF))
        xs.append(setw(x, 0, (-((x >> 336) & 0xFFFFFFFF)) & 0xFFFFFFFF))
        xs.append(setw(setw(x, 17, 0xFFFFFFFE), 16, 0xFFFFFFFF))
    xs += [rng.randrange(m) for _ in range(1500)]
    return [x for x in xs if x < m]


@pytest.mark.parametrize("p", (24, 2048))
def test_host_build_matches_oracle(harness, tmp_path, p):
    rng = random.Random(p)
    a_p = O.multiplier(p)
    tab = []
    for off in limb_offsets():
        tab += words(a_p * (1 << off) % O.M)
    xs = cases(rng)
    # step results that land on chosen values (top word all ones, m - 1, ...)
    inv = pow(a_p, -1, O.M)
    for t in (O.M - 1, O.M - 2, 1, 2 ** 576 - 2 ** 240 - 5, 2 ** 544 - 1):
        xs.append(t * inv % O.M)
    ys = [rng.getrandbits(576) for _ in xs]
    ys[:4] = [2 ** 288 - 1, O.M - 1, 2 ** 576 - 1, O.M]
    xs[:3] = [(2 ** 288 + 1), O.M - 1, 2 ** 576 - 2 ** 240 - 1]
    inp = tmp_path / "in.txt"
    outp = tmp_path / "out.txt"
    with open(inp, "w") as f:
        f.write(" ".join("%x" % v for v in tab) + "\n%d\n" % len(xs))
        for x, y in zip(xs, ys):
            f.write(" ".join("%x" % v for v in words(x)) + "\n" + " ".join("%x" % v for v in words(y)) + "\n")
    subprocess.run([harness, str(inp), str(outp)], check=True)
    lines = open(outp).read().split("\n")
    for i, (x, y) in enumerate(zip(xs, ys)):
        L = lines[i * 7:(i + 1) * 7]
        r, s1, s2 = (from_words(l.split()) for l in L[:3])
        assert r == x * y % O.M, i
        if x < O.M:
            exp_step = a_p * x % O.M
            assert s1 == exp_step and s2 == exp_step, i
            d1, d2 = (from_words(l.split()) for l in L[3:5])
            nums, c = O.to_ranlux(x)
            assert d1 == d2 == O.RANLUX.pack(nums), i
            assert int(L[5]) == c
            fl = L[6].split()
            f = O.fields(x)
            for k in range(12):
                assert int(fl[2 * k], 16) == f[k]
                assert float.fromhex(fl[2 * k + 1]) == O.field_to_double(f[k])
