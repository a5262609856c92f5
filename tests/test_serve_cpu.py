"""The serving loop's output-arena allocator, on the CPU: first fit,
coalescing on release, fragmentation, and zero-length ranges."""
import random

import pytest

from paper_2106_02504_amd.serve import Arena


def test_first_fit_and_coalescing():
    a = Arena(100)
    assert a.alloc(30) == 0 and a.alloc(30) == 30 and a.alloc(30) == 60
    assert a.alloc(11) is None                    # only 10 left
    a.release(30, 30)                             # hole in the middle
    assert a.used == 60 and a.free == [(30, 30), (90, 10)]
    assert a.alloc(20) == 30                      # first fit takes the hole
    a.release(0, 30)
    a.release(30, 20)
    assert a.free == [(0, 60), (90, 10)]          # neighbours merged
    a.release(60, 30)
    assert a.free == [(0, 100)] and a.used == 0


def test_fragmentation_blocks_a_large_request():
    a = Arena(64)
    offs = [a.alloc(8) for _ in range(8)]
    for o in offs[::2]:
        a.release(o, 8)
    assert a.used == 32
    assert a.alloc(16) is None                    # 32 free, but no 16 in one piece
    a.release(offs[1], 8)                         # joins the free ranges at 0 and 16
    assert a.alloc(16) == 0


def test_zero_length_ranges_leave_no_trace():
    a = Arena(10)
    o = a.alloc(0)
    assert o == 0 and a.free == [(0, 10)] and a.used == 0
    b = a.alloc(4)
    a.release(o, 0)
    a.release(b, 4)
    assert [r for r in a.free if r[1] > 0] == [(0, 10)] and a.used == 0


@pytest.mark.parametrize("seed", range(5))
def test_random_traffic_never_overlaps(seed):
    rng = random.Random(seed)
    cap = 1000
    a = Arena(cap)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            o = rng.choice(list(live))
            a.release(o, live.pop(o))
        else:
            n = rng.randint(1, 120)
            o = a.alloc(n)
            if o is not None:
                assert 0 <= o and o + n <= cap
                for p, m in live.items():          # no overlap with a live range
                    assert o + n <= p or p + m <= o
                live[o] = n
        assert a.used == sum(live.values())
        free = sum(ln for _, ln in a.free)
        assert free + a.used == cap                # every value is free or live, once
