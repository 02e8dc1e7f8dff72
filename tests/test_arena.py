"""First-fit device arena of the serving loop (host logic only)."""
import random

import pytest

from paper_2211_00645_amd.arena import Arena, NoSpace


def test_alloc_free_coalesce():
    a = Arena(1 << 20, align=256)
    x = a.alloc(1000)
    y = a.alloc(5000)
    z = a.alloc(256)
    assert (x, y, z) == (0, 1024, 1024 + 5120)
    assert a.used == 1024 + 5120 + 256
    a.free(y)
    assert a.alloc(4000) == 1024          # first fit reuses the hole
    a.free(x)
    a.free(1024)
    a.free(z)
    assert a.used == 0 and a.largest_free == 1 << 20


def test_no_space_and_fragmentation():
    a = Arena(4096, align=256)
    blocks = [a.alloc(1024) for _ in range(4)]
    with pytest.raises(NoSpace):
        a.alloc(1)
    a.free(blocks[0])
    a.free(blocks[2])
    assert a.largest_free == 1024
    with pytest.raises(NoSpace):
        a.alloc(2048)                      # 2 KiB free, but not contiguous
    a.free(blocks[1])
    assert a.alloc(3072) == 0              # the three neighbours merged


def test_random_workload_keeps_invariants():
    rng = random.Random(3)
    a = Arena(1 << 16, align=64)
    live = {}
    for _ in range(3000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            off = rng.choice(list(live))
            a.free(off)
            del live[off]
        else:
            n = rng.randint(1, 4000)
            try:
                off = a.alloc(n)
            except NoSpace:
                continue
            assert off % 64 == 0 and off + n <= a.size
            for o, m in live.items():          # no overlap with live blocks
                assert off + n <= o or o + m <= off
            live[off] = n
        assert a.used + sum(a._free_len.values()) == a.size
    for off in list(live):
        a.free(off)
    assert a._free_off == [0] and a.largest_free == a.size
