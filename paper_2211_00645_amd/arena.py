"""First-fit arena over one device allocation, for the serving loop.

The serving loop holds many multi-gigabyte outputs of different sizes at
once on several streams.  Allocating each through the framework's caching
allocator fragments its per-stream pools until an allocation fails and the
allocator frees and synchronises everything, which stalls the loop for
seconds.  The executor instead reserves one buffer of the memory budget up
front and places every batch's outputs in it with this allocator:
offsets only, no device calls, so it is tested on the CPU.

Blocks are aligned to ``align`` bytes; freeing coalesces with both
neighbours, so an empty arena is always one free block.
"""
from __future__ import annotations

import bisect
from typing import Dict, List, Optional


class NoSpace(Exception):
    """No free block is large enough (fragmentation); retry after a free."""


class Arena:
    def __init__(self, nbytes: int, align: int = 256):
        if nbytes <= 0 or align <= 0 or align & (align - 1):
            raise ValueError("arena size must be positive and alignment a power of two")
        self.size = int(nbytes) // align * align
        self.align = align
        self._free_off: List[int] = [0]          # sorted offsets of free blocks
        self._free_len: Dict[int, int] = {0: self.size}
        self._used: Dict[int, int] = {}

    def round(self, n: int) -> int:
        a = self.align
        return (int(n) + a - 1) // a * a

    @property
    def used(self) -> int:
        return sum(self._used.values())

    @property
    def largest_free(self) -> int:
        return max(self._free_len.values(), default=0)

    def alloc(self, n: int) -> int:
        """Offset of a new block of at least ``n`` bytes (first fit)."""
        need = self.round(max(1, n))
        for off in self._free_off:
            ln = self._free_len[off]
            if ln >= need:
                i = bisect.bisect_left(self._free_off, off)
                del self._free_off[i]
                del self._free_len[off]
                if ln > need:
                    rest = off + need
                    bisect.insort(self._free_off, rest)
                    self._free_len[rest] = ln - need
                self._used[off] = need
                return off
        raise NoSpace(f"no free block of {need} bytes (largest {self.largest_free})")

    def free(self, off: int) -> None:
        ln = self._used.pop(off)
        i = bisect.bisect_left(self._free_off, off)
        # merge with the following free block
        if i < len(self._free_off) and self._free_off[i] == off + ln:
            nxt = self._free_off.pop(i)
            ln += self._free_len.pop(nxt)
        # merge with the preceding free block
        if i > 0:
            prv = self._free_off[i - 1]
            if prv + self._free_len[prv] == off:
                self._free_len[prv] += ln
                return
        self._free_off.insert(i, off)
        self._free_len[off] = ln
