"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
harness.  Holds no coding arithmetic: only a public pseudo-random generator
(splitmix64, Vigna 2014) and the workload recipes built on it.

splitmix64: state += 0x9E3779B97F4A7C15; z = state;
z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) * 0x94D049BB133111EB;
out = z ^ (z >> 31).  Output words are emitted as 8 little-endian bytes.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
CONFIG_SEED = 0x5EED0000


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def words(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Words start .. start+count-1 of the splitmix64 stream seeded with seed."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        return _mix(np.uint64(seed & (2**64 - 1)) + i * GAMMA)


def random_bytes(seed: int, nbytes: int) -> np.ndarray:
    w = words(seed, (nbytes + 7) // 8)
    return w.view(np.uint8)[:nbytes].copy()


class Stream:
    """Sequential splitmix64 draws for small decisions (sizes, subsets)."""

    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def next(self) -> int:
        v = int(words(self.seed, 1, self.pos)[0])
        self.pos += 1
        return v

    def uniform(self) -> float:
        return (self.next() >> 11) / float(1 << 53)

    def below(self, m: int) -> int:
        return self.next() % m

    def log_uniform(self, a: int, b: int) -> int:
        return int(math.floor(a * (b / a) ** self.uniform()))

    def exponential(self, rate: float) -> float:
        return -math.log(1.0 - self.uniform()) / rate

    def subset(self, n: int, k: int, exclude=()) -> list:
        """k distinct items of range(n) minus exclude, by a partial Fisher-Yates
        shuffle; returned in ascending order."""
        pool = [i for i in range(n) if i not in set(exclude)]
        for i in range(k):
            j = i + self.below(len(pool) - i)
            pool[i], pool[j] = pool[j], pool[i]
        return sorted(pool[:k])


def split_object(S: int, B: int, seed: int, align: int = 64):
    """An object of S uniform random bytes cut into B sub-blocks of
    s = roundup(ceil(S / B), align) bytes, zero padded at the end.
    Returns (X as a B x s uint8 array, s)."""
    s = -(-S // B)
    s = -(-s // align) * align
    buf = np.zeros(B * s, np.uint8)
    buf[:S] = random_bytes(seed, S)
    return buf.reshape(B, s), s


def block_bytes_for(S: int, B: int, align: int = 64) -> int:
    s = -(-S // B)
    return -(-s // align) * align


def random_bytes_torch(seed: int, nbytes: int, device, chunk_words: int = 1 << 26):
    """The same splitmix64 byte stream as random_bytes(), generated with torch
    integer ops on `device` (int64 arithmetic wraps like uint64; logical right
    shifts are arithmetic shifts masked to the low bits).  Returns a uint8
    tensor of nbytes."""
    import torch
    nwords = (nbytes + 7) // 8
    out = torch.empty(nwords * 8, dtype=torch.uint8, device=device)
    words = out.view(torch.int64)

    def s64(v):
        v &= (1 << 64) - 1
        return v - (1 << 64) if v >= 1 << 63 else v

    gamma, m1, m2 = s64(0x9E3779B97F4A7C15), s64(0xBF58476D1CE4E5B9), s64(0x94D049BB133111EB)

    def shr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    for a in range(0, nwords, chunk_words):
        b = min(nwords, a + chunk_words)
        z = torch.arange(a + 1, b + 1, dtype=torch.int64, device=device) * gamma + s64(seed)
        z = (z ^ shr(z, 30)) * m1
        z = (z ^ shr(z, 27)) * m2
        words[a:b] = z ^ shr(z, 31)
    return out[:nbytes]
