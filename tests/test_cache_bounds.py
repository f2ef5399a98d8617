"""The per-failure-pattern caches are bounded (no GPU needed): cycling
through 10^4 decode node sets of the (16,30,32) code keeps host memory flat
once the caches are full, and evicted patterns are rebuilt identically when
they come back."""
import os

import numpy as np
import pytest

from paper_1412_3022_amd import pm, synth


def _rss_bytes():
    with open("/proc/self/statm") as f:
        return int(f.read().split()[1]) * os.sysconf("SC_PAGE_SIZE")


@pytest.mark.slow
def test_ten_thousand_decode_patterns_keep_host_memory_bounded():
    c = pm.Code(k=16, d=30, n=32)
    c.set_cache_limit(32)
    # a fixed table variant: the init phase builds matrices and table
    # programs only (no bit-sliced kernel is generated or compiled)
    c.set_variant(pm.OP_DECODE, 16, 2)
    rng = synth.Stream(0xCAC4E)
    sets = [rng.subset(c.n, c.k) for _ in range(10_000)]
    first = c.decode_matrix(sets[0])
    rss = []
    for i, K in enumerate(sets):
        # the decode's init phase: its matrix, program and (no GPU here)
        # nothing on a device
        st, _ = pm.pm_prepare(c.h, pm.OP_DECODE, 0, K, 0)
        assert st == pm.PM_OK
        if i in (500, 10_000 - 1):
            rss.append(_rss_bytes())
    # one cached pattern of this code is about 1.3 MB (a 240 x 240 decode
    # matrix and its packed tables); unbounded caches would hold ~13 GB here
    assert rss[1] - rss[0] < 128 << 20, rss
    # an evicted pattern comes back with the same matrix
    D, kept = c.decode_matrix(sets[0])
    assert np.array_equal(D, first[0]) and np.array_equal(kept, first[1])


def test_cache_limit_rejects_zero():
    c = pm.Code(k=4, d=6, n=8)
    with pytest.raises(pm.PMError):
        c.set_cache_limit(0)
