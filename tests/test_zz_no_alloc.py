"""rs_build_noalloc, the entry point for callers that cannot allocate device
memory, against rs_build through the C ABI: the serialised words must be
identical, call after call on the library's one fixed device array, the
later calls smaller than the earlier ones (stale contents must not leak into
a build), with device and host keys; the smallest also against the oracle.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2212_09562_amd import keygen

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


def test_noalloc_equals_rs_build_call_after_call():
    from paper_2212_09562_amd import recsplit as rs

    cases = [  # (n, l, b, rotation, device keys, seed); each call smaller than the one before
        (rs.RS_NOALLOC_MAX_KEYS, 8, 100, True, True, 71),
        (30000, 16, 2000, True, False, 72),
        (5000, 12, 7, False, True, 73),
    ]
    for n, l, b, rot, dev, seed in cases:
        _case(f"noalloc n={n} l={l} b={b} rot={rot} device_keys={dev}")
        keys = keygen.fingerprints(n, seed)
        arg = torch.from_numpy(keys.view(np.int64)).cuda() if dev else keys
        got = rs.build_noalloc(arg, l, b, rot)
        want = rs.build(arg, l, b, rot).serialize()
        assert got == want, f"n={n} l={l} b={b}: {len(got)} vs {len(want)} bytes"
        if n <= 5000:
            assert got == oracle.build(keys, l, b, rot)[0]
        torch.cuda.synchronize()


def test_noalloc_short_buffer_reports_its_size():
    from paper_2212_09562_amd import recsplit as rs

    keys = keygen.fingerprints(20000, 74)
    _case("noalloc short buffer n=20000 l=8 b=100")
    want = rs.build(keys, 8, 100, True).serialize()
    lib = rs.library()
    small = np.zeros(16, dtype=np.uint64)
    nw = ctypes.c_uint64()
    rc = lib.rs_build_noalloc(keys.ctypes.data, len(keys), 8, 100, rs.RS_FLAG_ROTATION,
                              small.ctypes.data, len(small), ctypes.byref(nw))
    assert rc == -1 and nw.value * 8 == len(want)
    assert not small.any()  # nothing written
    full = np.zeros(nw.value, dtype=np.uint64)
    rc = lib.rs_build_noalloc(keys.ctypes.data, len(keys), 8, 100, rs.RS_FLAG_ROTATION,
                              full.ctypes.data, len(full), ctypes.byref(nw))
    assert rc == 0 and full.tobytes() == want


def test_noalloc_duplicate_then_exact():
    from paper_2212_09562_amd import recsplit as rs

    keys = keygen.fingerprints(10000, 75)
    dup = keys.copy()
    dup[777] = dup[4242]
    _case("noalloc duplicate set, then the clean set")
    with pytest.raises(rs.RecSplitError) as e:
        rs.build_noalloc(dup, 8, 100, True)
    assert e.value.code == -2
    assert rs.build_noalloc(keys, 8, 100, True) == rs.build(keys, 8, 100, True).serialize()
