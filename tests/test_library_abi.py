"""Host-side checks of the C ABI library (no GPU needed, no compute calls)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "recsplit.h")).read()
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("rs_build", "rs_query", "rs_serialize", "rs_deserialize", "rs_free",
                 "rs_strerror", "rs_get_stats", "rs_debug_node_values", "rs_calibrate_valu"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2212_09562_amd import recsplit

    lib = recsplit.library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings():
    from paper_2212_09562_amd import recsplit

    for code in range(0, -8, -1):
        s = recsplit.strerror(code)
        assert s and s != "unknown error"
    assert recsplit.strerror(-99) == "unknown error"


def test_invalid_arguments_rejected_before_any_device_call():
    import numpy as np

    from paper_2212_09562_amd import recsplit

    keys = np.zeros((4, 2), dtype=np.uint64)
    for l, b in ((1, 100), (25, 100), (8, 0), (8, 4097)):
        with pytest.raises(recsplit.RecSplitError) as e:
            recsplit.build(keys, l, b)
        assert e.value.code == -1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_keygen_is_duplicate_free_and_deterministic():
    import numpy as np

    from paper_2212_09562_amd import keygen

    a = keygen.fingerprints(100000, 7)
    b = keygen.fingerprints(100000, 7)
    assert np.array_equal(a, b)
    assert len(np.unique(a.view(np.dtype((np.void, 16))))) == len(a)
    jobs = keygen.batched_jobs(8, seed=4)
    assert all(1000 <= j["n"] <= 1_000_000 and j["leaf_size"] in (8, 12, 16)
               and j["bucket_size"] in (100, 500, 2000) for j in jobs)
    reqs = keygen.served_requests(50)
    assert all(reqs[i]["arrival"] < reqs[i + 1]["arrival"] for i in range(49))


def test_torch_keygen_draws_the_same_keys():
    import numpy as np

    from paper_2212_09562_amd import keygen

    for n, seed in ((0, 1), (1, 0), (4097, 3), (100000, (5 << 32) + 7), (33, (1 << 64) - 1)):
        a = keygen.fingerprints(n, seed)
        b = keygen.fingerprints_torch(n, seed, "cpu").numpy().view(np.uint64)
        assert np.array_equal(a, b), (n, seed)


def test_server_config_rejected_before_any_device_call():
    import ctypes

    from paper_2212_09562_amd import recsplit

    lib = recsplit.library()
    h = ctypes.c_void_p()
    for budget, slots in ((1 << 30, 0), (1 << 30, 65), (1000, 2)):
        cfg = recsplit.ServerConfig(budget, slots, 4, 1)
        assert lib.rs_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert lib.rs_server_create(None, ctypes.byref(h)) == -1
    assert recsplit.strerror(recsplit.RS_PENDING) != "unknown error"


def test_schedule_defaults_and_validation():
    from paper_2212_09562_amd import recsplit

    d = recsplit.set_schedule(None)
    assert d["help_after_small"] >= 1 and d["help_after_large"] >= 1
    with pytest.raises(recsplit.RecSplitError) as e:
        recsplit.set_schedule(help_after_large=0)
    assert e.value.code == -1
    with pytest.raises(recsplit.RecSplitError) as e:
        recsplit.set_schedule(chunk_shift_large=64)
    assert e.value.code == -1
    assert recsplit.get_schedule() == d
    assert recsplit.set_schedule(chunk_shift_large=7)["chunk_shift_large"] == 7
    assert recsplit.set_schedule(None) == d


def test_query_output_tensor_checked_before_the_library_is_called():
    """A caller-supplied out tensor that is short, of the wrong element size,
    non-contiguous or on another device would let the query kernel write out
    of bounds: the binding refuses it first."""
    import torch

    from paper_2212_09562_amd import recsplit

    cpu = torch.device("cpu")
    recsplit._check_out(torch.empty(10, dtype=torch.int64), 10, cpu)
    bad = [(torch.empty(9, dtype=torch.int64), ValueError),
           (torch.empty(10, dtype=torch.int32), ValueError),
           (torch.empty(10, dtype=torch.float64), ValueError),
           (torch.empty(20, dtype=torch.int64)[::2], ValueError),
           (torch.empty(10, dtype=torch.int64, device="meta"), ValueError),
           ([0] * 10, TypeError)]
    for out, exc in bad:
        with pytest.raises(exc):
            recsplit._check_out(out, 10, cpu)


def test_noalloc_refuses_oversized_builds_before_any_device_call():
    import ctypes

    import numpy as np

    from paper_2212_09562_amd import recsplit

    lib = recsplit.library()
    keys = np.zeros((4, 2), dtype=np.uint64)
    words = np.zeros(64, dtype=np.uint64)
    nw = ctypes.c_uint64(123)
    # one key above the maximum (the keys are not read: the size is refused first)
    rc = lib.rs_build_noalloc(keys.ctypes.data, recsplit.RS_NOALLOC_MAX_KEYS + 1, 8, 100,
                              recsplit.RS_FLAG_ROTATION, words.ctypes.data, len(words),
                              ctypes.byref(nw))
    assert rc == -1 and nw.value == 0
    rc = lib.rs_build_noalloc(keys.ctypes.data, 4, 8, 100, recsplit.RS_FLAG_KEEP_VALUES,
                              words.ctypes.data, len(words), ctypes.byref(nw))
    assert rc == -1
    rc = lib.rs_build_noalloc(keys.ctypes.data, 4, 8, 100, 0, None, 0, ctypes.byref(nw))
    assert rc == -1
    hdr = open(os.path.join(ROOT, "include", "recsplit.h")).read()
    assert "#define RS_NOALLOC_MAX_KEYS (1u << 19)" in hdr
    assert recsplit.RS_NOALLOC_MAX_KEYS == 1 << 19
