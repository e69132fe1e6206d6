"""GPU: the paper's most space-efficient configuration at its own size
(tab:showcaseOverall: l = 24, b = 2000, rotation fitting, 5 million random
128-bit keys).

The build takes about ten minutes on one MI355X, so the test runs only when
RS_SHOWCASE=1 is set.  Three of its buckets were rebuilt by the oracle (an
hour or more each; tests/golden/make_l24_showcase_buckets.py stores their
node values and Golomb-Rice records); the GPU build must give the same
values and the same record bits for them, its bucket sizes must match a
count of the keys, and the ranks of all keys must form a permutation.
"""
import os
import time

import numpy as np
import pytest

import oracle
from paper_2212_09562_amd import keygen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "l24_b2000_n5e6_buckets.txt")


def _golden():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    out = {}
    for i in range(0, len(rows), 3):
        j, size, bits = (int(x) for x in rows[i])
        words = np.array([int(w, 16) for w in rows[i + 1]], dtype=np.uint64)
        vals = np.array([int(v) for v in rows[i + 2]], dtype=np.uint64)
        out[j] = (size, bits, words, vals)
    return out


@pytest.mark.skipif(not os.environ.get("RS_SHOWCASE"),
                    reason="a ten-minute build; RS_SHOWCASE=1 runs it")
def test_l24_b2000_five_million_keys():
    import torch

    from paper_2212_09562_amd import recsplit

    n, l, b = 5_000_000, 24, 2000
    want = _golden()
    keys = keygen.fingerprints(n, 55)
    dev = torch.from_numpy(keys.view(np.int64)).cuda()
    torch.cuda.synchronize()
    print(f"[case] l={l} b={b} n={n}, buckets {sorted(want)} against the oracle", flush=True)
    recsplit.build(dev[:2000], l, b, True).free()  # the leaf size's tables
    # the search's own progress (finished nodes) on stderr every 30 s; run
    # with -s to see it
    os.environ.setdefault("RS_PROGRESS", "30")
    t0 = time.perf_counter()
    f = recsplit.build(dev, l, b, True, keep_values=True)
    secs = time.perf_counter() - t0
    data = f.serialize()
    st = f.stats()
    print(f"[showcase] {secs:.1f} s, {secs * 1e6 / n:.1f} us per key, "
          f"{len(data) * 8 / n:.4f} bits per key, search {st['ms_search'] / 1e3:.1f} s", flush=True)
    nb = oracle.num_buckets(n, b)
    for j, (size, bits, words, vals) in sorted(want.items()):
        assert np.array_equal(f.node_values(j), vals), j
        gw, gb = oracle.bucket_record(data, j)
        assert gb == bits and np.array_equal(gw, words), j
    w0 = keys[:, 0]
    hi, lo = w0 >> np.uint64(32), w0 & np.uint64(0xFFFFFFFF)
    nbu = np.uint64(nb)
    bucket = ((hi * nbu + ((lo * nbu) >> np.uint64(32))) >> np.uint64(32)).astype(np.int64)
    sizes = np.bincount(bucket, minlength=nb)
    assert all(sizes[j] == want[j][0] for j in want)
    r = f.query(dev)
    assert torch.equal(torch.sort(r)[0], torch.arange(n, device=r.device, dtype=r.dtype))
    assert 1.4427 <= len(data) * 8 / n < 1.56
