"""Pins of the oracle's random streams.

The paper's multiply-with-carry generator (Sec. II.C.1, Eqs. 9-10) is replaced
by a counter-based Philox4x32-10 stream per particle.  Pins: the published
Philox known-answer vectors (Salmon et al., SC'11, Random123 distribution),
numpy's independent Philox4x64-10 bit generator for the shared round and
key-schedule structure, and a small statistical battery.
"""
import json
import os

import numpy as np
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_kat.json")


def test_philox4x32_known_answers(oracle):
    with open(GOLDEN) as f:
        kat = json.load(f)
    for case in kat["vectors"]:
        ctr = [int(x, 16) for x in case["ctr"]]
        key = [int(x, 16) for x in case["key"]]
        want = [int(x, 16) for x in case["out"]]
        assert list(oracle.philox4x32(ctr, key)) == want


def test_philox4x64_matches_numpy(oracle):
    # numpy.random.Philox advances its 256-bit counter before each block, so
    # its k-th block is Philox4x64-10(counter = k + 1).
    for key in ([0, 0], [0x0123456789ABCDEF, 0xFEDCBA9876543210], [7, 2 ** 63 + 5]):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=0)
        raw = bg.random_raw(4 * 6)
        for blk in range(6):
            got = oracle.philox4x64([blk + 1, 0, 0, 0], key)
            assert list(got) == list(raw[4 * blk:4 * blk + 4])
    # counter carry into the second word
    bg = np.random.Philox(key=np.array([3, 4], dtype=np.uint64),
                          counter=np.array([2 ** 64 - 1, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(4)
    assert list(oracle.philox4x64([0, 1, 0, 0], [3, 4])) == list(raw)


def test_stream_layout(oracle):
    # word n of (seed, beam, hist, path) is word n & 3 of
    # Philox4x32(ctr = (n >> 2, path lo, path hi, hist), key = (seed lo, seed hi ^ beam))
    seed, beam, hist, path = 0x1122334455667788, 9, 12345, 0xDEADBEEF00C0FFEE
    w, u = oracle.stream_words(seed, beam, hist, path, 5, 11)
    key = [seed & 0xFFFFFFFF, (seed >> 32) ^ beam]
    for i in range(11):
        n = 5 + i
        blk = oracle.philox4x32([n >> 2, path & 0xFFFFFFFF, path >> 32, hist], key)
        assert w[i] == blk[n & 3]
        # uniform: odd multiple of 2^-24 from the top 24 bits
        assert u[i] == ((int(w[i]) >> 8) | 1) * 2.0 ** -24
        assert np.float32(u[i]) == u[i]
        assert 0.0 < u[i] < 1.0


def test_child_paths_distinct(oracle):
    seen = set()
    for n in range(2000):
        for c in range(2):
            seen.add(oracle.child_path(0, n, c))
    assert len(seen) == 4000
    assert 0 not in seen
    # depends on the parent path too
    assert oracle.child_path(1, 0, 0) != oracle.child_path(0, 0, 0)


def test_uniform_battery(oracle):
    # chi^2 on 256 bins over many histories' streams, serial pairs on a
    # 16 x 16 grid, lag-1 correlation, and independence of adjacent histories
    u = np.concatenate([oracle.stream_words(1, 0, h, 0, 0, 64)[1] for h in range(4000)])
    counts = np.bincount((u * 256).astype(int), minlength=256)
    assert stats.chisquare(counts).pvalue > 1e-4
    pairs = (u[:-1:2] * 16).astype(int) * 16 + (u[1::2] * 16).astype(int)
    assert stats.chisquare(np.bincount(pairs, minlength=256)).pvalue > 1e-4
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 4.0 / np.sqrt(u.size)
    a = np.array([oracle.stream_words(1, 0, h, 0, 0, 1)[1][0] for h in range(20000)])
    b = np.array([oracle.stream_words(1, 0, h + 1, 0, 0, 1)[1][0] for h in range(20000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 4.0 / np.sqrt(a.size)
    # child stream vs parent stream
    c = np.array([oracle.stream_words(1, 0, h, oracle.child_path(0, 4, 0), 0, 1)[1][0] for h in range(20000)])
    assert abs(np.corrcoef(a, c)[0, 1]) < 4.0 / np.sqrt(a.size)
    assert stats.kstest(c, "uniform").pvalue > 1e-4
