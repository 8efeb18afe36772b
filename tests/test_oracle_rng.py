"""Pins for the oracle's random streams (readings R1, R2, R8).

Philox4x64-10 is pinned to the published known-answer vectors and to numpy's
independent implementation; Lemire's bounded draw is pinned to its closed
form for powers of two and to exact uniformity where skipping the rejection
step would be visibly biased.
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
M64 = 2**64


def numpy_block(ctr, key):
    """Philox4x64-10 block `ctr` via numpy (which generates block c+1 from state c)."""
    c = [int(x) % M64 for x in ctr]
    # subtract one from the 256-bit counter, little-endian words
    for i in range(4):
        if c[i] != 0:
            c[i] -= 1
            break
        c[i] = M64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4)


def numpy_stream(seed, c1, c2, c3, nwords):
    """Words of the stream key=(seed,0), counter=(b, c1, c2, c3), b = 0, 1, ..."""
    out = []
    b = 0
    while len(out) < nwords:
        out.extend(int(x) for x in numpy_block([b, c1, c2, c3], [seed, 0]))
        b += 1
    return out[:nwords]


def test_philox_known_answers():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        got = oracle.philox(ctr, key)
        assert [int(x) for x in got] == want


@pytest.mark.parametrize("ctr,key", [([0, 0, 0, 0], [0, 0]), ([7, 123, 4, 1], [99, 0]),
                                     ([2**64 - 1, 5, 6, 0], [1, 2]), ([0, 2**40 + 3, 17, 3], [2**63, 0])])
def test_philox_matches_numpy(ctr, key):
    assert [int(x) for x in oracle.philox(ctr, key)] == [int(x) for x in numpy_block(ctr, key)]


@pytest.mark.parametrize("k", [1, 5, 17, 63])
def test_bounded_power_of_two_is_top_bits(k):
    # W = 2^k never rejects ((2^64 - W) mod W = 0) and returns the top k bits.
    seed, c1, c2, c3 = 11, 42, 3, 0
    words = numpy_stream(seed, c1, c2, c3, 64)
    got = oracle.bounded_many(seed, c1, c2, c3, 2**k, 64)
    assert [int(x) for x in got] == [w >> (64 - k) for w in words]


def test_bounded_w1_is_zero():
    assert not oracle.bounded_many(5, 1, 2, 3, 1, 100).any()


def test_bounded_uniform_where_rejection_matters():
    # W = 3 * 2^62: a word x maps to floor(3x/4).  Without rejection the
    # residues mod 3 would come out with probabilities (1/2, 1/4, 1/4);
    # with Lemire's rejection (x = 0 mod 4 is rejected) they are uniform.
    W = 3 * 2**62
    n = 60000
    r = oracle.bounded_many(9, 1, 0, 0, W, n)
    assert (r < W).all()
    counts = np.bincount((r % np.uint64(3)).astype(np.int64), minlength=3)
    exp = n / 3
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 20.0, counts          # 2 dof; 1/2-1/4-1/4 would give chi2 ~ 7500


@pytest.mark.parametrize("W", [2, 3, 7, 10, 1000])
def test_bounded_chi2(W):
    n = 40000
    r = oracle.bounded_many(3, 77, 1, 0, W, n).astype(np.int64)
    assert r.max() < W
    counts = np.bincount(r, minlength=W)
    exp = n / W
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # mean W-1, sd sqrt(2(W-1)); 6 sd slack
    assert chi2 < (W - 1) + 6 * np.sqrt(2 * (W - 1)) + 10


def test_rademacher_bit_layout():
    # sigma_js = +1 iff bit (j mod 64) of word ((j mod 256) div 64) of block
    # (j div 256, s, instance, 1) is set (reading R8), checked on numpy words.
    seed, inst = 1234, 2
    for s in [0, 1, 999]:
        for jb in [0, 1]:
            words = numpy_block([jb, s, inst, 1], [seed, 0])
            for j in range(jb * 256, jb * 256 + 256, 7):
                w = int(words[(j % 256) // 64])
                want = 1 if (w >> (j % 64)) & 1 else -1
                assert oracle.rademacher(seed, inst, s, j) == want


def test_rademacher_balanced():
    vals = np.array([oracle.rademacher(5, 0, s, j) for s in range(200) for j in range(100)])
    assert abs(vals.mean()) < 5 / np.sqrt(len(vals))
