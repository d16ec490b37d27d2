"""Pins of the oracle's duplicated RM(1,7) code and its Hadamard decoder.

- The duplicated code's minimum distance must equal the d2 printed in
  Table I ([384, 8, 192] and [640, 8, 320]).
- The 128-point transform must equal the brute-force correlation with the
  Walsh functions, satisfy Parseval, and be its own inverse up to 128.
- The decoder must return the nearest of the 256 codewords in Hamming
  distance (smallest low-7-bit index on a tie), computed by brute force.
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def bits(words, nbits):
    return np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little")[:nbits]


def pack(b):
    return np.packbits(np.asarray(b, np.uint8), bitorder="little").view(np.uint64).copy()


def walsh_matrix(size):
    idx = np.arange(size)
    pc = np.array([[bin(u & i).count("1") & 1 for i in idx] for u in idx])
    return 1 - 2 * pc


@pytest.fixture(scope="module")
def codebooks(orc):
    return {mult: np.array([bits(orc.rm_encode(mult, b), 128 * mult) for b in range(256)])
            for mult in (3, 5)}


def test_fht_brute_force(orc):
    Hm = walsh_matrix(128)
    rng = np.random.default_rng(1)
    for _ in range(50):
        x = rng.integers(-700, 700, 128)
        assert (orc.fht128(x) == Hm @ x).all()


def test_fht_parseval_and_involution(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        x = rng.integers(-5, 6, 128)
        X = orc.fht128(x)
        assert int((X.astype(np.int64) ** 2).sum()) == 128 * int((x ** 2).sum())
        assert (orc.fht128(X) == 128 * x).all()
    for i in range(128):  # unit vectors give the Walsh rows
        e = np.zeros(128, np.int64)
        e[i] = 1
        assert (orc.fht128(e) == walsh_matrix(128)[:, i]).all()


def test_minimum_distance_matches_table_i(orc, codebooks):
    table = json.load(open(os.path.join(GOLD, "table1.json")))["rows"]
    for row in table:
        n2, dim, d2 = row["rm"]
        mult = n2 // 128
        cb = codebooks[mult].astype(np.int64)
        assert cb.shape == (2 ** dim, n2)
        dist = (cb[:, None, :] != cb[None, :, :]).sum(-1)
        np.fill_diagonal(dist, n2 + 1)
        assert dist.min() == d2


def test_codeword_structure(codebooks):
    for mult, cb in codebooks.items():
        w = cb.sum(1)
        assert w[0] == 0 and w[0x80] == 128 * mult
        assert set(w[np.r_[1:0x80, 0x81:256]].tolist()) == {64 * mult}
        # copies are identical
        r = cb.reshape(256, mult, 128)
        assert (r == r[:, :1, :]).all()
        # linear over GF(2): rm(a ^ b) = rm(a) ^ rm(b)
        for a, b in ((3, 5), (0x81, 0x7F), (0x40, 0xC0)):
            assert (cb[a ^ b] == cb[a] ^ cb[b]).all()


def nearest(cb, rbits):
    d = (cb != rbits[None, :]).sum(1)
    best = d.min()
    cands = np.flatnonzero(d == best)
    return min(cands, key=lambda b: (b & 0x7F))


@pytest.mark.parametrize("mult", [3, 5])
def test_decode_is_nearest_codeword(orc, codebooks, mult):
    cb = codebooks[mult]
    n2 = 128 * mult
    rng = np.random.default_rng(mult)
    for trial in range(600):
        b = int(rng.integers(0, 256))
        flips = int(rng.integers(0, n2 + 1)) if trial % 2 else int(rng.integers(0, n2 // 2 + 20))
        r = cb[b].copy()
        r[rng.choice(n2, flips, replace=False)] ^= 1
        got, T = orc.rm_decode(mult, pack(r))
        assert got == nearest(cb, r)
        # T is the correlation with the affine functions
        t = mult - 2 * r.reshape(mult, 128).astype(np.int64).sum(0)
        assert (T == walsh_matrix(128) @ t).all()


@pytest.mark.parametrize("mult", [3, 5])
def test_exact_recovery_within_radius(orc, codebooks, mult):
    cb = codebooks[mult]
    n2 = 128 * mult
    rho = (64 * mult - 1) // 2  # 95 / 159
    rng = np.random.default_rng(10 + mult)
    for trial in range(300):
        b = int(rng.integers(0, 256))
        r = cb[b].copy()
        r[rng.choice(n2, int(rng.integers(0, rho + 1)), replace=False)] ^= 1
        assert orc.rm_decode(mult, pack(r))[0] == b


def test_tie_break_smallest_index(orc, codebooks):
    # a block exactly between rm(0x01) and rm(0x02): equal distance to both
    cb = codebooks[3]
    a, b = cb[0x01].copy(), cb[0x02].copy()
    diff = np.flatnonzero(a != b)
    r = a.copy()
    r[diff[: len(diff) // 2]] = b[diff[: len(diff) // 2]]
    got, T = orc.rm_decode(3, pack(r))
    assert got == nearest(cb, r)
    assert (np.abs(T) == np.abs(T).max()).sum() >= 2
