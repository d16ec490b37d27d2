"""Pins for the adaptive ring multiplication of the oracle (ring_oracle.c):
both paths against numpy's convolution of the bit vectors, reduced mod 2 and
folded mod X^n - 1."""
import numpy as np
import pytest

import oracle
from paper_2512_12904_amd import synth


def bits(words, n):
    b = np.unpackbits(np.ascontiguousarray(words, np.uint64).view(np.uint8), bitorder="little")
    return b[:n].astype(np.int64)


def words(bitvec):
    n = len(bitvec)
    U = (n + 63) // 64
    b = np.zeros(64 * U, np.uint8)
    b[:n] = bitvec
    return np.packbits(b, bitorder="little").view(np.uint64)


def ring_ref(n, a, b):
    full = np.convolve(bits(a, n), bits(b, n)) % 2
    out = full[:n].copy()
    out[:len(full) - n] ^= full[n:]
    return words(out)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 200])
def test_dense_and_sparse_small(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        a = words(rng.integers(0, 2, n).astype(np.uint8))
        b = words(rng.integers(0, 2, n).astype(np.uint8))
        ref = ring_ref(n, a, b)
        assert (oracle.ring_mul_dense(n, a, b) == ref).all()
        assert (oracle.ring_mul_sparse(n, a, b) == ref).all()


def test_levels():
    # smallest depth with leaf blocks of at most 8 words
    assert [oracle.ring_levels(u) for u in (1, 8, 9, 16, 17, 277, 561, 901)] == [0, 0, 1, 1, 2, 6, 7, 7]


@pytest.mark.parametrize("n", [17669, 35851, 57637])
def test_hqc_sizes_and_threshold(n):
    U = (n + 63) // 64
    a = synth.words(n, (U,))
    b = synth.words(n + 1, (U,))
    a[-1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(n % 64)  # bits >= n are ignored
    ref = ring_ref(n, a, b)
    d = oracle.ring_mul_dense(n, a, b)
    assert (d == ref).all()
    w = int(bits(a, n).sum())
    out0, p0 = oracle.ring_mul(n, a, b, w)        # weight == threshold: sparse
    out1, p1 = oracle.ring_mul(n, a, b, w - 1)    # weight > threshold: dense
    assert (p0, p1) == (0, 1) and (out0 == ref).all() and (out1 == ref).all()
    # a sparse operand of HQC weight
    s = np.zeros(n, np.uint8)
    s[synth.fixed_weight(n + 2, n, 75)] = 1
    a2 = words(s)
    assert (oracle.ring_mul_dense(n, a2, b) == ring_ref(n, a2, b)).all()
