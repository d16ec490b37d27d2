"""Pins of the oracle's ring product in GF(2)[X]/(X^n - 1) (Eq. (1)).

The oracle forms the product as a XOR of word-shifted copies (Eq. (1)); the
pins compare it with the schoolbook definition of the ring product --
convolution of the coefficient vectors, folded mod X^n - 1, taken mod 2 --
and with the ring identities.
"""
import numpy as np
import pytest
from scipy.signal import fftconvolve


def bits_of(words, n):
    b = np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little")
    return b[:n].astype(np.int64)


def words_of(bits):
    n = len(bits)
    nw = (n + 63) // 64
    padded = np.zeros(nw * 64, np.uint8)
    padded[:n] = bits
    return np.packbits(padded, bitorder="little").view(np.uint64).copy()


def schoolbook(n, a_bits, supp):
    """(sum_i a_i X^i) * (sum_k X^(supp_k mod n)) mod (X^n - 1), coefficients mod 2."""
    b_bits = np.zeros(n, np.int64)
    for s in supp:
        b_bits[int(s) % n] += 1  # repeated indices add (and cancel mod 2)
    if n > 4096:
        full = np.rint(fftconvolve(a_bits.astype(np.float64), b_bits.astype(np.float64))).astype(np.int64)
    else:
        full = np.convolve(a_bits, b_bits)
    folded = full[:n].copy()
    folded[: len(full) - n] += full[n:]
    return folded % 2


@pytest.mark.parametrize("n", [7, 31, 63, 64, 65, 127, 128, 129, 200, 1000])
def test_matches_schoolbook_small(orc, n):
    rng = np.random.default_rng(n)
    for trial in range(20):
        a = rng.integers(0, 2, n)
        w = int(rng.integers(0, 9))
        supp = rng.integers(0, 3 * n, w).astype(np.uint32)  # also indices >= n and repeats
        out = orc.mul_sparse(n, words_of(a), supp)
        assert (bits_of(out, n) == schoolbook(n, a, supp)).all()
        # no bits at or above n
        assert bits_of(out, len(out) * 64)[n:].sum() == 0


def test_exhaustive_weight_le_2_tiny(orc):
    for n in (5, 7):
        for av in range(1 << n):
            a = np.array([(av >> i) & 1 for i in range(n)])
            for s1 in range(n):
                for s2 in (None, (s1 * 5 + 3) % n):
                    supp = [s1] if s2 is None else [s1, s2]
                    out = orc.mul_sparse(n, words_of(a), np.array(supp, np.uint32))
                    assert (bits_of(out, n) == schoolbook(n, a, supp)).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_matches_schoolbook_full_size(orc, pid):
    p = orc.param(pid)
    n = p["n"]
    rng = np.random.default_rng(pid)
    a = rng.integers(0, 2, n)
    supp = rng.choice(n, p["w"], replace=False).astype(np.uint32)
    out = orc.mul_sparse(n, words_of(a), supp)
    assert (bits_of(out, n) == schoolbook(n, a, supp)).all()


def test_monomials(orc):
    n = 17669
    rng = np.random.default_rng(5)
    for _ in range(50):
        i, j = (int(v) for v in rng.integers(0, n, 2))
        a = np.zeros(n, np.int64)
        a[i] = 1
        out = bits_of(orc.mul_sparse(n, words_of(a), np.array([j], np.uint32)), n)
        assert out.sum() == 1 and out[(i + j) % n] == 1


def test_commutative_and_linear(orc):
    n = 35851
    rng = np.random.default_rng(9)
    y1 = rng.choice(n, 40, replace=False)
    y2 = rng.choice(n, 37, replace=False)
    d1 = np.zeros(n, np.int64)
    d1[y1] = 1
    d2 = np.zeros(n, np.int64)
    d2[y2] = 1
    p12 = orc.mul_sparse(n, words_of(d1), y2.astype(np.uint32))
    p21 = orc.mul_sparse(n, words_of(d2), y1.astype(np.uint32))
    assert (p12 == p21).all()
    a1 = rng.integers(0, 2, n)
    a2 = rng.integers(0, 2, n)
    lhs = orc.mul_sparse(n, words_of(a1 ^ a2), y1.astype(np.uint32))
    rhs = orc.mul_sparse(n, words_of(a1), y1.astype(np.uint32)) ^ orc.mul_sparse(
        n, words_of(a2), y1.astype(np.uint32))
    assert (lhs == rhs).all()


def test_bits_above_n_ignored(orc):
    n = 57637
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2, n)
    w = words_of(a)
    dirty = w.copy()
    dirty[-1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(n % 64)
    supp = rng.choice(n, 131, replace=False).astype(np.uint32)
    assert (orc.mul_sparse(n, w, supp) == orc.mul_sparse(n, dirty, supp)).all()
