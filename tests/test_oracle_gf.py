"""Pins of the oracle's GF(2^8) arithmetic (field polynomial x^8+x^4+x^3+x^2+1).

Multiplication in GF(2^8) is fixed by: a*1 = a, a*x = the shift of a reduced
by the field polynomial, distributivity, associativity and commutativity.
Checking all five over every element pins the whole table (any b is a sum
of powers of x, and a*x^i = (a*x)*x^(i-1)).
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def table(orc):
    t = np.zeros((256, 256), np.uint8)
    for a in range(256):
        for b in range(256):
            t[a, b] = orc.gf_mul(a, b)
    return t


def test_identity_and_zero(table):
    a = np.arange(256)
    assert (table[a, 1] == a).all()
    assert (table[a, 0] == 0).all()


def test_multiply_by_x_uses_field_polynomial(table):
    # x^8 = x^4 + x^3 + x^2 + 1, i.e. 0x80 * 0x02 = 0x1D
    assert table[0x80, 0x02] == 0x1D
    for a in range(256):
        shifted = (a << 1) & 0xFF
        carry = a >> 7
        assert table[a, 2] == (shifted ^ (0x1D if carry else 0))


def test_commutative(table):
    assert (table == table.T).all()


def test_distributive_all_triples(table):
    a = np.arange(256)[:, None, None]
    b = np.arange(256)[None, :, None]
    c = np.arange(256)[None, None, :]
    assert (table[a, b ^ c] == (table[a, b] ^ table[a, c])).all()


def test_associative_all_triples(table):
    a = np.arange(256)[:, None, None]
    b = np.arange(256)[None, :, None]
    c = np.arange(256)[None, None, :]
    assert (table[table[a, b], c] == table[a, table[b, c]]).all()


def test_inverse_and_no_zero_divisors(orc, table):
    assert orc.gf_inv(0) == 0
    for a in range(1, 256):
        assert table[a, orc.gf_inv(a)] == 1
    assert (table[1:, 1:] != 0).all()


def test_alpha_is_primitive(orc):
    e, lg = orc.gf_tables()
    assert sorted(e.tolist()) == list(range(1, 256))  # order of alpha = 0x02 is 255
    x = 1
    for i in range(255):
        assert e[i] == x and lg[x] == i
        x = orc.gf_mul(x, 2)
    assert x == 1


def test_pow(orc, table):
    for a in (0, 1, 2, 3, 0x53, 0xCA, 0xFF):
        acc = 1
        for ex in range(300):
            assert orc.gf_pow(a, ex) == acc
            acc = table[acc, a]
