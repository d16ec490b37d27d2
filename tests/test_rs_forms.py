"""Host model of the decoder's Reed-Solomon forms against the oracle.

The kernels run Massey's recursion with the discrepancies read from a vector
that is updated like Lambda (the reformulation of Sarwate and Shanbhag) on
bit-sliced vectors, keeping Massey's division c = Delta / gamma, so that
Lambda_0 stays 1; they form Omega = S Lambda mod x^(2 delta) by a Horner
scheme on the same planes.  This is a plain-Python model of those steps
(planes as Python integers, scalar products as sum_k c_k alpha^k T with
alpha x as a renaming plus three XORs), compared with the oracle's
Berlekamp-Massey on random syndromes (decoder failure at every degree),
syndromes of words with at most delta errors, and sparse syndromes.  Lambda
and Omega must equal the oracle's exactly."""
import random

import numpy as np
import pytest

import oracle


def _inv(a):
    return int(oracle.gf_inv(a))


def _mul(a, b):
    return int(oracle.gf_mul(a, b))


def _planes(vals):
    P = [0] * 8
    for i, v in enumerate(vals):
        for j in range(8):
            if (v >> j) & 1:
                P[j] |= 1 << i
    return P


def _elems(P, n):
    return [sum(((P[j] >> i) & 1) << j for j in range(8)) for i in range(n)]


def _scalar_times(c, T):
    # sum_k c_k alpha^k T on planes; alpha x: (p0..p7) -> (p7, p0, p1^p7, p2^p7, p3^p7, p4, p5, p6)
    acc, cur = [0] * 8, list(T)
    for k in range(8):
        if (c >> k) & 1:
            acc = [a ^ b for a, b in zip(acc, cur)]
        p = cur
        cur = [p[7], p[0], p[1] ^ p[7], p[2] ^ p[7], p[3] ^ p[7], p[4], p[5], p[6]]
    return acc


def dvbm_model(S, td, width=64):
    """Lambda from S_1..S_td, as the kernels compute it.
    Planes are `width` bits wide and never masked during the steps: the
    elements that are not live only move upwards."""
    full = (1 << width) - 1
    A = _planes(S)
    TA = [(p << 1) & full for p in A]
    C = _planes([1])
    TC = [(p << 1) & full for p in C]
    gamma, k = 1, 0
    for r in range(td):
        d0 = sum(((A[j] >> r) & 1) << j for j in range(8))
        c = _mul(d0, _inv(gamma))
        sw = d0 != 0 and k >= 0
        UA, UC = (A, C) if sw else (TA, TC)
        A = [a ^ b for a, b in zip(A, _scalar_times(c, TA))]
        C = [a ^ b for a, b in zip(C, _scalar_times(c, TC))]
        TA = [(p << 1) & full for p in UA]
        TC = [(p << 1) & full for p in UC]
        if sw:
            gamma, k = d0, -k - 1
        else:
            k += 1
    return _elems(C, td + 1)


def omega_model(S, lam, td):
    """Omega = S(x) Lambda(x) mod x^td by Horner on planes, W <- x W + Lambda_i S."""
    SP = _planes(S)
    W = [0] * 8
    for i in range(td, -1, -1):
        W = [(w << 1) for w in W]
        W = [a ^ b for a, b in zip(W, _scalar_times(lam[i], SP))]
    return _elems([w & ((1 << td) - 1) for w in W], td)



@pytest.mark.parametrize("pid", [1, 3, 5])
def test_vector_form_equals_massey(pid):
    p = oracle.param(pid)
    n1, k = p["n1"], p["k"]
    td = n1 - k
    rng = random.Random(0xB17 + pid)
    degs = set()
    # single nonzero syndromes push L (and the degree of Lambda) up to 2 delta
    special = [[0] * i + [1 + i] + [0] * (td - 1 - i)
               for i in range(0, td, 3)] + [[5] * td, [0] * td]
    for trial in range(240 + len(special)):
        kind = trial % 3 if trial < 240 else 3
        if kind == 3:
            S = special[trial - 240]
        elif kind == 0:  # uniform syndromes: decoder failure, Lambda of any degree
            S = [rng.randrange(256) for _ in range(td)]
        elif kind == 1:  # a codeword with at most delta symbol errors
            m = np.array([rng.randrange(256) for _ in range(k)], np.uint8)
            c = oracle.rs_encode(n1, k, m).copy()
            for j in rng.sample(range(n1), rng.randint(0, td // 2)):
                c[j] ^= rng.randrange(1, 256)
            S = [int(x) for x in oracle.rs_syndromes(n1, td, c)]
        else:  # mostly zero syndromes
            S = [rng.choice([0, 0, 0, rng.randrange(256)]) for _ in range(td)]
        ref = [int(x) for x in oracle.rs_berlekamp_massey(td, np.array(S, np.uint8))[0]]
        got = dvbm_model(S, td)
        assert got == ref, (pid, trial, S)
        degs.add(max([i for i, v in enumerate(ref) if v] + [0]))
        # the Horner form of Omega equals the truncated product written out
        om = omega_model(S, got, td)
        direct = [0] * td
        for e in range(td):
            for i in range(e + 1):
                direct[e] ^= _mul(ref[i], S[e - i])
        assert om == direct
    # the failure cases reached degrees above delta
    assert max(degs) > td // 2 + 1


def test_scalar_times_is_field_multiplication():
    rng = random.Random(7)
    vals = [rng.randrange(256) for _ in range(40)]
    for c in [0, 1, 2, 0x1D, 0x80, 0xFF] + [rng.randrange(256) for _ in range(20)]:
        got = _elems(_scalar_times(c, _planes(vals)), len(vals))
        assert got == [_mul(c, v) for v in vals]
