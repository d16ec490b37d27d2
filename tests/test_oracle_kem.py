"""Pins for the KEM part of the oracle (kem_oracle.c): SHAKE256 against an
independent implementation (Python's hashlib, FIPS 202), Floyd's sampler
against exhaustive enumeration, and the KEM's correctness and implicit
rejection against hashes computed outside the oracle."""
import hashlib
import itertools

import numpy as np
import pytest

import oracle
from paper_2512_12904_amd import synth
from tests import datasets


def test_shake256_matches_hashlib():
    rng = np.random.default_rng(202)
    # lengths around the 136-byte rate, and the key-derivation inputs of the
    # three sets (k + 8 U + 8 V + 1 bytes)
    lens = [0, 1, 2, 134, 135, 136, 137, 271, 272, 273, 1000, 4441, 9073, 14441]
    for n in lens:
        data = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        for out in (1, 31, 32, 135, 136, 137, 900, 1788):
            assert oracle.shake256(data, out) == hashlib.shake_256(data).digest(out), (n, out)


def test_keccak_permutation_through_shake():
    # SHAKE256 of the empty string is one permutation of the padded block:
    # byte 0 = 0x1F, byte 135 = 0x80
    st = np.zeros(25, np.uint64)
    st[0] = 0x1F
    st[16] = np.uint64(0x80) << np.uint64(56)
    out = oracle.keccak_f1600(st)
    got = b"".join(int(w).to_bytes(8, "little") for w in out)[:136]
    assert got == hashlib.shake_256(b"").digest(136)


def _draw_for(n, i, t):
    # the smallest 32-bit a with i + floor(a (n - i) / 2^32) = i + t
    return -(-(t << 32) // (n - i))


@pytest.mark.parametrize("n,w", [(6, 3), (7, 4), (5, 5), (8, 1)])
def test_fixed_weight_is_floyd_uniform(n, w):
    # enumerate every tuple of exactly uniform draws p_i in [i, n): each
    # w-subset must come out the same number of times (w! each), all distinct
    counts = {}
    for ts in itertools.product(*[range(n - i) for i in range(w)]):
        a = np.array([_draw_for(n, i, t) for i, t in enumerate(ts)], np.uint32)
        s = oracle.fixed_weight(n, w, a)
        assert len(set(s.tolist())) == w and max(s) < n
        key = tuple(sorted(s.tolist()))
        counts[key] = counts.get(key, 0) + 1
    import math
    assert len(counts) == math.comb(n, w)
    assert set(counts.values()) == {math.factorial(w)}


def test_fixed_weight_draw_mapping_ends():
    n, w = 17669, 75
    z = oracle.fixed_weight(n, w, np.zeros(w, np.uint32))
    # all draws 0: p_i = i, no collisions
    assert z.tolist() == list(range(w))
    top = oracle.fixed_weight(n, w, np.full(w, 0xFFFFFFFF, np.uint32))
    # all draws maximal: p_i = n - 1 for every i; only the last keeps it
    assert top[-1] == n - 1 and top[:-1].tolist() == list(range(w - 1))


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_fixed_weight_at_hqc_sizes(pid):
    p = oracle.param(pid)
    a = synth.words(0x900 + pid, (64, p["we"] // 2 + 1)).view(np.uint32)[:, :p["we"]]
    for row in a:
        s = oracle.fixed_weight(p["n"], p["we"], row)
        assert len(set(s.tolist())) == p["we"] and int(s.max()) < p["n"]


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_seed_words_are_shake_of_m(pid):
    p = oracle.param(pid)
    m = synth.words(0x910 + pid, (p["k"] // 8,)).view(np.uint8)
    nw = 2 * p["wr"] + p["we"]
    ref = np.frombuffer(hashlib.shake_256(m.tobytes() + b"\x03").digest(4 * nw), "<u4")
    assert (oracle.kem_seed_words(pid, m) == ref).all()


def _kem_case(pid, seed):
    d = datasets.pke(pid, 1, seed)
    p = oracle.param(pid)
    sigma = synth.words(seed ^ 0x5157, (p["k"] // 8,)).view(np.uint8)
    return d["h"][0], d["s"][0], d["y_keys"][0], sigma, d["m"][0], p


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_kem_round_trip_and_key_definition(pid):
    h, s, y, sigma, m, p = _kem_case(pid, 0xA00 + pid)
    u, v, key = oracle.kem_encaps(pid, h, s, m)
    # the ciphertext is PKE.Encrypt with the supports drawn from Z(m)
    a = oracle.kem_seed_words(pid, m)
    wr, we = p["wr"], p["we"]
    r1 = oracle.fixed_weight(p["n"], wr, a[:wr])
    r2 = oracle.fixed_weight(p["n"], wr, a[wr:2 * wr])
    e = oracle.fixed_weight(p["n"], we, a[2 * wr:])
    u2, v2 = oracle.encrypt(pid, h, s, m, r1, r2, e)
    assert (u == u2).all() and (v == v2).all()
    ref = hashlib.shake_256(m.tobytes() + u.astype("<u8").tobytes() + v.astype("<u8").tobytes()
                            + b"\x04").digest(32)
    assert bytes(key) == ref
    k2, ok = oracle.kem_decaps(pid, h, s, y, sigma, u, v)
    assert ok and bytes(k2) == ref


@pytest.mark.parametrize("pid", [1, 3, 5])
@pytest.mark.parametrize("where", ["u", "v", "u_pad"])
def test_kem_implicit_rejection(pid, where):
    h, s, y, sigma, m, p = _kem_case(pid, 0xB00 + pid)
    u, v, key = oracle.kem_encaps(pid, h, s, m)
    u, v = u.copy(), v.copy()
    if where == "u":
        u[3] ^= np.uint64(1 << 17)
    elif where == "v":
        v[-1] ^= np.uint64(1)
    else:  # a bit >= n of u: ignored by decryption, but not the same ciphertext
        u[-1] ^= np.uint64(1) << np.uint64(63)
    k2, ok = oracle.kem_decaps(pid, h, s, y, sigma, u, v)
    assert not ok
    ref = hashlib.shake_256(sigma.tobytes() + u.astype("<u8").tobytes() +
                            v.astype("<u8").tobytes() + b"\x04").digest(32)
    assert bytes(k2) == ref and bytes(k2) != bytes(key)


def test_kem_batches_match_single_calls():
    pid = 1
    d = datasets.pke(pid, 6, 0xC00)
    p = oracle.param(pid)
    sigma = synth.words(0xC01, (6, p["k"] // 8)).view(np.uint8)
    u, v, key = oracle.kem_encaps_batch(pid, d["h"], d["s"], d["m"])
    for i in range(6):
        u1, v1, k1 = oracle.kem_encaps(pid, d["h"][i], d["s"][i], d["m"][i])
        assert (u[i] == u1).all() and (v[i] == v1).all() and (key[i] == k1).all()
    v[2, 0] ^= np.uint64(4)
    k2, ok = oracle.kem_decaps_batch(pid, d["h"], d["s"], d["y_keys"], sigma, u, v)
    assert ok.tolist() == [True, True, False, True, True, True]
    assert (np.delete(k2, 2, 0) == np.delete(key, 2, 0)).all() and (k2[2] != key[2]).any()
