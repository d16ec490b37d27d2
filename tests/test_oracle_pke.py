"""Pins of the oracle's HQC.PKE (Alg. 1-3) and concatenated code.

Ground truth: Decrypt(Encrypt(m)) = m, with keys and randomness from the
seeded generator.  Decrypting with the public s (the literal text of Alg. 2)
instead of the secret y must fail, which documents the reading that the
decryption key is y.
"""
import numpy as np
import pytest

from paper_2512_12904_amd import synth


def sizes(orc, pid):
    p = orc.param(pid)
    p["rho"] = (p["rm_d"] - 1) // 2  # unique-decoding radius of the duplicated RM code
    return p


def test_rho_is_rm_unique_radius(orc):
    assert [sizes(orc, i)["rho"] for i in (1, 3, 5)] == [95, 159, 159]


@pytest.mark.parametrize("pid,count", [(1, 48), (3, 24), (5, 16)])
def test_round_trip_own_keys(orc, pid, count):
    p = sizes(orc, pid)
    h, x, y = synth.keys(0x11, pid, p, count)
    s = orc.keygen_batch(pid, h, x, y)
    m, r1, r2, e = synth.encryptions(0x11, pid, p, count, key_of=np.arange(count))
    u, v = orc.encrypt_batch(pid, h, s, m, r1, r2, e, key_of=np.arange(count))
    got = orc.decrypt_batch(pid, y, u, v)
    assert (got == m).all()
    # the ciphertext really is noisy: v - u*y - mG has weight fraction well above the RM radius
    p_ = orc.param(pid)
    for i in range(2):
        uy = orc.mul_sparse(p_["n"], u[i], y[i])
        cw = orc.code_encode(pid, m[i])
        err = v[i] ^ uy[: p_["vwords"]] ^ cw
        frac = np.unpackbits(err.view(np.uint8)).sum() / (p_["n1"] * p_["n2"])
        assert 0.15 < frac < 0.45


def test_round_trip_shared_key(orc):
    pid, count = 1, 32
    p = sizes(orc, pid)
    h, x, y = synth.keys(0x12, pid, p, 1)
    s = orc.keygen_batch(pid, h, x, y)
    m, r1, r2, e = synth.encryptions(0x12, pid, p, count)  # key 0 for all
    key_of = np.zeros(count, np.int64)
    u, v = orc.encrypt_batch(pid, h, s, m, r1, r2, e, key_of=key_of)
    got = orc.decrypt_batch(pid, y, u, v, key_of=key_of)
    assert (got == m).all()
    assert len({bytes(r) for r in m}) == count


def test_decrypt_with_public_s_fails(orc):
    pid = 1
    p = sizes(orc, pid)
    h, x, y = synth.keys(0x13, pid, p, 3)
    s = orc.keygen_batch(pid, h, x, y)
    m, r1, r2, e = synth.encryptions(0x13, pid, p, 3, key_of=np.arange(3))
    u, v = orc.encrypt_batch(pid, h, s, m, r1, r2, e, key_of=np.arange(3))
    for i in range(3):
        assert (orc.decrypt(pid, y[i], u[i], v[i]) == m[i]).all()
        # s is dense: use u*s by treating s's support as the sparse operand
        sbits = np.unpackbits(s[i].view(np.uint8), bitorder="little")[: p["n"]]
        us = orc.mul_sparse(p["n"], u[i], np.flatnonzero(sbits).astype(np.uint32))
        r = v[i] ^ us[: p["vwords"]]
        wrong, _, _ = orc.code_decode(pid, r)
        assert not (wrong == m[i]).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_code_round_trip_and_decrypt_with_zero_u(orc, pid):
    p = orc.param(pid)
    rng = np.random.default_rng(pid)
    for _ in range(10):
        m = rng.integers(0, 256, p["k"]).astype(np.uint8)
        cw = orc.code_encode(pid, m)
        got, sym, tr = orc.code_decode(pid, cw)
        assert (got == m).all() and tr["L"] == 0
        # Decrypt with u = 0 reduces to C.Decode(v)
        y = rng.choice(p["n"], p["w"], replace=False).astype(np.uint32)
        assert (orc.decrypt(pid, y, np.zeros(p["nwords"], np.uint64), cw) == m).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_stress_words_have_delta_symbol_errors(orc, pid):
    p = sizes(orc, pid)
    cnt = 12
    m, bad, dval, noise = synth.stress(0x44, pid, p, cnt)
    r = orc.stress_batch(pid, m, bad, dval, noise)
    got = orc.decode_batch(pid, r)
    assert (got == m).all()
    for i in range(3):
        _, sym, tr = orc.code_decode(pid, r[i])
        c = orc.rs_encode(p["n1"], p["k"], m[i])
        wrong = np.flatnonzero(sym != c)
        assert sorted(wrong.tolist()) == sorted(bad[i].tolist())
        assert (sym[bad[i]] == (c[bad[i]] ^ dval[i])).all()
        assert tr["L"] == p["delta"]
        # the noise stays within the RM radius of each clean block
        nb = np.unpackbits(noise[i].view(np.uint8), bitorder="little").reshape(p["n1"], p["n2"])
        clean = np.setdiff1d(np.arange(p["n1"]), bad[i])
        assert nb[clean].sum(1).max() <= p["rho"]
        assert nb[bad[i]].sum() == 0
