"""Pins of the oracle's shortened Reed-Solomon code over GF(2^8).

- g(x) has exactly the roots alpha^1 .. alpha^(2 delta) (narrow sense).
- Codewords have zero syndromes; the code is MDS with the Table I distance.
- Decoding recovers m exactly for up to delta symbol errors, and the error
  locator equals the closed form prod (1 - X_l x) over the error locations.
- On a tiny code, decoding equals the brute-force nearest codeword.
- The syndrome indexing reproduces the Sec. III-D multiplication count.
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def poly_eval(orc, coeffs, x):
    acc = 0
    for c in reversed(list(coeffs)):
        acc = orc.gf_mul(acc, x) ^ int(c)
    return acc


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_generator_roots(orc, pid):
    p = orc.param(pid)
    td = 2 * p["delta"]
    g = orc.rs_generator(td)
    assert g[td] == 1
    roots = [i for i in range(255) if poly_eval(orc, g, orc.gf_pow(2, i)) == 0]
    assert roots == list(range(1, td + 1))


def test_table_i_consistency(orc):
    rows = json.load(open(os.path.join(GOLD, "table1.json")))["rows"]
    for row in rows:
        p = orc.param(row["id"])
        assert p["n"] == row["N"] and p["w"] == row["omega"]
        assert p["wr"] == p["we"] == row["omega_er"]
        assert [p["n1"], p["k"], p["rs_d"]] == row["rs"]
        assert [p["n2"], 8, p["rm_d"]] == row["rm"]
        # MDS: d = n1 - k + 1 = 2 delta + 1
        assert p["rs_d"] == p["n1"] - p["k"] + 1 == 2 * p["delta"] + 1


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_codewords_zero_syndromes_and_systematic(orc, pid):
    p = orc.param(pid)
    n1, k, td = p["n1"], p["k"], 2 * p["delta"]
    rng = np.random.default_rng(pid)
    for _ in range(300):
        m = rng.integers(0, 256, k).astype(np.uint8)
        c = orc.rs_encode(n1, k, m)
        assert (c[td:] == m).all()
        assert (orc.rs_syndromes(n1, td, c) == 0).all()
        # c(x) evaluated directly at the roots
        assert poly_eval(orc, c, orc.gf_pow(2, 1)) == 0
        assert poly_eval(orc, c, orc.gf_pow(2, td)) == 0


@pytest.fixture(scope="module")
def tiny_code(orc):
    """All 65,536 codewords of the shortened [6, 2, 5] code (delta = 2)."""
    n1, k = 6, 2
    cw = np.zeros((256 * 256, n1), np.uint8)
    for a in range(256):
        for b in range(256):
            cw[a * 256 + b] = orc.rs_encode(n1, k, np.array([a, b], np.uint8))
    return cw


def test_tiny_code_is_mds(tiny_code):
    weights = (tiny_code[1:] != 0).sum(1)
    assert weights.min() == 6 - 2 + 1


def test_tiny_code_brute_force_nearest(orc, tiny_code):
    n1, k = 6, 2
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(3000):
        if trial % 3 == 0:
            r = rng.integers(0, 256, n1).astype(np.uint8)  # arbitrary word
        else:
            r = tiny_code[int(rng.integers(0, 65536))].copy()
            pos = rng.choice(n1, int(rng.integers(0, 3)), replace=False)
            r[pos] ^= rng.integers(1, 256, len(pos)).astype(np.uint8)
        d = (tiny_code != r[None, :]).sum(1)
        best = np.flatnonzero(d == d.min())
        if d.min() <= 2:  # the unique nearest codeword (radius 2 < 5/2)
            assert len(best) == 1
            got, tr = orc.rs_decode(n1, k, r)
            assert (got == tiny_code[best[0]][n1 - k:]).all()
            assert tr["L"] == d.min()
            checked += 1
    assert checked > 1500


def test_syndrome_indexing_and_paper_count(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_counts.json")))
    p = orc.param(1)
    n1, td = p["n1"], 2 * p["delta"]
    for j in range(n1):
        c = np.zeros(n1, np.uint8)
        c[j] = 1
        S = orc.rs_syndromes(n1, td, c)
        assert list(S) == [orc.gf_pow(2, i * j) for i in range(1, td + 1)]
    # one product c_j * alpha^(i j) per syndrome i and position j >= 1 (position
    # 0 multiplies by alpha^0 = 1): 2 delta (n1 - 1) = 1,350 for HQC-1, the
    # Sec. III-D figure.  Indexing the syndromes from i = 0 instead would give
    # (2 delta - 1)(n1 - 1) = 1,305.
    products = sum(1 for i in range(1, td + 1) for j in range(1, n1))
    assert products == gold["syndrome_multiplications_hqc1"]
    assert sum(1 for i in range(0, td) for j in range(1, n1) if i) != products


def closed_form_locator(orc, positions, length):
    lam = [1] + [0] * (length - 1)
    for j in positions:
        X = orc.gf_pow(2, j)
        new = lam[:]
        for i in range(1, length):
            new[i] ^= orc.gf_mul(X, lam[i - 1])
        lam = new
    return np.array(lam, np.uint8)


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decode_within_radius(orc, pid):
    p = orc.param(pid)
    n1, k, delta = p["n1"], p["k"], p["delta"]
    td = 2 * delta
    rng = np.random.default_rng(100 + pid)
    for trial in range(200):
        m = rng.integers(0, 256, k).astype(np.uint8)
        c = orc.rs_encode(n1, k, m)
        nerr = trial % (delta + 1) if trial < 150 else delta
        pos = rng.choice(n1, nerr, replace=False)
        if trial == 0:
            pos = np.array([0, n1 - 1][: max(0, min(2, nerr))], dtype=np.int64)
            nerr = len(pos)
        val = rng.integers(1, 256, nerr).astype(np.uint8)
        r = c.copy()
        r[pos] ^= val
        got, tr = orc.rs_decode(n1, k, r)
        assert (got == m).all()
        assert tr["L"] == nerr
        assert (tr["lambda"] == closed_form_locator(orc, pos, td + 1)).all()
        assert sorted(np.flatnonzero(tr["located"]).tolist()) == sorted(pos.tolist())
        err = np.zeros(n1, np.uint8)
        err[pos] = val
        assert (tr["err"] == err).all()


def test_berlekamp_massey_zero_syndromes(orc):
    lam, L = orc.rs_berlekamp_massey(30, np.zeros(30, np.uint8))
    assert L == 0 and lam[0] == 1 and (lam[1:] == 0).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_beyond_radius_is_deterministic(orc, pid):
    # parity unpinned beyond delta: only determinism and totality are checked
    p = orc.param(pid)
    rng = np.random.default_rng(200 + pid)
    for _ in range(50):
        r = rng.integers(0, 256, p["n1"]).astype(np.uint8)
        a, _ = orc.rs_decode(p["n1"], p["k"], r)
        b, _ = orc.rs_decode(p["n1"], p["k"], r)
        assert (a == b).all()
