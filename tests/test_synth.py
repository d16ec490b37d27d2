"""The seeded input generator: published SplitMix64 output, determinism,
and the shape of its fixed-weight draws."""
import hashlib

import numpy as np

from paper_2512_12904_amd import synth

SIZES1 = dict(n=17669, n1=46, n2=384, k=16, delta=15, w=66, wr=75, we=75, rho=95)


def test_splitmix64_published_first_output():
    # first output of SplitMix64 from state 0 (Steele, Lea, Flood 2014)
    assert int(synth.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_fixed_weight_distinct_in_range():
    for bound, w in ((17669, 66), (57637, 149), (46, 15), (384, 95), (5, 5)):
        out = synth.fixed_weight(12345 + bound, bound, w)
        assert len(set(out.tolist())) == w
        assert out.max() < bound


def test_fixed_weight_roughly_uniform():
    counts = np.zeros(10, np.int64)
    for s in range(4000):
        counts[synth.fixed_weight(s, 10, 3)] += 1
    assert counts.min() > 0.9 * counts.mean() and counts.max() < 1.1 * counts.mean()


def test_keys_deterministic_and_frozen():
    h, x, y = synth.keys(0x1, 1, SIZES1, 4)
    h2, x2, y2 = synth.keys(0x1, 1, SIZES1, 4)
    assert (h == h2).all() and (x == x2).all() and (y == y2).all()
    assert int(h[:, -1].max() >> np.uint64(17669 % 64)) == 0  # bits >= n clear
    dig = hashlib.sha256(h.tobytes() + x.tobytes() + y.tobytes()).hexdigest()
    # the streams are frozen: a change of the generator changes every dataset
    assert dig == FROZEN_KEYS_SHA256, dig


def test_key_ranges_are_independent_of_batching():
    h, x, y = synth.keys(0x9, 3, dict(SIZES1, n=35851, w=100), 10)
    h2, x2, y2 = synth.keys(0x9, 3, dict(SIZES1, n=35851, w=100), 4, key_id0=6)
    assert (h[6:] == h2).all() and (y[6:] == y2).all()


def test_stress_draws_shape():
    m, bad, dval, noise = synth.stress(0x4, 1, SIZES1, 5)
    for i in range(5):
        assert len(set(bad[i].tolist())) == 15 and bad[i].max() < 46
        assert dval[i].min() >= 1
        nb = np.unpackbits(noise[i].view(np.uint8), bitorder="little").reshape(46, 384)
        assert nb[bad[i]].sum() == 0
        assert nb.sum(1).max() <= 95


FROZEN_KEYS_SHA256 = "813fb329f9c3f8a0e08aa32666a71fc40e30ffc0a48dc68b4028d61c72b354ea"
