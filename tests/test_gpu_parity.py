"""GPU parity: the HIP path (through the C ABI) against the CPU oracle and the
ground-truth messages, bit-exact (integer work: the tolerance is zero)."""
import numpy as np
import pytest

import oracle
from paper_2512_12904_amd import synth
from tests import datasets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hqc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc as h
    h.lib()
    return h


def dev(a):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("shared", [False, True])
def test_hqc1_batch64(hqc, shared):
    say("case: HQC-1 x64 shared_key=%s" % shared)
    d = datasets.pke(1, 64, 0x1, shared_key=shared)
    got = host(hqc.decrypt_batch(1, dev(d["u"]), dev(d["v"]), dev(d["y"])))
    assert (got == d["m"]).all()
    ref = oracle.decrypt_batch(1, d["y"], d["u"], d["v"])
    assert (got == ref).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
@pytest.mark.parametrize("count,grid", [(1, 0), (7, 0), (130, 0), (130, 7), (257, 64)])
def test_ragged_counts_and_persistent_grid(hqc, pid, count, grid):
    say("case: pid=%d count=%d grid=%d" % (pid, count, grid))
    d = datasets.pke(pid, count, 0x100 + pid)
    got = host(hqc.decrypt_batch(pid, dev(d["u"]), dev(d["v"]), dev(d["y"]), grid=grid))
    assert (got == d["m"]).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_beyond_radius_matches_oracle(hqc, pid):
    say("case: beyond radius pid=%d" % pid)
    u, v, y = _random_inputs(pid)
    got = host(hqc.decrypt_batch(pid, dev(u), dev(v), dev(y)))
    ref = oracle.decrypt_batch(pid, y, u, v)
    assert (got == ref).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_u_zero_and_high_bits_ignored(hqc, pid):
    say("case: u edge pid=%d" % pid)
    d = datasets.pke(pid, 24, 0x200 + pid)
    p = datasets.sizes(pid)
    u = d["u"].copy()
    u[:, -1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(p["n"] % 64)  # bits >= n set
    got = host(hqc.decrypt_batch(pid, dev(u), dev(d["v"]), dev(d["y"])))
    assert (got == d["m"]).all()
    # u = 0: decryption is C.Decode(v)
    z = np.zeros_like(d["u"])
    cw = np.stack([oracle.code_encode(pid, mm) for mm in d["m"]])
    got = host(hqc.decrypt_batch(pid, dev(z), dev(cw), dev(d["y"])))
    assert (got == d["m"]).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decode_stress(hqc, pid):
    say("case: decode stress pid=%d" % pid)
    d = datasets.stress(pid, 300, 0x4)
    got = host(hqc.decode_batch(pid, dev(d["r"])))
    assert (got == d["m"]).all()
    # decode == decrypt with u = 0
    p = datasets.sizes(pid)
    z = np.zeros((300, p["nwords"]), np.uint64)
    y = np.tile(np.arange(p["w"], dtype=np.uint32), (300, 1))
    got2 = host(hqc.decrypt_batch(pid, dev(z), dev(d["r"]), dev(y)))
    assert (got2 == got).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decode_random_words_match_oracle(hqc, pid):
    say("case: decode random pid=%d" % pid)
    p = datasets.sizes(pid)
    r = synth.words(0x71 + pid, (64, p["vwords"]))
    r[0] = 0
    r[1] = np.uint64(0xFFFFFFFFFFFFFFFF)
    got = host(hqc.decode_batch(pid, dev(r)))
    assert (got == oracle.decode_batch(pid, r)).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
@pytest.mark.parametrize("tile", [1, 5, 16, 31, 32, 33, 64])
def test_tile_sizes(hqc, pid, tile):
    # tiles of at most 32 items decode each Reed-Solomon word on a pair of
    # lanes (the words of consecutive small tiles of a workgroup together,
    # up to 32), larger ones on one lane; 200 = 6 * 33 + 2 also leaves a
    # ragged last tile
    say("case: pid=%d tile=%d grid=3" % (pid, tile))
    d = datasets.stress(pid, 200, 0x600 + tile)
    got = host(hqc.decode_batch(pid, dev(d["r"]), grid=3, tile=tile))
    assert (got == d["m"]).all()
    p = datasets.sizes(pid)
    r = synth.words(0x700 + tile + pid, (70, p["vwords"]))
    got = host(hqc.decode_batch(pid, dev(r), grid=3, tile=tile))
    assert (got == oracle.decode_batch(pid, r)).all()


def test_mixed_launch_equals_separate(hqc):
    say("case: mixed decrypt + decode")
    ds = {pid: datasets.pke(pid, 50 + pid, 0x300 + pid) for pid in (5, 1, 3)}
    items = [{"pid": pid, "u": dev(d["u"]), "v": dev(d["v"]), "y": dev(d["y"])} for pid, d in ds.items()]
    outs = hqc.decrypt_mixed(items, grid=37)
    for (pid, d), o in zip(ds.items(), outs):
        assert (host(o) == d["m"]).all()
    st = {pid: datasets.stress(pid, 40, 0x44) for pid in (1, 3, 5)}
    outs = hqc.decode_mixed([{"pid": pid, "r": dev(d["r"])} for pid, d in st.items()])
    for (pid, d), o in zip(st.items(), outs):
        assert (host(o) == d["m"]).all()


def test_per_item_and_graph_modes(hqc):
    say("case: per-item and graph launch modes")
    d = datasets.pke(3, 33, 0x400)
    u, v, y = dev(d["u"]), dev(d["v"]), dev(d["y"])
    a = host(hqc.decrypt_batch(3, u, v, y, flags=hqc.F_PER_ITEM_LAUNCH))
    assert (a == d["m"]).all()
    for _ in range(3):
        out = hqc.decrypt_batch(3, u, v, y, flags=hqc.F_GRAPH)
        assert (host(out) == d["m"]).all()


@pytest.mark.parametrize("tile", [0, 64])
def test_keystore(hqc, tile):
    say("case: keystore tile=%d" % tile)
    import torch
    d = datasets.pke(1, 40, 0x500)
    ks = hqc.KeyStore(40, 1, 1)
    ks.put(1, 0, d["y_keys"])
    ids = torch.arange(40, dtype=torch.int32, device="cuda")
    got = host(hqc.decrypt_batch_keyed(1, ks, dev(d["u"]), dev(d["v"]), ids, tile=tile))
    assert (got == d["m"]).all()
    ids[5] = 1000  # out of range: zeros, counted
    got = host(hqc.decrypt_batch_keyed(1, ks, dev(d["u"]), dev(d["v"]), ids, tile=tile))
    assert (got[5] == 0).all() and (np.delete(got, 5, 0) == np.delete(d["m"], 5, 0)).all()
    assert ks.bad_ids() == 1
    with pytest.raises(hqc.HqcError):
        ks.put(1, 0, np.zeros(66, np.uint32))  # repeated index
    with pytest.raises(hqc.HqcError):
        ks.put(1, 40, d["y_keys"][:1])  # slot beyond capacity
    ks.close()


def test_bad_buffer_sizes_rejected(hqc):
    import torch
    say("case: size validation")
    p = datasets.sizes(1)
    r = torch.zeros((4, p["vwords"]), dtype=torch.int64, device="cuda")
    out = torch.zeros((4, 16), dtype=torch.uint8, device="cuda")
    L = hqc.lib()
    import ctypes
    prm = hqc.Params(1, 0, None, 0, 0)
    # count larger than the allocation behind r: refused
    rc = L.hqc_decode_batch(ctypes.byref(prm), ctypes.c_void_p(r.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), 1 << 20)
    assert rc == hqc.HQC_EINVAL


def _bits(words, nbits):
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:nbits]


def _words(bits):
    return np.packbits(bits, bitorder="little").view(np.uint64)


def _structured_words(pid):
    """Received words at the decoders' edges: codewords with exactly
    delta + 1, delta + 2 and 2 delta wrong RS symbols (just past the radius:
    Berlekamp-Massey ends above degree delta), blocks set to all zeros or all
    ones, and blocks equidistant from two RM codewords (Hadamard peaks of
    equal magnitude: the tie rule decides).  64 words, 8 of each kind."""
    p = datasets.sizes(pid)
    par = oracle.param(pid)
    n1, n2, delta = par["n1"], par["n2"], par["delta"]
    mult = n2 // 128
    words = n2 // 64
    rng = np.random.default_rng(0xB7 + pid)
    rows = []
    for kind in range(8):
        for rep in range(8):
            m = rng.integers(0, 256, p["k"], dtype=np.uint8)
            r = oracle.code_encode(pid, m).copy()
            blocks = r.reshape(n1, words)
            if kind < 3:
                # exactly delta + 1, delta + 2 or 2 delta blocks replaced by
                # other RM codewords (each a whole wrong symbol)
                t = (delta + 1, delta + 2, 2 * delta)[kind]
                for b in rng.choice(n1, t, replace=False):
                    cur = oracle.rm_decode(mult, blocks[b])[0]
                    new = (int(cur) + 1 + int(rng.integers(0, 255))) % 256
                    blocks[b] = oracle.rm_encode(mult, new)
            elif kind == 3:
                blocks[rng.choice(n1, delta + 1, replace=False)] = 0
            elif kind == 4:
                blocks[rng.choice(n1, delta + 1, replace=False)] = np.uint64(0xFFFFFFFFFFFFFFFF)
            else:
                # ties: a block halfway between the codewords of a and b (half
                # of the positions where they differ flipped), on 1, delta + 1
                # or every block
                t = (1, delta + 1, n1)[kind - 5]
                for blk in rng.choice(n1, t, replace=False):
                    a, b = (int(v) for v in rng.choice(256, 2, replace=False))
                    ca = _bits(oracle.rm_encode(mult, a), n2)
                    cb = _bits(oracle.rm_encode(mult, b), n2)
                    diff = np.flatnonzero(ca != cb)
                    flip = rng.choice(diff, len(diff) // 2, replace=False)
                    c = ca.copy()
                    c[flip] ^= 1
                    blocks[blk] = _words(c)
            rows.append(r)
    return np.stack(rows)


def _random_inputs(pid, cnt=96):
    """Uniform u and v with arbitrary y (indices >= n, repeats, 0 and n - 1):
    no valid message exists, the output is fixed only by the decoder
    conventions."""
    p = datasets.sizes(pid)
    u = synth.words(0x51 + pid, (cnt, p["nwords"]))
    v = synth.words(0x61 + pid, (cnt, p["vwords"]))
    rng = np.random.default_rng(pid)
    y = rng.integers(0, 2 ** 32, (cnt, p["w"]), dtype=np.uint64).astype(np.uint32)
    y[0, :] = 0
    y[1, :2] = [0, p["n"] - 1]
    y[2, :] = p["n"] - 1
    y[3, 1] = y[3, 0]
    y[4:40] %= p["n"]
    return u, v, y


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_structured_beyond_radius_matches_oracle(hqc, pid):
    """_structured_words decoded by the GPU and the oracle, then decrypted
    with u = 0."""
    say("case: structured beyond radius pid=%d" % pid)
    p = datasets.sizes(pid)
    r = _structured_words(pid)
    got = host(hqc.decode_batch(pid, dev(r)))
    assert (got == oracle.decode_batch(pid, r)).all()
    # the same words through decryption with u = 0
    z = np.zeros((len(r), p["nwords"]), np.uint64)
    y = np.tile(np.arange(p["w"], dtype=np.uint32), (len(r), 1))
    assert (host(hqc.decrypt_batch(pid, dev(z), dev(r), dev(y))) == got).all()


@pytest.mark.parametrize("tile", [0, 64, 1, 3, 20])
def test_mixed_kernel_beyond_radius_matches_oracle(hqc, tile):
    """The three-set kernel (the instance the decoder-stress launch runs) on
    the inputs of the single-set beyond-radius tests: random ciphertexts with
    arbitrary keys, uniformly random received words and the structured edge
    words, all three sets in one launch each, every byte against the oracle.
    Tile 0 is the library's choice (lane pairs at these sizes), 64 the
    one-lane Reed-Solomon form for HQC-1 and HQC-3; small tiles on small
    grids give each workgroup many tiles, whose words are decoded together
    and whose run crosses from one parameter set to the next."""
    say("case: mixed kernel beyond radius tile=%d" % tile)
    sets = (1, 3, 5)
    rnd = {pid: _random_inputs(pid) for pid in sets}
    outs = hqc.decrypt_mixed([{"pid": pid, "u": dev(u), "v": dev(v), "y": dev(y)}
                              for pid, (u, v, y) in rnd.items()], grid=11, tile=tile)
    for (pid, (u, v, y)), o in zip(rnd.items(), outs):
        assert (host(o) == oracle.decrypt_batch(pid, y, u, v)).all(), pid
    words = {}
    for pid in sets:
        p = datasets.sizes(pid)
        rw = synth.words(0x81 + pid, (32, p["vwords"]))
        rw[0] = 0
        rw[1] = np.uint64(0xFFFFFFFFFFFFFFFF)
        words[pid] = np.concatenate([_structured_words(pid), rw])
    outs = hqc.decode_mixed([{"pid": pid, "r": dev(r)} for pid, r in words.items()],
                            grid=5, tile=tile)
    for (pid, r), o in zip(words.items(), outs):
        assert (host(o) == oracle.decode_batch(pid, r)).all(), pid
    # the same words through the mixed decryption with u = 0
    items = []
    for pid, r in words.items():
        p = datasets.sizes(pid)
        z = np.zeros((len(r), p["nwords"]), np.uint64)
        y = np.tile(np.arange(p["w"], dtype=np.uint32), (len(r), 1))
        items.append({"pid": pid, "u": dev(z), "v": dev(r), "y": dev(y)})
    outs2 = hqc.decrypt_mixed(items, tile=tile)
    for o, o2 in zip(outs, outs2):
        assert (host(o) == host(o2)).all()


@pytest.mark.parametrize("tile", [0, 64, 3])
def test_keyed_kernels_beyond_radius_match_oracle(hqc, tile):
    """The keyed kernel (the instance the serving loop runs), per set and as
    one mixed launch, on random ciphertexts and on the structured edge words
    (u = 0), with keystore keys that include the extreme supports
    {0 .. w-1} and {n-w .. n-1}; every byte against the oracle."""
    import torch
    say("case: keyed kernels beyond radius tile=%d" % tile)
    sets = (1, 3, 5)
    nkeys = 8
    keys, cases = {}, {}
    for pid in sets:
        p = datasets.sizes(pid)
        y = synth.keys(0x91 + pid, pid, p, nkeys)[2]
        y[0] = np.arange(p["w"], dtype=np.uint32)
        y[1] = np.arange(p["n"] - p["w"], p["n"], dtype=np.uint32)
        keys[pid] = y
    ks = hqc.KeyStore(nkeys, nkeys, nkeys)
    try:
        for pid in sets:
            ks.put(pid, 0, keys[pid])
        for pid in sets:
            p = datasets.sizes(pid)
            cnt = 80
            u = synth.words(0xA1 + pid, (cnt, p["nwords"]))
            v = synth.words(0xA2 + pid, (cnt, p["vwords"]))
            r = _structured_words(pid)
            u = np.concatenate([u, np.zeros((len(r), p["nwords"]), np.uint64)])
            v = np.concatenate([v, r])
            kid = (np.arange(len(u)) * 5 % nkeys).astype(np.uint32)
            cases[pid] = (u, v, kid, oracle.decrypt_batch(pid, keys[pid][kid], u, v))
        for pid, (u, v, kid, ref) in cases.items():
            got = host(hqc.decrypt_batch_keyed(pid, ks, dev(u), dev(v), dev(kid), tile=tile))
            assert (got == ref).all(), pid
        outs = hqc.decrypt_mixed_keyed(ks, [{"pid": pid, "u": dev(u), "v": dev(v), "key_ids": dev(kid)}
                                            for pid, (u, v, kid, _) in cases.items()],
                                       grid=7, tile=tile)
        for (pid, (u, v, kid, ref)), o in zip(cases.items(), outs):
            assert (host(o) == ref).all(), pid
        assert ks.bad_ids() == 0
        # an out-of-range id in one segment of a mixed launch: zeros there, counted
        u, v, kid, ref = cases[3]
        kid = kid.copy()
        kid[4] = nkeys + 100
        outs = hqc.decrypt_mixed_keyed(ks, [{"pid": 3, "u": dev(u), "v": dev(v), "key_ids": dev(kid)},
                                            {"pid": 1, "u": dev(cases[1][0]), "v": dev(cases[1][1]),
                                             "key_ids": dev(cases[1][2])}], tile=tile)
        got3 = host(outs[0])
        assert (got3[4] == 0).all() and (np.delete(got3, 4, 0) == np.delete(ref, 4, 0)).all()
        assert (host(outs[1]) == cases[1][3]).all()
        assert ks.bad_ids() == 1
        torch.cuda.synchronize()
    finally:
        ks.close()


@pytest.mark.parametrize("pid", [1, 3])
@pytest.mark.parametrize("tile", [0, 1, 31, 32, 33, 64])
def test_shape_b_kernels_match_oracle(hqc, pid, tile):
    """The second kernel shape (RM blocks on lane pairs, smaller LDS, three
    wavefronts per SIMD; separate kernel instances for decryption, decoding
    and keyed decryption): honest ciphertexts (ground truth), random
    ciphertexts with arbitrary keys and the structured edge words (oracle),
    over tile sizes with a ragged last tile, every byte compared."""
    say("case: shape B pid=%d tile=%d" % (pid, tile))
    p = datasets.sizes(pid)
    d = datasets.pke(pid, 70, 0x800 + pid)
    got = host(hqc.decrypt_batch(pid, dev(d["u"]), dev(d["v"]), dev(d["y"]), grid=3, tile=tile,
                                 shape=2))
    assert (got == d["m"]).all()
    u, v, y = _random_inputs(pid)
    got = host(hqc.decrypt_batch(pid, dev(u), dev(v), dev(y), grid=5, tile=tile, shape=2))
    assert (got == oracle.decrypt_batch(pid, y, u, v)).all()
    r = _structured_words(pid)
    got = host(hqc.decode_batch(pid, dev(r), grid=2, tile=tile, shape=2))
    assert (got == oracle.decode_batch(pid, r)).all()
    st = datasets.stress(pid, 50, 0x810 + pid)
    assert (host(hqc.decode_batch(pid, dev(st["r"]), tile=tile, shape=2)) == st["m"]).all()
    ks = hqc.KeyStore(70 if pid == 1 else 1, 70 if pid == 3 else 1, 1)
    try:
        ks.put(pid, 0, d["y_keys"])
        import torch
        ids = torch.arange(70, dtype=torch.int32, device="cuda")
        got = host(hqc.decrypt_batch_keyed(pid, ks, dev(d["u"]), dev(d["v"]), ids, tile=tile,
                                           shape=2))
        assert (got == d["m"]).all()
    finally:
        ks.close()


def test_shape_argument_checks(hqc):
    """Shape B exists for single-set HQC-1 / HQC-3 launches only."""
    say("case: shape argument checks")
    d = datasets.pke(5, 4, 0x820)
    with pytest.raises(hqc.HqcError):
        hqc.decrypt_batch(5, dev(d["u"]), dev(d["v"]), dev(d["y"]), shape=2)
    with pytest.raises(hqc.HqcError):
        hqc.decrypt_batch(5, dev(d["u"]), dev(d["v"]), dev(d["y"]), shape=3)
    # shape A explicitly: the same messages
    assert (host(hqc.decrypt_batch(5, dev(d["u"]), dev(d["v"]), dev(d["y"]), shape=1)) == d["m"]).all()
