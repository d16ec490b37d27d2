"""GPU KEM (hqc_kem_encaps_batch / hqc_kem_decaps_batch) against the CPU
oracle, bit-exact: ciphertexts and keys of encapsulation, keys of
decapsulation for honest and for rejected ciphertexts."""
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
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a


def say(*a):
    print(*a, flush=True)


def kem_data(pid, count, master):
    d = datasets.pke(pid, count, master)
    p = datasets.sizes(pid)
    d["sigma"] = synth.words(master ^ 0x5157, (count, p["k"] // 8)).view(np.uint8)
    return d


@pytest.mark.parametrize("pid", [1, 3, 5])
@pytest.mark.parametrize("count", [1, 65])
def test_encaps_matches_oracle(hqc, pid, count):
    say("case: encaps pid=%d count=%d" % (pid, count))
    d = kem_data(pid, count, 0xD00 + pid + count)
    u, v, key = hqc.kem_encaps_batch(pid, dev(d["h"]), dev(d["s"]), dev(d["m"]))
    ru, rv, rkey = oracle.kem_encaps_batch(pid, d["h"], d["s"], d["m"])
    assert (host(u) == ru).all() and (host(v) == rv).all()
    assert (host(key) == rkey).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decaps_honest_and_rejected(hqc, pid):
    say("case: decaps pid=%d" % pid)
    count = 70
    d = kem_data(pid, count, 0xE00 + pid)
    u, v, key = oracle.kem_encaps_batch(pid, d["h"], d["s"], d["m"])
    u, v = u.copy(), v.copy()
    p = datasets.sizes(pid)
    # rows 0..7 tampered in different ways; the rest honest
    u[0, 5] ^= np.uint64(1)
    v[1, -1] ^= np.uint64(1) << np.uint64(63)
    u[2, -1] ^= np.uint64(1) << np.uint64(63)          # a padding bit of u (>= n)
    v[3] = synth.words(0xE10, (p["vwords"],))           # v replaced
    u[4] = synth.words(0xE11, (p["nwords"],))           # u replaced
    u[5], v[5] = u[8], v[8]                              # another key's ciphertext
    v[6, 10] ^= np.uint64(0xFFFF)                        # many bits of one block
    u[7], v[7] = 0, 0                                    # the zero ciphertext
    got = hqc.kem_decaps_batch(pid, dev(d["h"]), dev(d["s"]), dev(d["y_keys"]),
                               dev(d["sigma"]), dev(u), dev(v))
    ref, ok = oracle.kem_decaps_batch(pid, d["h"], d["s"], d["y_keys"], d["sigma"], u, v)
    assert not ok[:8].any() and ok[8:].all()
    assert (host(got) == ref).all()
    assert (host(got)[8:] == key[8:]).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_gpu_round_trip_many(hqc, pid):
    # GPU keygen + encaps + decaps over a few thousand items with a small
    # persistent grid; sampled items against the oracle
    import torch
    say("case: KEM round trip pid=%d" % pid)
    count = 3000
    p = datasets.sizes(pid)
    h, x, y = synth.keys(0xF00 + pid, pid, p, count)
    m = synth.encryptions(0xF00 + pid, pid, p, count)[0]
    sigma = synth.words(0xF10 + pid, (count, p["k"] // 8)).view(np.uint8)
    hd, yd = dev(h), dev(y)
    s = hqc.keygen_batch(pid, hd, dev(x), yd)
    u, v, key = hqc.kem_encaps_batch(pid, hd, s, dev(m), grid=97)
    key2 = hqc.kem_decaps_batch(pid, hd, s, yd, dev(sigma), u, v, grid=97)
    torch.cuda.synchronize()
    assert torch.equal(key, key2)
    idx = np.array([0, 1, count // 2, count - 1])
    ru, rv, rkey = oracle.kem_encaps_batch(pid, h[idx], host(s)[idx], m[idx])
    assert (host(key)[idx] == rkey).all() and (host(u)[idx] == ru).all()


def test_workspace_too_small_is_rejected(hqc):
    import torch
    say("case: KEM workspace size")
    pid = 1
    d = kem_data(pid, 4, 0xF80)
    need = hqc.kem_workspace_bytes(pid, 4)
    ws = torch.empty(need - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        hqc.kem_encaps_batch(pid, dev(d["h"]), dev(d["s"]), dev(d["m"]), workspace=ws)
    # through the C ABI directly: a short workspace_bytes is refused
    import ctypes
    big = torch.empty(need, dtype=torch.uint8, device="cuda")
    u = torch.empty((4, datasets.sizes(pid)["nwords"]), dtype=torch.int64, device="cuda")
    v = torch.empty((4, datasets.sizes(pid)["vwords"]), dtype=torch.int64, device="cuda")
    key = torch.empty((4, 32), dtype=torch.uint8, device="cuda")
    prm = hqc.Params(pid, 0, None, 0, 0)
    vp = ctypes.c_void_p
    hd, sd, md = dev(d["h"]), dev(d["s"]), dev(d["m"])
    rc = hqc.lib().hqc_kem_encaps_batch(
        ctypes.byref(prm), vp(hd.data_ptr()), vp(sd.data_ptr()), vp(md.data_ptr()),
        vp(u.data_ptr()), vp(v.data_ptr()), vp(key.data_ptr()), vp(big.data_ptr()), need - 1, 4)
    assert rc == hqc.HQC_EINVAL


def _draw_for(n, i, t):
    # the smallest 32-bit draw with i + floor(a (n - i) / 2^32) = i + t
    return -(-(t << 32) // (n - i))


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_fixed_weight_sampling_edge_draws(hqc, pid):
    # crafted draws: no collision, every draw maximal (a chain of collisions),
    # a position equal to the index of a replaced later position, random, and
    # two rows of dense collisions
    say("case: Floyd sampling pid=%d" % pid)
    p = datasets.sizes(pid)
    n, wr, we = p["n"], p["wr"], p["we"]
    nd = 2 * wr + we
    rows = [np.zeros(nd, np.uint32), np.full(nd, 0xFFFFFFFF, np.uint32)]
    r = np.zeros(nd, np.uint32)
    for off, w in ((0, wr), (wr, wr), (2 * wr, we)):
        P = w + 107
        t = {w - 1: P - (w - 1), w - 2: P - (w - 2)}   # p = P twice: w-2 is replaced
        t[3] = (w - 2) - 3                             # p_3 = w - 2: hits the replaced index
        t[1] = (w - 1) - 1                             # p_1 = w - 1: index of a kept position
        for i in range(w):
            r[off + i] = _draw_for(n, i, t.get(i, 0) if i in t else 50 + 3 * i)
    rows.append(r)
    rows.append(synth.words(0x7E57 + pid, (nd + 1) // 2).view(np.uint32)[:nd])
    # dense collisions: p_i within i .. i + 2, and p_i anywhere in i .. w - 1
    # (positions that are indices of earlier-replaced entries: long chains)
    rng = np.random.default_rng(0xF10 + pid)
    for span in (3, None):
        r = np.zeros(nd, np.uint32)
        for off, w in ((0, wr), (wr, wr), (2 * wr, we)):
            for i in range(w):
                t = int(rng.integers(0, span if span else w - i))
                r[off + i] = _draw_for(n, i, t)
        rows.append(r)
    draws = np.stack(rows)
    import torch
    out = hqc.fixed_weight_batch(pid, dev(draws))
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    for k, d in enumerate(draws):
        ref = np.concatenate([oracle.fixed_weight(n, wr, d[:wr]), oracle.fixed_weight(n, wr, d[wr:2 * wr]),
                              oracle.fixed_weight(n, we, d[2 * wr:])])
        assert (got[k] == ref).all(), k
