"""Parity at the workload sizes, in the launch configuration bench.py times
(default persistent grid, hipGraph launch):

- 65,536 HQC-1 decryptions with independent keys, one launch;
- 65,536 HQC-3 and 65,536 HQC-5 decryptions, one launch each;
- 1,048,576 decoder stress words, 50/30/20 HQC-1/3/5, one mixed launch:
  exactly delta RS symbol errors per word (duplicated RM codewords added to
  delta blocks) plus noise within the RM radius elsewhere;
- 65,536 HQC-1 and 65,536 HQC-5 key generations, encryptions and KEM
  encapsulations / decapsulations.

Every output is compared with the message that was encrypted / encoded
(ground truth); a sample is also decrypted by the CPU oracle.
"""
import numpy as np
import pytest

import oracle
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


# launch configurations: the library's default (its built-in table at this
# size, which bench.py times: HQC-1 and HQC-3 shape B, tiles of 16, 3,072
# workgroups; HQC-5 shape A, tiles of 16, 2,048) and another (HQC-1 and
# HQC-3: shape A with 32-item tiles; HQC-5: tiles of one item)
@pytest.mark.parametrize("pid,master,launch", [(1, 0x2, None), (1, 0x2, (1, 32, 3072)),
                                               (3, 0x3, None), (3, 0x3, (1, 32, 2048)),
                                               (5, 0x5, None), (5, 0x5, (1, 1, 2048))])
def test_decrypt_65536_one_launch(hqc, pid, master, launch):
    import torch
    count = 65536
    print("case: full-size decrypt pid=%d count=%d launch=%s" % (pid, count, launch), flush=True)
    d = datasets.pke(pid, count, master)
    print("  generated", flush=True)
    shape, tile, grid = launch or (0, 0, 0)
    out = hqc.decrypt_batch(pid, dev(d["u"]), dev(d["v"]), dev(d["y"]), flags=hqc.F_GRAPH,
                            shape=shape, tile=tile, grid=grid)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    bad = np.flatnonzero((got != d["m"]).any(1))
    assert len(bad) == 0, "items differing from the encrypted message: %s" % bad[:10]
    rng = np.random.default_rng(pid)
    sample = np.sort(rng.choice(count, 512, replace=False))
    ref = oracle.decrypt_batch(pid, d["y"][sample], d["u"][sample], d["v"][sample])
    assert (got[sample] == ref).all()


def test_decode_stress_1m_mixed_one_launch(hqc):
    import torch
    counts = {1: 524288, 3: 314573, 5: 209715}  # 50 / 30 / 20 of 1,048,576
    assert sum(counts.values()) == 1 << 20
    print("case: stress 1M mixed", flush=True)
    data = {pid: datasets.stress(pid, c, 0x4) for pid, c in counts.items()}
    print("  generated", flush=True)
    items = [{"pid": pid, "r": dev(d["r"])} for pid, d in data.items()]
    outs = hqc.decode_mixed(items, flags=hqc.F_GRAPH)
    torch.cuda.synchronize()
    for (pid, d), o in zip(data.items(), outs):
        got = o.cpu().numpy()
        bad = np.flatnonzero((got != d["m"]).any(1))
        assert len(bad) == 0, "pid %d: %d words wrong, first %s" % (pid, len(bad), bad[:10])
    # the same words in separate homogeneous launches give the same bytes
    for it, o in zip(items, outs):
        sep = hqc.decode_batch(it["pid"], it["r"][:4096])
        torch.cuda.synchronize()
        assert torch.equal(sep, o[:4096])
    # oracle on a sample of each set
    for pid, d in data.items():
        ref = oracle.decode_batch(pid, d["r"][:256])
        assert (outs[[1, 3, 5].index(pid)][:256].cpu().numpy() == ref).all()


@pytest.mark.parametrize("pid", [1, 5])
def test_keygen_encrypt_kem_65536(hqc, pid):
    """Key generation, encryption and the KEM at 65,536 items with the
    default persistent grid (the configuration bench.py times): sampled items
    against the oracle, every item through the GPU round trips."""
    import torch
    from paper_2512_12904_amd import synth
    print("case: keygen/encrypt/KEM 65536 pid=%d" % pid, flush=True)
    count = 65536
    p = datasets.sizes(pid)
    h, x, y = synth.keys(0x6E00 + pid, pid, p, count)
    ko = np.arange(count, dtype=np.int64)
    m, r1, r2, e = synth.encryptions(0x6E00 + pid, pid, p, count, key_of=ko)
    sigma = synth.words(0x6E10 + pid, (count, p["k"] // 8)).view(np.uint8)
    hd, yd, md = dev(h), dev(y), dev(m)
    s = hqc.keygen_batch(pid, hd, dev(x), yd)
    u, v = hqc.encrypt_batch(pid, hd, s, md, dev(r1), dev(r2), dev(e))
    got = hqc.decrypt_batch(pid, u, v, yd, flags=hqc.F_GRAPH)
    ku, kv, key = hqc.kem_encaps_batch(pid, hd, s, md)
    key2 = hqc.kem_decaps_batch(pid, hd, s, yd, dev(sigma), ku, kv)
    torch.cuda.synchronize()
    assert torch.equal(got, md)
    assert torch.equal(key, key2)
    rng = np.random.default_rng(pid)
    idx = np.unique(np.concatenate([[0, 1, 2047, 2048, count // 2, count - 1],
                                    rng.choice(count, 26, replace=False)]))
    s_h = s.cpu().numpy().view(np.uint64)
    assert (s_h[idx] == oracle.keygen_batch(pid, h[idx], x[idx], y[idx])).all()
    u_ref, v_ref = oracle.encrypt_batch(pid, h[idx], s_h[idx], m[idx], r1[idx], r2[idx], e[idx])
    assert (u.cpu().numpy().view(np.uint64)[idx] == u_ref).all()
    assert (v.cpu().numpy().view(np.uint64)[idx] == v_ref).all()
    ru, rv, rkey = oracle.kem_encaps_batch(pid, h[idx], s_h[idx], m[idx])
    assert (ku.cpu().numpy().view(np.uint64)[idx] == ru).all()
    assert (kv.cpu().numpy().view(np.uint64)[idx] == rv).all()
    assert (key.cpu().numpy()[idx] == rkey).all()
