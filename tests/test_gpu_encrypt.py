"""GPU key generation (Alg. 3) and encryption (Alg. 1) against the CPU oracle,
bit for bit, with the same seeded randomness; and the GPU round trip
Decrypt(Encrypt(m)) = m."""
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


@pytest.mark.parametrize("pid", [1, 3, 5])
@pytest.mark.parametrize("count,grid", [(1, 0), (67, 0), (67, 5)])
def test_keygen_encrypt_match_oracle(hqc, pid, count, grid):
    print("case: keygen/encrypt pid=%d count=%d grid=%d" % (pid, count, grid), flush=True)
    p = datasets.sizes(pid)
    h, x, y = synth.keys(0x900 + pid, pid, p, count)
    x[0, 0] = x[0, 1]  # a repeated index cancels, as in the oracle
    n = p["n"]
    x[-1, 2] = n + 11  # indices are taken mod n
    y[-1, 0] = n
    s_ref = oracle.keygen_batch(pid, h, x, y)
    s_gpu = host(hqc.keygen_batch(pid, dev(h), dev(x), dev(y), grid=grid)).view(np.uint64)
    assert (s_gpu == s_ref).all()
    ko = np.arange(count, dtype=np.int64)
    m, r1, r2, e = synth.encryptions(0x900 + pid, pid, p, count, key_of=ko)
    e[-1, :3] = [0, p["n"] - 1, p["n1"] * p["n2"] - 1]  # edges of the truncation and the ring
    r1[0, :2] = [n + 5, 5]    # the same position twice (mod n): cancels
    r2[-1, 1] = r2[-1, 0]     # a repeated index of the product cancels
    e[0, 3] = n + 7           # taken mod n
    u_ref, v_ref = oracle.encrypt_batch(pid, h, s_ref, m, r1, r2, e, key_of=ko)
    u, v = hqc.encrypt_batch(pid, dev(h), dev(s_ref), dev(m), dev(r1), dev(r2), dev(e), grid=grid)
    assert (host(u).view(np.uint64) == u_ref).all()
    assert (host(v).view(np.uint64) == v_ref).all()


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_gpu_round_trip(hqc, pid):
    import torch
    print("case: GPU round trip pid=%d" % pid, flush=True)
    p = datasets.sizes(pid)
    cnt = 2048
    h, x, y = synth.keys(0xA00 + pid, pid, p, cnt)
    ko = np.arange(cnt, dtype=np.int64)
    m, r1, r2, e = synth.encryptions(0xA00 + pid, pid, p, cnt, key_of=ko)
    hd, yd = dev(h), dev(y)
    s = hqc.keygen_batch(pid, hd, dev(x), yd)
    u, v = hqc.encrypt_batch(pid, hd, s, dev(m), dev(r1), dev(r2), dev(e))
    got = hqc.decrypt_batch(pid, u, v, yd)
    torch.cuda.synchronize()
    assert torch.equal(got, dev(m))


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_code_encode_matches_oracle(hqc, pid):
    """hqc_code_encode_batch: C.Encode(m) against the oracle's concatenated
    encoder, and with a symbol-error pattern (delta symbols, the decoder
    stress construction) plus the drawn noise against the oracle's stress
    words; 200 items (a ragged tail at every grid) in two launch shapes."""
    print("case: code encode pid=%d" % pid, flush=True)
    p = datasets.sizes(pid)
    cnt = 200
    m, bad, dval, noise = synth.stress(0xE0C + pid, pid, p, cnt)
    m[0] = 0
    m[1] = 0xFF
    ref = np.stack([oracle.code_encode(pid, mm) for mm in m])
    for grid in (0, 3):
        got = host(hqc.code_encode_batch(pid, dev(m), grid=grid)).view(np.uint64)
        assert (got == ref).all(), grid
    err = np.zeros((cnt, p["n1"]), np.uint8)
    np.put_along_axis(err, bad.astype(np.int64), dval, axis=1)
    r = host(hqc.code_encode_batch(pid, dev(m), sym_err=dev(err))).view(np.uint64) ^ noise
    want = oracle.stress_batch(pid, m, bad, dval, noise)
    assert (r == want).all()
    # the stress words decode to m on the GPU
    assert (host(hqc.decode_batch(pid, dev(r))) == m).all()
