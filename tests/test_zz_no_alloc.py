"""The allocation-free decapsulation entry point (hqc_kem_decaps_batch_noalloc,
through the C ABI) against hqc_kem_decaps_batch with a caller workspace:
byte-identical keys on two calls in a row, the second with a smaller batch
(the fixed scratch keeps the first call's contents), for honest, tampered
and random ciphertexts of every parameter set; counts beyond the scratch
are refused before any launch."""
import numpy as np
import pytest

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


def _case(hqc, pid, count, master):
    """Device tensors of count decapsulation inputs: honest ciphertexts, a
    third with one bit of v flipped, a third replaced by random words."""
    import torch
    d = datasets.pke(pid, count, master)
    p = datasets.sizes(pid)
    u, v = d["u"].copy(), d["v"].copy()
    v[1::3, 0] ^= np.uint64(1)
    rnd = np.arange(count) % 3 == 2
    u[rnd] = synth.words(master + 1, (int(rnd.sum()), p["nwords"]))
    v[rnd] = synth.words(master + 2, (int(rnd.sum()), p["vwords"]))
    sigma = synth.words(master ^ 0x5157, (count, p["k"] // 8)).view(np.uint8)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    return {"h": t(d["h"], np.int64), "s": t(d["s"], np.int64), "y": t(d["y"], np.int32),
            "sigma": t(sigma, np.uint8), "u": t(u, np.int64), "v": t(v, np.int64)}


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_noalloc_decaps_equals_workspace_decaps(hqc, pid):
    import torch
    for count, master in ((150, 0xA110 + pid), (37, 0xA120 + pid)):
        print("case: noalloc decaps pid=%d count=%d" % (pid, count), flush=True)
        c = _case(hqc, pid, count, master)
        args = (c["h"], c["s"], c["y"], c["sigma"], c["u"], c["v"])
        want = hqc.kem_decaps_batch(pid, *args)
        got = torch.empty_like(want)
        hqc.kem_decaps_batch_noalloc(pid, *args, key_out=got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (pid, count)


def test_noalloc_count_limit(hqc):
    """One item more than the scratch holds is refused (HQC_ERANGE), nothing
    written; the largest count that fits is accepted."""
    import torch
    pid = 1
    sz = hqc.sizes(pid)
    L = hqc.lib()
    limit = 0
    while L.hqc_kem_workspace_bytes(pid, limit + 1) <= hqc.NOALLOC_SCRATCH_BYTES:
        limit += 1024
    while L.hqc_kem_workspace_bytes(pid, limit) > hqc.NOALLOC_SCRATCH_BYTES:
        limit -= 1
    print("case: noalloc count limit pid=%d limit=%d" % (pid, limit), flush=True)
    n = limit + 1
    z = lambda *shape, dt=torch.int64: torch.zeros(shape, dtype=dt, device="cuda")
    h, s, u = z(n, sz["u_words"]), z(n, sz["u_words"]), z(n, sz["u_words"])
    v = z(n, sz["v_words"])
    y = torch.arange(sz["w"], dtype=torch.int32, device="cuda").repeat(n, 1)
    sigma = z(n, sz["k"], dt=torch.uint8)
    key = torch.full((n, 32), 0xAB, dtype=torch.uint8, device="cuda")
    with pytest.raises(hqc.HqcError) as ei:
        hqc.kem_decaps_batch_noalloc(pid, h, s, y, sigma, u, v, key)
    assert ei.value.code == hqc.HQC_ERANGE
    torch.cuda.synchronize()
    assert bool((key == 0xAB).all())
    # exactly at the limit: accepted, keys equal the workspace call's
    args = (h[:limit], s[:limit], y[:limit], sigma[:limit], u[:limit], v[:limit])
    hqc.kem_decaps_batch_noalloc(pid, *args, key_out=key[:limit])
    want = hqc.kem_decaps_batch(pid, *args)
    torch.cuda.synchronize()
    assert torch.equal(key[:limit], want)
