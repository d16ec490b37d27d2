"""Determinism of the decryption launch: repeated launches give identical
messages, a permuted batch gives the permuted messages, and every launch
configuration (kernel shape, tile, grid, graph or direct, tuned table
entry) gives the same bytes.  Honest ciphertexts and uniformly random words (decoder
failure, where the output is fixed only by the conventions) are mixed."""
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


def _batch(pid, count):
    p = datasets.sizes(pid)
    d = datasets.pke(pid, count, 0xD0 + pid)
    u, v, y = d["u"].copy(), d["v"].copy(), d["y"].copy()
    # every third item: uniformly random words under the same key
    rnd = np.arange(count) % 3 == 2
    u[rnd] = synth.words(0xD1 + pid, (int(rnd.sum()), p["nwords"]))
    v[rnd] = synth.words(0xD2 + pid, (int(rnd.sum()), p["vwords"]))
    return u, v, y


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_repeat_permute_and_configurations(hqc, pid):
    import torch
    print("case: determinism pid=%d" % pid, flush=True)
    count = 1500
    u, v, y = _batch(pid, count)
    du, dv, dy = (torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()
                  for a in (u, v, y))
    ref = hqc.decrypt_batch(pid, du, dv, dy).cpu().numpy()
    assert np.array_equal(ref, oracle.decrypt_batch(pid, y, u, v))
    for _ in range(3):
        assert np.array_equal(hqc.decrypt_batch(pid, du, dv, dy).cpu().numpy(), ref)
    perm = np.random.default_rng(pid).permutation(count)
    pt = torch.from_numpy(perm).cuda()
    got = hqc.decrypt_batch(pid, du[pt].contiguous(), dv[pt].contiguous(), dy[pt].contiguous())
    assert np.array_equal(got.cpu().numpy(), ref[perm])
    shapes = (1, 2) if pid != 5 else (1,)
    for shape in shapes:
        for tile, grid, flags in [(1, 0, 0), (5, 37, 0), (32, 0, hqc.F_GRAPH), (33, 0, 0),
                                  (64, 11, 0), (0, 3, hqc.F_GRAPH)]:
            got = hqc.decrypt_batch(pid, du, dv, dy, tile=tile, grid=grid, flags=flags, shape=shape)
            assert np.array_equal(got.cpu().numpy(), ref), (tile, grid, flags, shape)
    hqc.tune_clear()
    try:
        for shape in shapes:
            hqc.tune_set(pid, count, 16, 50, shape)  # a table entry for this batch size
            assert np.array_equal(hqc.decrypt_batch(pid, du, dv, dy).cpu().numpy(), ref), shape
    finally:
        hqc.tune_clear()
