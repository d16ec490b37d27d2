"""GPU adaptive ring multiplication (hqc_ring_mul_batch) against the CPU
oracle, bit-exact, on both paths: operands of HQC weight and dense ones,
items of both paths mixed in one launch, and chunked dense processing."""
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
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a


def say(*a):
    print(*a, flush=True)


def operands(pid, count, seed, weights):
    """a rows: row i has weight weights[i % len] (None = uniform dense), b dense"""
    p = datasets.sizes(pid)
    n, U = p["n"], p["nwords"]
    a = synth.words(seed, (count, U))
    b = synth.words(seed + 1, (count, U))
    for i in range(count):
        w = weights[i % len(weights)]
        if w is not None:
            row = np.zeros(64 * U, np.uint8)
            row[synth.fixed_weight(seed * 1000 + i, n, w)] = 1
            a[i] = np.packbits(row, bitorder="little").view(np.uint64)
    # bits >= n set in some rows: ignored
    a[::3, -1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(n % 64)
    b[1::3, -1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(n % 64)
    return a, b, n


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_mixed_paths_match_oracle(hqc, pid):
    say("case: ring mixed pid=%d" % pid)
    a, b, n = operands(pid, 12, 0x7100 + pid, [66, None, 0, 1, 4096, 4097])
    thr = 3000
    out, path = hqc.ring_mul_batch(pid, dev(a), dev(b), threshold=thr)
    got, gp = host(out), host(path)
    for i in range(len(a)):
        ref, rp = oracle.ring_mul(n, a[i], b[i], thr)
        assert gp[i] == rp, i
        assert (got[i] == ref).all(), i


@pytest.mark.parametrize("pid", [1, 5])
@pytest.mark.parametrize("thr", [0xFFFFFFFF, 0])
def test_forced_paths_and_chunks(hqc, pid, thr):
    # threshold 0: every nonzero a dense (processed 3 items at a time);
    # threshold max: sparse unless the weight exceeds the sparse-list capacity
    import torch
    say("case: ring forced thr=%d pid=%d" % (thr, pid))
    a, b, n = operands(pid, 7, 0x7200 + pid, [75, 149, 2000, None])
    ws = torch.empty(hqc.ring_workspace_bytes(pid, 7, 3), dtype=torch.uint8, device="cuda")
    out, path = hqc.ring_mul_batch(pid, dev(a), dev(b), threshold=thr, workspace=ws)
    got, gp = host(out), host(path)
    for i in range(len(a)):
        ref, rp = oracle.ring_mul(n, a[i], b[i], min(thr, 4096))
        assert gp[i] == rp and (got[i] == ref).all(), i


def test_default_thresholds(hqc):
    for pid in (1, 3, 5):
        t = hqc.ring_default_threshold(pid)
        # far above the HQC weights: the sparse path for every PKE operand
        assert datasets.sizes(pid)["we"] < t <= hqc.RING_SPARSE_MAX
