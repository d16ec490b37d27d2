"""Serving loop: every request's messages are the same when served alone and
inside the continuous-batching mix (integer work: tolerance zero), also when
the memory budget forces requests to be split across batches; each batch is
one keyed launch over every parameter set it holds, and the server's own
check of every served message against the pool's messages agrees."""
import numpy as np
import pytest

import oracle
from paper_2512_12904_amd import synth
from tests import datasets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    hqc.lib()
    nkeys = {1: 5, 3: 4, 5: 3}
    per_key = 40
    ks = hqc.KeyStore(nkeys[1], nkeys[3], nkeys[5])
    pools, truth = {}, {}
    for pid in (1, 3, 5):
        p = datasets.sizes(pid)
        h, x, y = synth.keys(0x77, pid, p, nkeys[pid])
        s = oracle.keygen_batch(pid, h, x, y)
        key_of = np.repeat(np.arange(nkeys[pid]), per_key).astype(np.int64)
        m, r1, r2, e = synth.encryptions(0x77, pid, p, len(key_of), key_of=key_of)
        u, v = oracle.encrypt_batch(pid, h, s, m, r1, r2, e, key_of=key_of)
        ks.put(pid, 0, y)
        pools[pid] = {"u": torch.from_numpy(u.view(np.int64)).pin_memory(),
                      "v": torch.from_numpy(v.view(np.int64)).pin_memory(),
                      "key": torch.from_numpy(key_of.astype(np.int32)).pin_memory(),
                      "m": m}
        truth[pid] = m
    return hqc, ks, pools, truth, nkeys, per_key


def make_requests(nkeys, per_key, n, seed, spacing):
    from paper_2512_12904_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        pid = (1, 3, 5)[int(rng.integers(0, 3))]
        key = int(rng.integers(0, nkeys[pid]))
        off = int(rng.integers(0, per_key))
        b = int(rng.integers(1, per_key - off + 1))
        reqs.append(Request(i, pid, key, b, i * spacing, key * per_key + off))
    return reqs


@pytest.mark.parametrize("budget,streams,realtime", [(256 << 10, 3, False), (64 << 20, 4, True)])
def test_alone_equals_mixed(env, budget, streams, realtime):
    import torch
    hqc, ks, pools, truth, nkeys, per_key = env
    from paper_2512_12904_amd.serve import Server
    print("case: serving budget=%d streams=%d realtime=%s" % (budget, streams, realtime), flush=True)
    reqs = make_requests(nkeys, per_key, 60, 5, 2e-4 if realtime else 0.0)
    srv = Server(ks, pools, streams=streams, budget_bytes=budget)
    srv.run(reqs, keep_results=True, realtime=realtime)
    assert srv.checked == sum(r.b for r in reqs) and srv.mismatches == 0
    for r in reqs:
        want = truth[r.pid][r.src:r.src + r.b]
        assert r.t_done is not None and r.t_done >= r.arrival
        assert (r.m == want).all(), r.rid
        # the same request alone, one keyed launch
        pool = pools[r.pid]
        kid = torch.full((r.b,), r.key, dtype=torch.int32, device="cuda")
        assert (pool["key"][r.src:r.src + r.b] == r.key).all()
        alone = hqc.decrypt_batch_keyed(r.pid, ks, pool["u"][r.src:r.src + r.b].cuda(),
                                        pool["v"][r.src:r.src + r.b].cuda(), kid)
        torch.cuda.synchronize()
        assert (alone.cpu().numpy() == r.m).all()
