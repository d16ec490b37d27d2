"""Default launches at every batch-size bucket of the built-in launch table
(power-of-two buckets from 2^8 items, the sizes just above and below a
boundary, and sizes under 2^8): each decrypts honest ciphertexts to the
encrypted messages, plain and through a cached graph.  The ciphertexts come
from the library's key generation and encryption, which the encryption
tests compare with the oracle."""
import numpy as np
import pytest

from paper_2512_12904_amd import synth
from tests import datasets

pytestmark = pytest.mark.gpu

SIZES = [1, 7, 200, 256, 257, 511, 512, 1024, 2048, 2049, 4096, 8192, 16384, 32768]


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_default_launches_at_every_bucket_recover_messages(pid):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    hqc.tune_clear()
    count = max(SIZES)
    print("case: launch table pid=%d up to %d items" % (pid, count), flush=True)
    s = datasets.sizes(pid)
    h, x, y = synth.keys(0x7AB + pid, pid, s, count)
    m, r1, r2, e = synth.encryptions(0x7AB + pid, pid, s, count, key_of=np.arange(count))

    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()

    hd, yd, md = T(h, np.int64), T(y, np.int32), T(m, np.uint8)
    sd = hqc.keygen_batch(pid, hd, T(x, np.int32), yd)
    u, v = hqc.encrypt_batch(pid, hd, sd, md, T(r1, np.int32), T(r2, np.int32), T(e, np.int32))
    torch.cuda.synchronize()
    for c in SIZES:
        sh, tile, grid = hqc.launch_config(pid, c)
        assert sh in ((1, 2) if pid != 5 else (1,)) and 1 <= tile <= 64
        assert 1 <= grid <= -(-c // tile), (c, sh, tile, grid)
        for flags in (0, hqc.F_GRAPH):
            out = hqc.decrypt_batch(pid, u[:c], v[:c], yd[:c], flags=flags)
            torch.cuda.synchronize()
            assert torch.equal(out, md[:c]), (pid, c, flags, (sh, tile, grid))
