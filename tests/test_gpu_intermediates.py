"""Stage-by-stage parity through the debug entry point (hqc_decrypt_debug):
the same kernels store each item's received word v + u*y, RM symbols,
syndromes, error locator and error values, which are compared with the
oracle's component functions (product, RM decoder, syndromes,
Berlekamp-Massey, the Reed-Solomon decoder's trace), all exactly: the
decoder keeps Massey's division, so its Lambda is Massey's (Lambda_0 = 1).
Honest ciphertexts and uniformly random words (decoder failure)
are mixed; both Reed-Solomon mappings (lane pairs for tiles of at most 32,
one lane for larger tiles) are exercised."""
import numpy as np
import pytest

import oracle
from paper_2512_12904_amd import synth
from tests import datasets

pytestmark = pytest.mark.gpu



@pytest.mark.parametrize("pid,tile,grid", [(1, 32, 0), (1, 64, 0), (3, 32, 0), (3, 64, 0), (5, 32, 0),
                                           (1, 7, 2), (5, 5, 3)])
def test_intermediates_match_checker_components(pid, tile, grid):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    print("case: intermediates pid=%d tile=%d grid=%d" % (pid, tile, grid), flush=True)
    p = datasets.sizes(pid)
    par = oracle.param(pid)
    n, n1, n2, k = par["n"], par["n1"], par["n2"], par["k"]
    td = n1 - k
    mult = n2 // 128
    count = 96
    d = datasets.pke(pid, count, 0x1D0 + pid)
    u, v, y = d["u"].copy(), d["v"].copy(), d["y"]
    rnd = np.arange(count) % 3 == 2
    u[rnd] = synth.words(0x1D1 + pid, (int(rnd.sum()), p["nwords"]))
    v[rnd] = synth.words(0x1D2 + pid, (int(rnd.sum()), p["vwords"]))
    du = torch.from_numpy(u.view(np.int64)).cuda()
    dv = torch.from_numpy(v.view(np.int64)).cuda()
    dy = torch.from_numpy(y.view(np.int32)).cuda()
    m, rec = hqc.decrypt_debug(pid, du, dv, dy, tile=tile, grid=grid)
    m = m.cpu().numpy()
    # the debug kernel decrypts exactly like the plain one
    assert np.array_equal(m, hqc.decrypt_batch(pid, du, dv, dy, tile=tile).cpu().numpy())
    assert np.array_equal(m, oracle.decrypt_batch(pid, y, u, v))
    nv = n1 * n2 // 64
    for i in range(count):
        # S0-S2: received word
        prod = oracle.mul_sparse(n, u[i], y[i])
        r = v[i] ^ prod[:nv]
        assert np.array_equal(rec["r"][i], r), (i, "r")
        # S3-S5: one RM symbol per block of n2 bits
        words = n2 // 64
        sym = np.array([oracle.rm_decode(mult, r[j * words:(j + 1) * words])[0] for j in range(n1)],
                       np.uint8)
        assert np.array_equal(rec["sym"][i], sym), (i, "sym")
        # S6: syndromes
        S = oracle.rs_syndromes(n1, td, sym)
        assert np.array_equal(rec["S"][i], S), (i, "S")
        # S7: Lambda, exactly (Massey's division keeps Lambda_0 = 1)
        lam = oracle.rs_berlekamp_massey(td, S)[0]
        assert np.array_equal(rec["lam"][i], lam), (i, "lambda")
        # S8-S10: error values at the message positions
        mm, tr = oracle.rs_decode(n1, k, sym)
        assert np.array_equal(rec["e"][i], tr["err"][td:]), (i, "e")
        assert np.array_equal(m[i], mm)
