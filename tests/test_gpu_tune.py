"""The autotuner on the GPU: every candidate configuration gives the same
messages, the chosen one lands in the table and is used by default launches,
and decryption under it still matches the checker."""
import numpy as np
import pytest

from tests import datasets

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_autotune_then_default_launch_matches_checker(pid):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    print("case: autotune pid=%d" % pid, flush=True)
    hqc.tune_clear()
    count = 4096
    r = hqc.autotune_decrypt(pid, count, reps=2)
    assert r["identical"] == 1 and r["count"] == count and r["candidates"] >= 1
    assert 1 <= r["tile"] <= 64 and r["grid"] >= 1
    assert r["shape"] in ((1, 2) if pid != 5 else (1,)) and r["heuristic_shape"] in (1, 2)
    assert r["ms"] <= r["heuristic_ms"] + 1e-6
    assert hqc.tune_get(pid, count) == (r["tile"], r["grid"], r["shape"])
    # the launch a default call makes is the tuned entry's; explicit knobs win
    assert hqc.launch_config(pid, count) == (r["shape"], r["tile"], min(r["grid"],
                                                                        -(-count // r["tile"])))
    assert hqc.launch_config(pid, count, grid=64, tile=8, shape=1) == (1, 8, 64)
    d = datasets.pke(pid, count, 0x7A0 + pid)
    dev = "cuda"
    u = torch.from_numpy(d["u"].view(np.int64)).to(dev)
    v = torch.from_numpy(d["v"].view(np.int64)).to(dev)
    y = torch.from_numpy(d["y"].view(np.int32)).to(dev)
    got = hqc.decrypt_batch(pid, u, v, y)  # grid = tile = 0: the tuned entry
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), d["m"])
    hqc.tune_clear()


def test_autotune_rejects_bad_arguments():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    for args in [(2, 100, 2), (1, 0, 2), (1, 100, 0)]:
        with pytest.raises(hqc.HqcError):
            hqc.autotune_decrypt(*args)
    with pytest.raises(hqc.HqcError):
        hqc.autotune_decrypt(1, (1 << 20) + 1, 1)


def test_builtin_launch_config():
    """Without a table entry: single-set decryption with every knob open
    takes the built-in table's choice (a valid launch: shape B only where it
    exists, tile 1 .. 64, grid at most the tiles); with the shape given, the
    occupancy grid of that shape and the largest power-of-two tile not above
    count / grid (at most 64)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    hqc.tune_clear()
    for pid in (1, 3, 5):
        shapes = (1, 2) if pid != 5 else (1,)
        full = {sh: hqc.launch_config(pid, 1 << 20, shape=sh)[2] for sh in shapes}
        for count in (1, 100, 4096, 16384, 65536, 262144, 1 << 20):
            sh, t, g = hqc.launch_config(pid, count)
            assert sh in shapes and 1 <= t <= 64 and 1 <= g <= min(full[sh], -(-count // t)), \
                (pid, count, sh, t, g)
            for want_sh in shapes:
                sh, t, g = hqc.launch_config(pid, count, shape=want_sh)
                want_t = 1
                while want_t < 64 and 2 * want_t <= count // full[want_sh]:
                    want_t *= 2
                assert (sh, t, g) == (want_sh, want_t, min(full[want_sh], -(-count // want_t))), \
                    (pid, count, want_sh)
    with pytest.raises(hqc.HqcError):
        hqc.launch_config(5, 100, shape=2)
    with pytest.raises(hqc.HqcError):
        hqc.launch_config(1, 0)
