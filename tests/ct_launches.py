"""Decryption launches of three input classes in a seeded random order, for
the constant-time test (tests/test_gpu_timing.py runs this script under
rocprofv3's counter collection and reads the per-dispatch counters).

usage: python ct_launches.py PID REPS ORDER_JSON

Classes (16,384 items each, the library's default launch for that size):
  zero:   one fixed key, u = 0, v = codewords of random messages (the decoder
          sees no error: every syndrome is zero, Lambda = 1);
  honest: one fixed key, honest ciphertexts (decryption recovers m);
  random: fresh random keys and uniformly random (u, v) (every word is past
          the decoding radius, so Berlekamp-Massey runs at full degree).
Writes the class name of every decryption launch, in launch order, to
ORDER_JSON and prints 'launches done' last."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COUNT = 16384


def classes(pid, dev="cuda"):
    import torch
    import oracle
    from paper_2512_12904_amd import synth
    from tests import datasets

    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(dev)

    p = datasets.sizes(pid)
    n = COUNT
    h, x, y = synth.keys(0xC7A + pid, pid, p, 1)
    m = synth.encryptions(0xC7A + pid, pid, p, 64)[0]
    cw = np.stack([oracle.code_encode(pid, mm) for mm in m])
    c = {"zero": (torch.zeros((n, p["nwords"]), dtype=torch.int64, device=dev),
                  T(cw[np.arange(n) % 64], np.int64), T(np.repeat(y, n, axis=0), np.int32))}
    d = datasets.pke(pid, 512, 0xC7E + pid, shared_key=True)
    idx = np.arange(n) % 512
    c["honest"] = (T(d["u"][idx], np.int64), T(d["v"][idx], np.int64), T(d["y"][idx], np.int32))
    c["random"] = (T(synth.words(0xC7C + pid, (n, p["nwords"])), np.int64),
                   T(synth.words(0xC7D + pid, (n, p["vwords"])), np.int64),
                   T(synth.keys(0xC7B + pid, pid, p, n)[2], np.int32))
    return c, d["m"][idx], p


def main():
    pid, reps, order_path = int(sys.argv[1]), int(sys.argv[2]), sys.argv[3]
    import torch
    from paper_2512_12904_amd import hqc
    print("classes pid=%d" % pid, flush=True)
    c, m_honest, p = classes(pid)
    names = list(c)
    out = torch.empty((COUNT, p["k"]), dtype=torch.uint8, device="cuda")
    # the honest class decrypts to its messages (the timing is of real
    # decryptions)
    hqc.decrypt_batch(pid, *c["honest"], out=out)
    torch.cuda.synchronize()
    if not np.array_equal(out.cpu().numpy(), m_honest):
        print("honest class not recovered", flush=True)
        sys.exit(3)
    order = np.random.default_rng(pid).permutation(np.repeat(np.arange(len(names)), reps))
    seq = []
    for i in order:
        hqc.decrypt_batch(pid, *c[names[i]], out=out)
        seq.append(names[i])
    torch.cuda.synchronize()
    with open(order_path, "w") as f:
        json.dump(seq, f)
    print("launches done", flush=True)


if __name__ == "__main__":
    main()
