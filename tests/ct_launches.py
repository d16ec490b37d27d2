"""Calls of three input classes in a seeded random order, for the
constant-time tests (tests/test_gpu_timing.py runs this script under
rocprofv3's counter collection and reads the per-dispatch counters).

usage: python ct_launches.py decrypt|decaps PID REPS ORDER_JSON

decrypt -- one decryption launch per call (16,384 items, the library's
default launch for that size), classes:
  zero:   one fixed key, u = 0, v = codewords of random messages (the decoder
          sees no error: every syndrome is zero, Lambda = 1);
  honest: one fixed key, honest ciphertexts (decryption recovers m);
  random: fresh random keys and uniformly random (u, v) (every word is past
          the decoding radius, so Berlekamp-Massey runs at full degree).
decaps -- one KEM decapsulation per call (16,384 items, 256 keys), classes:
  honest:   honest encapsulations (the re-encryption check passes);
  tampered: the same with one bit of v flipped (rejected by the check);
  random:   uniformly random (u, v) (rejected, past the decoding radius).
Each call first copies its class's inputs into one set of buffers that
every class shares, so that the classes differ in data only, not in the
addresses the kernels read (the copies are not library kernels and are not
counted).  Writes the class name of every timed call, in call order, to
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


def library_kernel(name):
    return "hqc_" in name or "kem_" in name


def parse_profile(cc_path, kt_path, n_calls, per_call=None):
    """The library dispatches of the last n_calls calls from rocprofv3's
    counter-collection and kernel-trace CSV files: per call a list of
    (kernel name, {counter: value summed over its rows}, duration in ns).
    Every call makes the same sequence of per_call library dispatches; when
    per_call is None it is the period of the kernel-name sequence at the
    end of the run.  Earlier dispatches (class checks, other kernels) are
    left out."""
    import csv
    counters, names = {}, {}
    with open(cc_path) as f:
        for row in csv.DictReader(f):
            if library_kernel(row["Kernel_Name"]):
                i = int(row["Dispatch_Id"])
                d = counters.setdefault(i, {})
                d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
                names[i] = row["Kernel_Name"]
    ns = {}
    with open(kt_path) as f:
        for row in csv.DictReader(f):
            if library_kernel(row["Kernel_Name"]):
                ns[int(row["Dispatch_Id"])] = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
    ids = sorted(counters)
    k = per_call
    if k is None:
        k = next((kk for kk in range(1, 9) if len(ids) >= 4 * kk and
                  all(names[ids[-j - 1]] == names[ids[-j - 1 - kk]] for j in range(3 * kk))), None)
        if k is None:
            raise ValueError("no repeating dispatch sequence")
    ids = ids[-k * n_calls:]
    if len(ids) != k * n_calls or any(i not in ns for i in ids):
        raise ValueError("%d library dispatches for %d calls of %d" % (len(ids), n_calls, k))
    calls = [[(names[i], counters[i], ns[i]) for i in ids[c * k:(c + 1) * k]] for c in range(n_calls)]
    for c in calls:
        if [n for n, _, _ in c] != [n for n, _, _ in calls[0]]:
            raise ValueError("calls launch different kernels")
    return calls


def decaps_calls(pid, dev="cuda"):
    """the three decapsulation classes as calls; checks that each class is
    what it claims"""
    import torch
    from paper_2512_12904_amd import hqc, synth
    from tests import datasets

    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(dev)

    p = datasets.sizes(pid)
    n, nkeys = COUNT, 256
    d = datasets.pke(pid, nkeys, 0xC80 + pid)
    idx = np.arange(n) % nkeys
    h, s, y = T(d["h"][idx], np.int64), T(d["s"][idx], np.int64), T(d["y_keys"][idx], np.int32)
    m = T(synth.words(0xC81 + pid, (n, p["k"] // 8)).view(np.uint8), np.uint8)
    sigma = T(synth.words(0xC82 + pid, (n, p["k"] // 8)).view(np.uint8), np.uint8)
    u, v, key = hqc.kem_encaps_batch(pid, h, s, m)
    vt = v.clone()
    vt[:, 0] ^= 1
    c = {"honest": (u, v), "tampered": (u, vt),
         "random": (T(synth.words(0xC83 + pid, (n, p["nwords"])), np.int64),
                    T(synth.words(0xC84 + pid, (n, p["vwords"])), np.int64))}
    ws = torch.empty(hqc.kem_workspace_bytes(pid, n), dtype=torch.uint8, device=dev)
    out = torch.empty((n, hqc.KEM_KEY_BYTES), dtype=torch.uint8, device=dev)
    buf = tuple(torch.empty_like(a) for a in c["honest"])

    def run(name):
        # every class is decapsulated from the same buffers (only their
        # contents differ, not the addresses the kernels read)
        for b, a in zip(buf, c[name]):
            b.copy_(a)
        return hqc.kem_decaps_batch(pid, h, s, y, sigma, *buf, key_out=out, workspace=ws)

    ok = torch.equal(run("honest"), key) and not (run("tampered") == key).all(dim=1).any()
    torch.cuda.synchronize()
    return list(c), run, bool(ok)


def decrypt_calls(pid):
    import torch
    from paper_2512_12904_amd import hqc
    c, m_honest, p = classes(pid)
    out = torch.empty((COUNT, p["k"]), dtype=torch.uint8, device="cuda")
    buf = tuple(torch.empty_like(a) for a in c["honest"])

    def run(name):
        # every class is decrypted from the same buffers (only their
        # contents differ, not the addresses the kernel reads)
        for b, a in zip(buf, c[name]):
            b.copy_(a)
        return hqc.decrypt_batch(pid, *buf, out=out)

    # the honest class decrypts to its messages (the timing is of real
    # decryptions)
    run("honest")
    torch.cuda.synchronize()
    return list(c), run, bool(np.array_equal(out.cpu().numpy(), m_honest))


def main():
    mode, pid, reps, order_path = sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), sys.argv[4]
    import torch
    print("classes %s pid=%d" % (mode, pid), flush=True)
    names, run, ok = {"decrypt": decrypt_calls, "decaps": decaps_calls}[mode](pid)
    if not ok:
        print("a class is not what it claims", flush=True)
        sys.exit(3)
    order = np.random.default_rng(pid).permutation(np.repeat(np.arange(len(names)), reps))
    seq = []
    for i in order:
        run(names[i])
        seq.append(names[i])
    torch.cuda.synchronize()
    with open(order_path, "w") as f:
        json.dump(seq, f)
    print("launches done", flush=True)


if __name__ == "__main__":
    main()
