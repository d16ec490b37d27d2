"""Timing checks of decryption and decapsulation against their input data,
in the style of dudect (Reparaz, Balasch, Verbauwhede, "Dude, is my code
constant time?", 2017): measurements of input classes launched interleaved
in a seeded random order, compared by Welch's t.

Decryption (tests/ct_launches.py, run under rocprofv3's counter
collection): classes zero (u = 0, v = codewords: no error at all), honest
(honest ciphertexts under one key) and random (random keys, uniform u and
v: every word past the decoding radius).  Every dispatch must execute the
same instructions (VALU, SALU, LDS) with the same LDS bank conflicts, and
the kernel's duration in shader-clock cycles (SQ_BUSY_CYCLES) must pass
dudect's test, |t| < 4.5, between honest and random and between zero and
random.  Cycles, not wall time: the chip runs its clock faster on data that
switches fewer bits (measured: all-zero data 2-4 % shorter launches at equal
cycle counts, honest data up to about 1 %), which a t statistic over wall
time flags at any launch size given enough launches, though no instruction
differs.  The wall times of the same dispatches are held to bounds on the
relative difference of the means (2 % honest, 5 % zero): a control-flow
shortcut (an early exit on zero syndromes, a degree-dependent loop) would
move cycles and wall time by more than that."""
import csv
import glob
import json
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from paper_2512_12904_amd import synth
from tests import datasets

pytestmark = pytest.mark.gpu

# dudect's threshold on Welch's t between two classes
T_BOUND = 4.5
# bounds on |mean(class) / mean(reference class) - 1| of wall times
# (measured: up to about 1 % honest and 2-4 % all-zero, at equal cycles)
HONEST_BOUND = 0.02
ZERO_BOUND = 0.05
# counters that must be equal in every dispatch, and the cycle counter
SAME = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT"]
CYCLES = "SQ_BUSY_CYCLES"
REPS = 40


def welch_t(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return (a.mean() - b.mean()) / np.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))


def cropped(x, frac=0.95):
    """the fastest 95 % of a class's measurements (interrupts, clock steps
    and profiler stalls removed), as dudect crops"""
    x = np.sort(np.asarray(x, float))
    return x[:max(2, int(frac * len(x)))]


def profile_classes(pid, tmp):
    """run tests/ct_launches.py under rocprofv3; returns (order, counters per
    dispatch, duration in ns per dispatch) of the decryption launches"""
    exe = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(exe):
        pytest.skip("rocprofv3 not installed")
    helper = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ct_launches.py")
    order_path = os.path.join(tmp, "order.json")
    cmd = [exe, "--kernel-trace", "--pmc", *SAME, CYCLES, "--output-format", "csv",
           "-d", os.path.join(tmp, "prof"), "-o", "c", "--",
           sys.executable, "-u", helper, str(pid), str(REPS), order_path]
    print("case: constant time pid=%d: %s" % (pid, " ".join(cmd)), flush=True)
    r = subprocess.run(cmd, cwd=tmp, env=dict(os.environ, TMPDIR="/tmp"), capture_output=True,
                       text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    # the profiler may end with a signal of its own after the program's
    # last line: the results are used when the program finished
    assert "launches done" in r.stdout and os.path.exists(order_path), tail
    order = json.load(open(order_path))
    cc = glob.glob(os.path.join(tmp, "prof", "**", "c_counter_collection.csv"), recursive=True)
    kt = glob.glob(os.path.join(tmp, "prof", "**", "c_kernel_trace.csv"), recursive=True)
    assert len(cc) == 1 and len(kt) == 1, (cc, kt, tail)
    counters = {}
    for row in csv.DictReader(open(cc[0])):
        if "hqc_kernel" in row["Kernel_Name"]:
            d = counters.setdefault(int(row["Dispatch_Id"]), {})
            d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    ns = {}
    for row in csv.DictReader(open(kt[0])):
        if "hqc_kernel" in row["Kernel_Name"]:
            ns[int(row["Dispatch_Id"])] = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
    # the last len(order) decryption dispatches are the interleaved launches
    # (the first one checks the honest messages)
    ids = sorted(counters)[-len(order):]
    assert len(ids) == len(order) and all(i in ns for i in ids), (len(ids), len(order))
    return order, [counters[i] for i in ids], [ns[i] for i in ids]


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decrypt_time_independent_of_data(pid, tmp_path):
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    order, cnt, ns = profile_classes(pid, str(tmp_path))
    names = ["zero", "honest", "random"]
    assert sorted(set(order)) == sorted(names) and len(order) == 3 * REPS
    # the same instructions and LDS bank conflicts in every dispatch
    for k in SAME:
        vals = {c[k] for c in cnt}
        assert len(vals) == 1, (k, sorted(vals)[:4])
    cyc = {n: cropped([c[CYCLES] for c, o in zip(cnt, order) if o == n]) for n in names}
    wall = {n: cropped([t for t, o in zip(ns, order) if o == n]) for n in names}
    for n in names:
        print("pid %d %-6s cycles %.0f (t vs random %.2f)  wall %.4f ms (t vs random %.2f, %+.2f %%)" % (
            pid, n, cyc[n].mean(), welch_t(cyc[n], cyc["random"]), wall[n].mean() / 1e6,
            welch_t(wall[n], wall["random"]), 100 * (wall[n].mean() / wall["random"].mean() - 1)),
            flush=True)
    assert abs(welch_t(cyc["honest"], cyc["random"])) < T_BOUND
    assert abs(welch_t(cyc["zero"], cyc["random"])) < T_BOUND
    rel = {n: wall[n].mean() / wall["random"].mean() - 1.0 for n in names}
    assert abs(rel["honest"]) < HONEST_BOUND, rel
    assert abs(rel["zero"]) < ZERO_BOUND, rel


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decaps_time_independent_of_rejection(pid):
    """Implicit rejection must not show in the time: decapsulation of honest
    ciphertexts, of ciphertexts with one bit of v flipped (rejected by the
    re-encryption check) and of uniformly random ciphertexts (rejected, and
    past the decoding radius) run the same kernels with the same launch
    shapes; the selection of m' or sigma is a per-item select."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12904_amd import hqc
    print("case: constant-time decapsulation pid=%d" % pid, flush=True)
    p = datasets.sizes(pid)
    count, nkeys = 16384, 256
    dev = "cuda"

    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(dev)

    d = datasets.pke(pid, nkeys, 0xC80 + pid)
    idx = np.arange(count) % nkeys
    h, s, y = T(d["h"][idx], np.int64), T(d["s"][idx], np.int64), T(d["y_keys"][idx], np.int32)
    m = T(synth.words(0xC81 + pid, (count, p["k"] // 8)).view(np.uint8), np.uint8)
    sigma = T(synth.words(0xC82 + pid, (count, p["k"] // 8)).view(np.uint8), np.uint8)
    u, v, key = hqc.kem_encaps_batch(pid, h, s, m)
    vt = v.clone()
    vt[:, 0] ^= 1
    classes = {
        "honest": (u, v),
        "tampered": (u, vt),
        "random": (T(synth.words(0xC83 + pid, (count, p["nwords"])), np.int64),
                   T(synth.words(0xC84 + pid, (count, p["vwords"])), np.int64)),
    }
    names = list(classes)
    ws = torch.empty(hqc.kem_workspace_bytes(pid, count), dtype=torch.uint8, device=dev)
    out = torch.empty((count, hqc.KEM_KEY_BYTES), dtype=torch.uint8, device=dev)

    def run(n):
        return hqc.kem_decaps_batch(pid, h, s, y, sigma, *classes[n], key_out=out, workspace=ws)

    for _ in range(3):
        for n in names:
            run(n)
    # the classes are what they claim: honest keys match, tampered ones differ
    assert torch.equal(run("honest"), key)
    assert not (run("tampered") == key).all(dim=1).any()
    torch.cuda.synchronize()

    reps = 60
    order = np.random.default_rng(pid + 7).permutation(np.repeat(np.arange(len(names)), reps))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in order]
    for (a, b), c in zip(ev, order):
        a.record()
        run(names[c])
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    keep = int(0.95 * reps)
    ts = {n: np.sort(t[order == i])[:keep] for i, n in enumerate(names)}
    for n in names:
        print("pid %d %-8s mean %.4f ms  sd %.4f  t vs honest %.2f" % (
            pid, n, ts[n].mean(), ts[n].std(), welch_t(ts[n], ts["honest"])), flush=True)
    rel = {n: ts[n].mean() / ts["honest"].mean() - 1.0 for n in names}
    assert abs(welch_t(ts["tampered"], ts["honest"])) < T_BOUND
    assert abs(rel["tampered"]) < HONEST_BOUND, rel
    assert abs(rel["random"]) < ZERO_BOUND, rel
