"""Timing checks of decryption and decapsulation against their input data,
after dudect (Reparaz, Balasch, Verbauwhede, "Dude, is my code constant
time?", 2017): calls of input classes made interleaved in a seeded random
order, measured per call, compared between classes.

Both run tests/ct_launches.py under rocprofv3's counter collection, which
copies each call's inputs into one set of buffers shared by all classes (so
that only the data differ, not the addresses read).  The deterministic
check: every dispatch of a kernel executes the same instructions (VALU,
SALU, LDS) with the same LDS bank conflicts in every class -- a branch or
loop that depended on the data would change these counts.  The statistical
check: durations in shader-clock cycles (SQ_BUSY_CYCLES) and in wall time,
with the mean of every class within a bound of the reference class's.

No bound is placed on Welch's t (it is printed).  Wall time differs between
classes that run the same instructions because the chip clocks higher on
data that switch fewer bits: all-zero data give 4-5 % shorter decryption
launches at equal cycle counts, honest data up to 1.5 % (wall-time |t| up
to 17 with 40 calls a class).  Cycles remove most of that, but not all:
over repeated runs the honest and random decryption classes differed by up
to 0.2 % in mean cycles (|t| from 0.1 to 7.4, on different boxes), with
identical instruction counts, and the decapsulation key kernel (one
wavefront per CU, mostly waiting on memory) by up to 0.3 %.

Decryption: classes zero (u = 0, v = codewords: no error at all), honest
(honest ciphertexts under one key) and random (random keys, uniform u and
v: every word past the decoding radius).  Mean cycles within 0.5 %
(honest) / 1 % (zero) of random, wall times within 2 % / 5 %.

Decapsulation: classes honest, tampered (one bit of v flipped: rejected by
the re-encryption check) and random (rejected, past the decoding radius);
each call is four launches (decryption, SHAKE256 draws, sampling with the
re-encryption check, key), their cycles summed: within 0.5 % of the honest
class's, wall times within 2 % (tampered) / 5 % (random)."""
import glob
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from tests.ct_launches import parse_profile


pytestmark = pytest.mark.gpu

# bounds on |mean(class) / mean(reference class) - 1| of wall times
# (measured: up to about 1 % honest and 2-4 % all-zero, at equal cycles)
HONEST_BOUND = 0.02
ZERO_BOUND = 0.05
# bound on the relative difference of mean cycles (measured: at most about
# 0.2 % for decryption, 0.1 % for a whole decapsulation; skipping a pass of
# the decoder would change far more, and the instruction counts besides)
CYCLE_BOUND = 0.005
# the all-zero class, the extreme of low switching activity: measured up to
# 0.23 % in cycles
ZERO_CYCLE_BOUND = 0.01
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


def profile_calls(mode, pid, tmp):
    """run tests/ct_launches.py under rocprofv3; returns the class of every
    timed call and, per call, its library dispatches as (kernel name,
    counters, duration in ns)"""
    exe = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(exe):
        pytest.skip("rocprofv3 not installed")
    helper = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ct_launches.py")
    order_path = os.path.join(tmp, "order.json")
    cmd = [exe, "--kernel-trace", "--pmc", *SAME, CYCLES, "--output-format", "csv",
           "-d", os.path.join(tmp, "prof"), "-o", "c", "--",
           sys.executable, "-u", helper, mode, str(pid), str(REPS), order_path]
    print("case: constant time %s pid=%d: %s" % (mode, pid, " ".join(cmd)), flush=True)
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
    calls = parse_profile(cc[0], kt[0], len(order), 1 if mode == "decrypt" else None)
    return order, calls


def check_classes(mode, pid, tmp, names, ref, cycle_bounds, wall_bounds):
    """the same instructions per kernel in every call; bounds on the
    relative difference of the mean cycles and wall times per call against
    the reference class"""
    order, calls = profile_calls(mode, pid, tmp)
    assert sorted(set(order)) == sorted(names) and len(order) == len(names) * REPS
    for j in range(len(calls[0])):
        for key in SAME:
            vals = {c[j][1][key] for c in calls}
            assert len(vals) == 1, (calls[0][j][0], key, sorted(vals)[:4])
    cyc = {n: cropped([sum(d[1][CYCLES] for d in c) for c, o in zip(calls, order) if o == n])
           for n in names}
    wall = {n: cropped([sum(d[2] for d in c) for c, o in zip(calls, order) if o == n]) for n in names}
    t = {n: welch_t(cyc[n], cyc[ref]) for n in names}
    rc = {n: cyc[n].mean() / cyc[ref].mean() - 1.0 for n in names}
    rw = {n: wall[n].mean() / wall[ref].mean() - 1.0 for n in names}
    for n in names:
        print("%s pid %d %-8s cycles %.0f (t vs %s %.2f, %+.3f %%)  wall %.4f ms (t vs %s %.2f, %+.2f %%)" % (
            mode, pid, n, cyc[n].mean(), ref, t[n], 100 * rc[n], wall[n].mean() / 1e6, ref,
            welch_t(wall[n], wall[ref]), 100 * rw[n]), flush=True)
    for n, bound in cycle_bounds.items():
        assert abs(rc[n]) < bound, rc
    for n, bound in wall_bounds.items():
        assert abs(rw[n]) < bound, rw


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decrypt_time_independent_of_data(pid, tmp_path):
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    check_classes("decrypt", pid, str(tmp_path), ["zero", "honest", "random"], "random",
                  cycle_bounds={"honest": CYCLE_BOUND, "zero": ZERO_CYCLE_BOUND},
                  wall_bounds={"honest": HONEST_BOUND, "zero": ZERO_BOUND})


@pytest.mark.parametrize("pid", [1, 3, 5])
def test_decaps_time_independent_of_rejection(pid, tmp_path):
    """Implicit rejection must not show in the time: decapsulation of honest
    ciphertexts, of ciphertexts with one bit of v flipped (rejected by the
    re-encryption check) and of uniformly random ciphertexts (rejected, and
    past the decoding radius) run the same kernels with the same launch
    shapes and the same instructions; the selection of m' or sigma is a
    per-item select of two loaded values."""
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    check_classes("decaps", pid, str(tmp_path), ["honest", "tampered", "random"], "honest",
                  cycle_bounds={"tampered": CYCLE_BOUND, "random": CYCLE_BOUND},
                  wall_bounds={"tampered": HONEST_BOUND, "random": ZERO_BOUND})
