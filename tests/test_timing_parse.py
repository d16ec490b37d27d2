"""Host-side checks of the profile parsing that the GPU timing tests use
(tests/ct_launches.py parse_profile), on small synthetic rocprofv3 CSV
files: library dispatches are grouped into calls, the per-call dispatch
count is found from the kernel-name sequence, counters reported in several
rows are summed, and other kernels and the earlier check calls are left out."""
import csv

import pytest

from tests.ct_launches import parse_profile

CC_FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
KT_FIELDS = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def write(tmp_path, dispatches):
    """dispatches: (name, cycles) in launch order; each counter is written
    as two rows (halves), as rocprofv3 does per hardware instance"""
    cc, kt = tmp_path / "cc.csv", tmp_path / "kt.csv"
    with open(cc, "w", newline="") as f, open(kt, "w", newline="") as g:
        wc, wk = csv.DictWriter(f, CC_FIELDS), csv.DictWriter(g, KT_FIELDS)
        wc.writeheader()
        wk.writeheader()
        t = 1000
        for i, (name, cyc) in enumerate(dispatches, start=1):
            for half in (0, 1):
                wc.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": "SQ_BUSY_CYCLES",
                             "Counter_Value": cyc / 2})
            wc.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": "SQ_INSTS_VALU",
                         "Counter_Value": 77})
            wk.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Start_Timestamp": t,
                         "End_Timestamp": t + 10 * i})
            t += 100000
    return str(cc), str(kt)


DEC = "void hqc::(anonymous namespace)::hqc_kernel<0, 1u, 1>(hqc::KArgs)"
CALL = [DEC, "void hqc::(anonymous namespace)::kem_draws_kernel<1>(...)",
        "void hqc::(anonymous namespace)::hqc_encrypt_kernel<3, 1>(hqc::EncArgs)",
        "void hqc::(anonymous namespace)::kem_key_kernel<1, true>(...)"]
TORCH = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<long>>(...)"


def test_one_dispatch_per_call(tmp_path):
    # a fill, one check launch, then five timed launches with copies between
    d = [(TORCH, 5), (DEC, 900)]
    for c in range(5):
        d += [(TORCH, 1), (DEC, 1000 + c)]
    cc, kt = write(tmp_path, d)
    calls = parse_profile(cc, kt, 5, 1)
    assert [len(c) for c in calls] == [1] * 5
    assert [c[0][1]["SQ_BUSY_CYCLES"] for c in calls] == [1000.0 + c for c in range(5)]
    assert all(c[0][1]["SQ_INSTS_VALU"] == 77 for c in calls)
    # durations come from the kernel trace of the same dispatch
    assert [c[0][2] for c in calls] == [10 * i for i in (4, 6, 8, 10, 12)]


def test_period_found_from_kernel_names(tmp_path):
    # three check calls with a torch compare between, then six timed calls
    d = [(n, 1) for n in CALL] + [(TORCH, 1)] + [(n, 2) for n in CALL] * 2
    for c in range(6):
        d += [(TORCH, 1)] + [(n, 100 * c + j) for j, n in enumerate(CALL)]
    cc, kt = write(tmp_path, d)
    calls = parse_profile(cc, kt, 6)
    assert len(calls) == 6 and all([x[0] for x in c] == CALL for c in calls)
    assert [sum(x[1]["SQ_BUSY_CYCLES"] for x in c) for c in calls] == [400 * c + 6 for c in range(6)]


def test_inconsistent_calls_rejected(tmp_path):
    d = [(n, 1) for n in CALL] * 3 + [(CALL[0], 1), (CALL[2], 1), (CALL[1], 1), (CALL[3], 1)]
    cc, kt = write(tmp_path, d)
    with pytest.raises(ValueError):
        parse_profile(cc, kt, 4, 4)
    # fewer dispatches than the calls need
    cc, kt = write(tmp_path, [(DEC, 1)] * 3)
    with pytest.raises(ValueError):
        parse_profile(cc, kt, 4, 1)
