"""Autotuner driver for the decryption kernel's launch configuration.

`hqc_autotune_decrypt` (the C library) times (tile, grid) candidates on the
device and keeps the fastest in a per-device table that single-set calls
use when they leave grid and tile at 0.  This module runs it over parameter
sets and batch sizes and saves or restores the chosen configurations as
JSON, keyed by the GPU architecture, so that a process can start with a
tuned table without timing again:

    python -m paper_2512_12904_amd.tune --sets 1,3,5 --counts 4096,65536
    ...
    from paper_2512_12904_amd import tune; tune.load()
"""
import argparse
import json
import os

from . import hqc

DEFAULT_COUNTS = (1024, 4096, 16384, 65536)


def device_arch():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def default_path(arch=None):
    root = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    arch = arch or device_arch()
    safe = "".join(ch if ch.isalnum() or ch in "-_." else "_" for ch in arch)
    return os.path.join(root, "paper_2512_12904_amd", "tune_%s.json" % safe)


def tune(sets=(1, 3, 5), counts=DEFAULT_COUNTS, reps=5, stream=None):
    """Autotune every (set, count); returns the reports (the table is filled)."""
    return [hqc.autotune_decrypt(pid, int(c), reps, stream) for pid in sets for c in counts]


def to_json(reports, arch):
    return {"arch": arch, "entries": [
        {"param_id": r["param_id"], "count": r["count"], "tile": r["tile"], "grid": r["grid"],
         "shape": r["shape"], "ms": r["ms"], "heuristic_tile": r["heuristic_tile"],
         "heuristic_grid": r["heuristic_grid"], "heuristic_shape": r["heuristic_shape"],
         "heuristic_ms": r["heuristic_ms"],
         "candidates": r["candidates"], "identical": r["identical"]} for r in reports]}


def save(reports, path=None, arch=None):
    arch = arch or device_arch()
    path = path or default_path(arch)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(to_json(reports, arch), f, indent=1)
    os.replace(tmp, path)
    return path


def apply(doc, arch):
    """Put the entries of a saved document into the library's table.  Entries
    of another architecture, or whose candidates did not all agree, are
    skipped.  Returns the number applied."""
    if doc.get("arch") != arch:
        return 0
    n = 0
    for e in doc.get("entries", []):
        if not e.get("identical"):
            continue
        tile, grid, shape = int(e["tile"]), int(e["grid"]), int(e.get("shape", 1))
        if not (1 <= tile <= 64 and grid >= 1 and shape in (1, 2)):
            continue
        hqc.tune_set(int(e["param_id"]), int(e["count"]), tile, grid, shape)
        n += 1
    return n


def load(path=None, arch=None):
    """Restore a saved table for the current device; returns the entry count
    applied (0 when there is no file for this architecture)."""
    arch = arch or device_arch()
    path = path or default_path(arch)
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        return apply(json.load(f), arch)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sets", default="1,3,5")
    ap.add_argument("--counts", default=",".join(str(c) for c in DEFAULT_COUNTS))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=None, help="JSON path (default: the per-arch cache file)")
    a = ap.parse_args(argv)
    reports = []
    for pid in (int(x) for x in a.sets.split(",")):
        # one set at a time, so that progress shows as it goes
        reports += tune([pid], [int(x) for x in a.counts.split(",")], a.reps)
        print("HQC-%d tuned" % pid, flush=True)
    for r in reports:
        print("HQC-%d count %7d: shape %s tile %2d grid %5d %.4f ms (default shape %s tile %2d "
              "grid %5d %.4f ms, %d candidates, identical %d)" % (
                  r["param_id"], r["count"], "AB"[r["shape"] - 1], r["tile"], r["grid"], r["ms"],
                  "AB"[r["heuristic_shape"] - 1], r["heuristic_tile"], r["heuristic_grid"],
                  r["heuristic_ms"], r["candidates"], r["identical"]),
              flush=True)
    print("saved", save(reports, a.out))


if __name__ == "__main__":
    main()
