"""The launch-configuration table and the autotuner's JSON cache, without a
GPU: the table keys on (device, parameter set, power-of-two bucket of the
count), rejects bad entries, and the cache applies only entries of the same
architecture whose candidates all agreed."""
import pytest


@pytest.fixture(scope="module")
def hqc():
    from paper_2512_12904_amd import build, hqc
    if build.gpu_stale():
        build.build_gpu()
    return hqc


def test_table_buckets_and_errors(hqc):
    hqc.tune_clear()
    assert hqc.tune_get(1, 65536) == (0, 0, 0)
    hqc.tune_set(1, 65536, 32, 2048)
    # same bucket: 32769 .. 65536
    assert hqc.tune_get(1, 65536) == (32, 2048, 1)
    assert hqc.tune_get(1, 40000) == (32, 2048, 1)
    assert hqc.tune_get(1, 32768) == (0, 0, 0)
    assert hqc.tune_get(1, 65537) == (0, 0, 0)
    assert hqc.tune_get(3, 65536) == (0, 0, 0)
    hqc.tune_set(1, 65536, 0, 0, 0)  # removes the entry
    assert hqc.tune_get(1, 65536) == (0, 0, 0)
    # shape B exists for HQC-1 and HQC-3
    hqc.tune_set(1, 131072, 32, 3072, 2)
    hqc.tune_set(3, 1000, 8, 100, 2)
    assert hqc.tune_get(1, 100000) == (32, 3072, 2)
    assert hqc.tune_get(3, 1000) == (8, 100, 2)
    for bad in [(2, 10, 8, 8, 1), (1, 0, 8, 8, 1), (1, 10, 65, 8, 1), (1, 10, 8, 0, 1),
                (1, 10, 0, 8, 1), (1, 10, 8, 8, 3), (1, 10, 8, 8, 0), (5, 10, 8, 8, 2)]:
        with pytest.raises(hqc.HqcError):
            hqc.tune_set(*bad)
    hqc.tune_set(5, 7, 8, 100)
    hqc.tune_clear()
    assert hqc.tune_get(5, 7) == (0, 0, 0)


def test_cache_round_trip(hqc, tmp_path):
    from paper_2512_12904_amd import tune
    hqc.tune_clear()
    reports = [
        {"param_id": 1, "count": 65536, "tile": 24, "grid": 1536, "shape": 2, "ms": 0.4,
         "heuristic_tile": 32, "heuristic_grid": 2048, "heuristic_shape": 1, "heuristic_ms": 0.41,
         "candidates": 30, "identical": 1},
        {"param_id": 3, "count": 4096, "tile": 16, "grid": 256, "shape": 1, "ms": 0.1,
         "heuristic_tile": 2, "heuristic_grid": 2048, "heuristic_shape": 1, "heuristic_ms": 0.2,
         "candidates": 12, "identical": 0},
    ]
    path = tune.save(reports, str(tmp_path / "t.json"), arch="gfx950")
    assert tune.load(path, arch="gfx942") == 0  # another architecture
    assert hqc.tune_get(1, 65536) == (0, 0, 0)
    assert tune.load(path, arch="gfx950") == 1  # the disagreeing entry is skipped
    assert hqc.tune_get(1, 65536) == (24, 1536, 2)
    assert hqc.tune_get(3, 4096) == (0, 0, 0)
    assert tune.load(str(tmp_path / "missing.json"), arch="gfx950") == 0
    hqc.tune_clear()
