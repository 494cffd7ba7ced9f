"""Host side of the autotuner: the persisted table (one tuning per workload
class, reused by later runs) and the workload classes."""
import json

from paper_2504_04564_amd import autotune


def test_tuning_is_measured_once_and_persisted(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def fake_tune():
        calls.append(1)
        return {"macrocell": 64, "tile_w": 32, "cache": 2, "ms": 74.4}, []

    key = autotune.workload_key("vdb", (1987, 1351, 2449), 0.10, 64)
    first = autotune.cached_render_tuning(path, key, fake_tune)
    again = autotune.cached_render_tuning(path, key, fake_tune)
    assert first == again == {"macrocell": 64, "tile_w": 32, "cache": 2, "ms": 74.4}
    assert len(calls) == 1
    assert json.load(open(path)) == {key: first}
    # another class is tuned on its own and kept beside the first
    key2 = autotune.workload_key("vdb", (512, 512, 512), 0.10, 16)
    autotune.cached_render_tuning(path, key2, fake_tune)
    assert len(calls) == 2 and set(autotune.load(path)) == {key, key2}


def test_workload_classes():
    # log2 bucket of the largest side, rate to 1/100, spp
    assert autotune.workload_key("vdb", (1987, 1351, 2449), 0.1, 64) == "vdb/n11/q0.10/spp64"
    assert autotune.workload_key("dense", (512, 512, 512), 0.25, 16) == "dense/n9/q0.25/spp16"
    assert autotune.workload_key("vdb", (700, 10, 10), 0.05, 1) == "vdb/n9/q0.05/spp1"
    # the render search space covers the macrocells the frames were tuned to
    assert {16, 64} <= set(autotune.RENDER_SPACE["macrocell"])
