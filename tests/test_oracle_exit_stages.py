"""Pins of oracle/exit_stages.py against the paper's multi-stage exit.

The stage boundaries follow the definition (one interval per stage); the
per-stage resources are checked against Table 4's resnet50 breakdown: in
each stage column, which setup components are charged in full, reduced or
not at all."""
import json
import os

import pytest

from oracle import exit_stages as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_resnet50.json")


def test_stage_boundaries():
    T = 30_000.0  # the paper's 30 s per stage
    assert X.stage(0, T) == 1
    assert X.stage(T - 1e-6, T) == 1
    assert X.stage(T, T) == 2
    assert X.stage(2 * T - 1e-6, T) == 2
    assert X.stage(2 * T, T) == 3
    assert X.stage(3 * T, T) == 4
    assert X.stage(100 * T, T) == 4
    with pytest.raises(ValueError):
        X.stage(1.0, 0.0)
    with pytest.raises(ValueError):
        X.stage(-1.0, T)


def test_release_order_data_then_code_then_host_memory():
    # read-only data leaves the GPU first, then the GPU context, then CPU memory
    on_gpu = [X.resources(s)["data"] == "gpu" for s in (1, 2, 3, 4)]
    code = [X.resources(s)["code_loaded"] for s in (1, 2, 3, 4)]
    in_host = [X.resources(s)["data"] == "host_cache" for s in (1, 2, 3, 4)]
    assert on_gpu == [True, False, False, False]
    assert code == [True, True, False, False]
    assert in_host == [False, True, True, False]


def test_setup_work_matches_table4_columns():
    cols = json.load(open(GOLDEN))["columns"]
    base = cols["baseline"]
    for st in (1, 2, 3, 4):
        col = cols[f"stage{st}"]
        w = X.setup_work(st)
        # GPU context: charged in full exactly when the code must be loaded
        assert (col["gpu_ctx"] == base["gpu_ctx"]) == w["load_code"]
        assert (col["gpu_ctx"] == 0) == (not w["load_code"])
        # GPU data: the full load exactly when the data is not on the GPU
        assert (col["gpu_data"] == base["gpu_data"]) == w["move_data_to_gpu"]
        # CPU data: the full load exactly when the data is back at its source
        assert (col["cpu_data"] == base["cpu_data"]) == w["read_data_from_source"]


def test_planted_mistake_is_caught():
    # swapping the order of the second and third stages contradicts Table 4
    cols = json.load(open(GOLDEN))["columns"]
    wrong = {2: {"data": "host_cache", "code_loaded": False}}
    st = 2
    w = {"load_code": not wrong[st]["code_loaded"]}
    assert (cols["stage2"]["gpu_ctx"] == cols["baseline"]["gpu_ctx"]) != w["load_code"]
