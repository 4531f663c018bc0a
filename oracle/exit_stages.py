"""Oracle: the multi-stage resource exit (test infrastructure only).

Section "Multi-stage Resource Exit": when an invocation finishes, its
resources are released in order, one stage per interval T (the paper uses
T = 30 s for every stage):

  stage 1  GPU context and read-only data kept on the GPU;
  stage 2  GPU context kept, read-only data cached in CPU memory;
  stage 3  GPU context dropped, CPU memory (the cached data) kept;
  stage 4  CPU memory dropped, only the container (here: the registered
           function and its source) kept.

A new invocation in any stage reuses what is left.  Here the stage of a
resource follows from how long it has been idle: data from when its last
reference went, code from the last use of any function of its code object.

Pins (tests/test_oracle_exit_stages.py): which setup work Table 4 charges in
each stage (tests/golden/table4_resnet50.json): a stage skips GPU-context
creation exactly when `code_loaded`, pays the full GPU-data load exactly
when the data is not on the GPU, and pays the full CPU-data load exactly
when the data is back at its source.
"""
from __future__ import annotations


def stage(idle_ms: float, interval_ms: float) -> int:
    """Exit stage reached after `idle_ms` of idleness (1..4)."""
    if interval_ms <= 0:
        raise ValueError("interval must be positive")
    if idle_ms < 0:
        raise ValueError("idle time must be >= 0")
    return min(4, 1 + int(idle_ms // interval_ms))


def resources(st: int) -> dict:
    """Where a function's read-only data is and whether its GPU code is
    loaded, in exit stage `st`."""
    table = {
        1: {"data": "gpu", "code_loaded": True},
        2: {"data": "host_cache", "code_loaded": True},
        3: {"data": "host_cache", "code_loaded": False},
        4: {"data": "source", "code_loaded": False},
    }
    if st not in table:
        raise ValueError("stages are 1..4")
    return dict(table[st])


def setup_work(st: int) -> dict:
    """Setup work an invocation arriving in stage `st` has to do."""
    r = resources(st)
    return {"load_code": not r["code_loaded"],
            "move_data_to_gpu": r["data"] != "gpu",
            "read_data_from_source": r["data"] == "source"}
