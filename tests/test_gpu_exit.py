"""Multi-stage exit on the GPU: as the idle time crosses one, two and three
intervals, the function's unreferenced blocks move to the host cache, its
code object is unloaded, and the host copies are dropped (the stages the
oracle's exit_stages table gives); every later invocation returns the same
bits as the first, reloading from wherever the bytes are."""
import time

import numpy as np
import pytest

from oracle import exit_stages as X
from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu

T_MS = 400.0  # interval of each stage; generous against the time of one setup + invoke


def _run(S, ctx, fn, x, width):
    inv = S.fn_setup(ctx, fn, x.shape[0])
    y = np.zeros((x.shape[0], width), dtype=np.float32)
    S.fn_invoke(ctx, inv, x, y)
    S.fn_release(ctx, inv)
    return y, time.monotonic()


def _sleep_until(t0, idle_ms):
    dt = t0 + idle_ms / 1e3 - time.monotonic()
    if dt > 0:
        time.sleep(dt)


def test_exit_stages_move_data_and_code_and_keep_results(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(exit_stage_ms=T_MS)
    layers, width = 3, 256
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=layers, width=width, share_frac=0.0, seed=21)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(w.blobs[0])])
    n_blocks = S.sage_fn_block_count(ctx, fn)
    x = synth.bf16_inputs(7, width, 21, 0)
    y0, t_rel = _run(S, ctx, fn, x, width)

    # first stage: everything stays
    st = S.sage_get_stats(ctx)
    assert X.stage((time.monotonic() - t_rel) * 1e3, T_MS) == 1
    assert st["resident_slots"] == n_blocks and st["demotions"] == 0 and st["module_unloads"] == 0

    # second stage: the blocks are in the host cache, the code still loaded
    _sleep_until(t_rel, 1.25 * T_MS)
    S.sage_tick(ctx)
    st = S.sage_get_stats(ctx)
    assert X.resources(2) == {"data": "host_cache", "code_loaded": True}
    assert st["resident_slots"] == 0 and st["demotions"] == n_blocks
    assert st["host_cached_bytes"] == n_blocks * 65536 and st["module_unloads"] == 0
    y, t_rel = _run(S, ctx, fn, x, width)
    st = S.sage_get_stats(ctx)
    assert np.array_equal(y, y0)
    assert st["host_reloads"] == n_blocks and st["host_cached_bytes"] == 0
    loads = st["module_loads"]

    # third stage: host copy kept, code object unloaded; both come back in one setup
    _sleep_until(t_rel, 2.25 * T_MS)
    S.sage_tick(ctx)
    st = S.sage_get_stats(ctx)
    assert st["module_unloads"] >= 1 and st["host_cached_bytes"] == n_blocks * 65536
    y, t_rel = _run(S, ctx, fn, x, width)
    st = S.sage_get_stats(ctx)
    assert np.array_equal(y, y0)
    assert st["module_loads"] == loads + 1 and st["host_reloads"] == 2 * n_blocks
    reloads = st["reloads"]

    # fourth stage: host copies dropped; the next setup reads the source again
    _sleep_until(t_rel, 3.25 * T_MS)
    S.sage_tick(ctx)
    st = S.sage_get_stats(ctx)
    assert st["host_cached_bytes"] == 0 and st["resident_slots"] == 0
    y, _ = _run(S, ctx, fn, x, width)
    st = S.sage_get_stats(ctx)
    assert np.array_equal(y, y0)
    assert st["host_reloads"] == 2 * n_blocks and st["reloads"] == reloads + n_blocks
    S.fn_unregister(ctx, fn)


def test_exit_is_per_block_idle_time(sage_ctx_factory, torch_cuda):
    """Blocks a live setup of another function still references stay in
    HBM; only the idle function's own blocks are demoted."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(exit_stage_ms=T_MS)
    layers, width = 2, 256
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=layers, width=width, share_frac=0.5, seed=22)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, layers, width)
    f1 = S.fn_register(ctx, desc, [S.make_blob(w.blobs[0])])
    f2 = S.fn_register(ctx, desc, [S.make_blob(w.blobs[1])])
    n = S.sage_fn_block_count(ctx, f1)
    shared = len(w.shared_idx)
    x = synth.bf16_inputs(3, width, 22, 0)
    y2, t_rel = _run(S, ctx, f2, x, width)
    held = S.fn_setup(ctx, f1, 3)  # f1 stays live through the interval
    _sleep_until(t_rel, 1.25 * T_MS)
    S.sage_tick(ctx)
    st = S.sage_get_stats(ctx)
    assert st["demotions"] == n - shared  # f2's own blocks only
    assert st["resident_slots"] == n
    y1 = np.zeros((3, width), dtype=np.float32)
    S.fn_invoke(ctx, held, x, y1)
    S.fn_release(ctx, held)
    y2b, _ = _run(S, ctx, f2, x, width)
    assert np.array_equal(y2b, y2)
