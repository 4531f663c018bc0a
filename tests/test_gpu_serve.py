"""The serving loop: requests arriving while others run are admitted as
memory frees up (with eviction), batched into shared launches, and every
result equals the same request run alone."""
import time

import numpy as np
import pytest
import torch  # noqa: F401

from oracle import mlp as OM
from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu

WIDTH, LAYERS = 256, 4


def test_serving_mix_equals_solo_under_eviction(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    budget = 16                                  # < unique blocks of the 3 functions: forces eviction
    ctx = sage_ctx_factory(pool_budget_bytes=budget * 65536, inflight_groups=3)
    w = synth.shared_mlp_bf16_functions(n_fns=3, layers=LAYERS, width=WIDTH, share_frac=0.25, seed=11)
    fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH), [S.make_blob(b)]) for b in w.blobs]
    rng = np.random.default_rng(0)
    reqs = [(int(rng.integers(0, 3)), int(rng.integers(1, 40))) for _ in range(40)]
    xs = [synth.bf16_inputs(b, WIDTH, 11, i) for i, (_, b) in enumerate(reqs)]
    solo = []
    for (f, b), x in zip(reqs, xs):
        inv = S.fn_setup(ctx, fns[f], b)
        y = np.zeros((b, WIDTH), dtype=np.float32)
        S.fn_invoke(ctx, inv, x, y)
        S.fn_release(ctx, inv)
        solo.append(y)
    for (f, b), x, y in zip(reqs, xs, solo):
        ref = OM.mlp_forward(OM.bf16_to_f64(x), OM.bf16_to_f64(w.blobs[f]).reshape(LAYERS, WIDTH, WIDTH))
        assert OM.normwise_error(y, ref) <= 2e-2
    ev0 = S.sage_get_stats(ctx)["evictions"]

    S.sage_serve_start(ctx)
    with pytest.raises(S.SageError) as e:
        S.fn_invoke_batch(ctx, [1], [xs[0]], [solo[0]])
    assert e.value.status == S.SAGE_ESTATE
    outs = [np.full((b, WIDTH), np.nan, dtype=np.float32) for _, b in reqs]
    ids = []
    for i, ((f, b), x) in enumerate(zip(reqs, xs)):
        ids.append(S.sage_submit(ctx, fns[f], b, x, outs[i]))
        if i % 7 == 3:
            time.sleep(0.002)                     # arrivals while earlier launches run
    infos = [S.sage_wait(ctx, r, 30000) for r in ids]
    rep = S.sage_serve_stats(ctx)
    S.sage_serve_stop(ctx)

    for y, o in zip(solo, outs):
        assert np.array_equal(y, o)
    assert all(i["status"] == 0 and i["e2e_ms"] >= i["setup_ms"] >= 0 for i in infos)
    assert rep["completed"] == len(reqs) and rep["failed"] == 0
    assert rep["launches"] < len(reqs)            # requests were batched together
    st = S.sage_get_stats(ctx)
    assert st["refcount_sum"] == 0 and st["live_setups"] == 0
    assert st["evictions"] > ev0                  # admission had to evict
    assert rep["setup_p99_ms"] <= rep["e2e_p99_ms"]


def test_serving_rejects_inadmissible_request(sage_ctx_factory, torch_cuda):
    """A function larger than the whole pool can never be admitted: the
    request fails with ENOMEM instead of waiting forever."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(pool_budget_bytes=8 * 65536)
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=LAYERS, width=WIDTH, share_frac=0.0, seed=12)
    f0 = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH), [S.make_blob(w.blobs[0])])
    f1 = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH), [S.make_blob(w.blobs[1])])
    inv = S.fn_setup(ctx, f1, 1)                  # pins all 8 slots for f1
    S.sage_serve_start(ctx)
    x = synth.bf16_inputs(2, WIDTH, 12, 0)
    y = np.zeros((2, WIDTH), dtype=np.float32)
    r = S.sage_submit(ctx, f0, 2, x, y)
    with pytest.raises(S.SageError) as e:
        S.sage_wait(ctx, r, 30000)
    assert e.value.status == S.SAGE_ENOMEM
    S.sage_serve_stop(ctx)
    S.fn_release(ctx, inv)


def test_unregister_while_queued_fails_the_request(sage_ctx_factory, torch_cuda):
    """A request whose function is unregistered while it waits in the queue
    fails with ENOTFOUND; the serving loop keeps running.  A long sweep keeps
    the device busy so the request waits (the pool is held by a live setup of
    another function) instead of failing at once."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=LAYERS, width=WIDTH, share_frac=0.0, seed=13)
    blocks = LAYERS * WIDTH * WIDTH * 2 // 65536
    ctx = sage_ctx_factory(pool_budget_bytes=blocks * 65536, inflight_groups=2)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH)
    f0 = S.fn_register(ctx, desc, [S.make_blob(w.blobs[0])])
    f1 = S.fn_register(ctx, desc, [S.make_blob(w.blobs[1])])
    hold = S.fn_setup(ctx, f1, 1)                 # f1's blocks fill the pool: f0 cannot be admitted
    nz, ny, nx = 64, 256, 1024                    # 64 MiB field, 400 sweeps: tens of ms on the device
    busy = S.fn_register(ctx, S.relax_desc(nx, ny, nz, 400, 0.5), [])
    u0 = torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda")
    u1 = torch.empty_like(u0)
    torch.cuda.synchronize()
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    S.sage_serve_start(ctx)
    rb = S.sage_submit(ctx, busy, 1, (u0.data_ptr(), u0.numel() * 4), (u1.data_ptr(), u1.numel() * 4), io)
    time.sleep(0.002)
    x = synth.bf16_inputs(2, WIDTH, 13, 0)
    y = np.zeros((2, WIDTH), dtype=np.float32)
    r0 = S.sage_submit(ctx, f0, 2, x, y)
    S.fn_unregister(ctx, f0)
    with pytest.raises(S.SageError) as e:
        S.sage_wait(ctx, r0, 30000)
    assert e.value.status == S.SAGE_ENOTFOUND
    assert S.sage_wait(ctx, rb, 30000)["status"] == 0
    # the loop still serves
    x1 = synth.bf16_inputs(3, WIDTH, 13, 1)
    y1 = np.zeros((3, WIDTH), dtype=np.float32)
    assert S.sage_wait(ctx, S.sage_submit(ctx, f1, 3, x1, y1), 30000)["status"] == 0
    S.sage_serve_stop(ctx)
    ref = OM.mlp_forward(OM.bf16_to_f64(x1), OM.bf16_to_f64(w.blobs[1]).reshape(LAYERS, WIDTH, WIDTH))
    assert OM.normwise_error(y1, ref) <= 2e-2
    with pytest.raises(S.SageError) as e:
        S.sage_submit(ctx, f1, 3, x1, y1)
    assert e.value.status == S.SAGE_ESTATE
    S.fn_release(ctx, hold)


def test_serving_width_4096_host_sources_vs_oracle(sage_ctx_factory, torch_cuda):
    """Serving at width 4096 from pinned host sources with a pool of half the
    unique bytes (every eviction reloads over the host link, reloads issued
    without waiting): each request's output in the mix equals its solo
    output bit for bit, and sampled outputs match the float64 oracle."""
    from paper_2404_14691_amd import sage as S
    W = 4096
    layers = [2, 3, 1, 4]
    blobs = synth.serving_blobs(layers, W, 0.2, seed=5)
    ctx0 = sage_ctx_factory(pool_budget_bytes=1 << 30)
    f0 = [S.fn_register(ctx0, S.mlp_desc(S.SAGE_MLP_BF16, l, W), [S.make_blob(b)]) for l, b in zip(layers, blobs)]
    unique = S.sage_get_stats(ctx0)["unique_bytes"]
    for f in f0:
        S.fn_unregister(ctx0, f)
    budget = unique // 2 // 65536 * 65536
    assert budget >= max(layers) * W * W * 2           # the largest function still fits alone
    ctx = sage_ctx_factory(pool_budget_bytes=budget, progressive=1)
    srcs = []
    for b in blobs:
        a = S.pinned_array(ctx, b.shape, b.dtype)
        a[:] = b
        srcs.append(a)
    fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, l, W), [S.make_blob(a)]) for l, a in zip(layers, srcs)]
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(0, len(layers))), int(rng.integers(1, 9))) for _ in range(48)]
    xs = [synth.bf16_inputs(b, W, 5, i) for i, (_, b) in enumerate(reqs)]
    solo = []
    for (f, b), x in zip(reqs, xs):
        inv = S.fn_setup(ctx, fns[f], b)
        y = np.zeros((b, W), dtype=np.float32)
        S.fn_invoke(ctx, inv, x, y)
        S.fn_release(ctx, inv)
        solo.append(y)
    ev0 = S.sage_get_stats(ctx)["evictions"]
    S.sage_serve_start(ctx)
    outs = [np.full((b, W), np.nan, dtype=np.float32) for _, b in reqs]
    ids = []
    for i, ((f, b), x) in enumerate(zip(reqs, xs)):
        ids.append(S.sage_submit(ctx, fns[f], b, x, outs[i]))
        if i % 5 == 2:
            time.sleep(0.003)
    infos = [S.sage_wait(ctx, r, 60000) for r in ids]
    S.sage_serve_stop(ctx)
    assert all(i["status"] == 0 for i in infos)
    for y, o in zip(solo, outs):
        assert np.array_equal(y, o)
    st = S.sage_get_stats(ctx)
    assert st["evictions"] > ev0 and st["refcount_sum"] == 0
    picks = sorted(set(int(k) for k in rng.choice(len(reqs), 6, replace=False)))
    wref = {}
    for k in picks:
        f, b = reqs[k]
        if f not in wref:
            wref[f] = OM.bf16_to_f64(blobs[f]).reshape(layers[f], W, W)
        ref = OM.mlp_forward(OM.bf16_to_f64(xs[k]), wref[f])
        assert OM.normwise_error(outs[k], ref) <= 2e-2, k
    for f in fns:
        S.fn_unregister(ctx, f)
    for a in srcs:
        S.sage_host_free(ctx, a.ctypes.data)
