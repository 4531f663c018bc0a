"""The C ABI's contract on the GPU: argument and state errors return the
documented status and change nothing; empty work is a no-op."""
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)
import numpy as np
import pytest

from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu


def _status(fn, *a):
    from paper_2404_14691_amd import sage as S
    with pytest.raises(S.SageError) as e:
        fn(*a)
    return e.value.status


def test_open_rejects_bad_configs(torch_cuda):
    from paper_2404_14691_amd import sage as S
    cfg = S.sage_config_default()
    cfg.chunk_bytes = 65536 + 1
    assert _status(S.sage_open, 0, cfg) == S.SAGE_EINVAL
    cfg = S.sage_config_default()
    cfg.exit_stage_ms = -1.0
    assert _status(S.sage_open, 0, cfg) == S.SAGE_EINVAL
    assert _status(S.sage_open, 64, S.sage_config_default()) == S.SAGE_EINVAL


def test_setup_and_invoke_argument_errors(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=2, width=256, share_frac=0.0, seed=31)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 2, 256), [S.make_blob(w.blobs[0])])
    assert _status(S.sage_last_launch, ctx) == S.SAGE_ENOTFOUND
    assert _status(S.fn_setup, ctx, fn, 0) == S.SAGE_EINVAL
    inv = S.fn_setup(ctx, fn, 4)
    x = synth.bf16_inputs(4, 256, 31, 0)
    y = np.zeros((4, 256), dtype=np.float32)
    # wrong byte counts
    assert _status(S.fn_invoke, ctx, inv, x[:3], y) == S.SAGE_EINVAL
    assert _status(S.fn_invoke, ctx, inv, x, y[:, :128].copy()) == S.SAGE_EINVAL
    # the same invocation twice in one batch
    assert _status(S.fn_invoke_batch, ctx, [inv, inv], [x, x], [y, y]) == S.SAGE_EINVAL
    # device buffers must be 16-byte aligned
    dx = torch.zeros(4 * 256 + 8, dtype=torch.int16, device="cuda")
    dy = torch.zeros(4 * 256, dtype=torch.float32, device="cuda")
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    assert _status(S.fn_invoke, ctx, inv, (dx.data_ptr() + 2, 4 * 256 * 2), (dy.data_ptr(), 4 * 256 * 4),
                   io) == S.SAGE_EINVAL
    # an empty batch is a no-op; the invocation still runs afterwards
    S.fn_invoke_batch(ctx, [], [], [])
    S.fn_invoke(ctx, inv, x, y)
    assert np.isfinite(y).all() and np.abs(y).sum() > 0
    assert S.sage_last_launch(ctx).endswith(tuple("0123456789"))
    # a live function cannot be dropped; a released invocation cannot be used
    assert _status(S.fn_unregister, ctx, fn) == S.SAGE_EBUSY
    S.fn_release(ctx, inv)
    assert _status(S.fn_invoke, ctx, inv, x, y) == S.SAGE_ESTATE
    assert _status(S.fn_release, ctx, inv) == S.SAGE_ESTATE
    S.fn_unregister(ctx, fn)
    assert _status(S.fn_setup, ctx, fn, 1) == S.SAGE_ENOTFOUND


def test_failed_calls_change_no_counter(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=2, width=256, share_frac=0.0, seed=32)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 2, 256), [S.make_blob(w.blobs[0])])
    before = S.sage_get_stats(ctx)
    for bad in (lambda: S.fn_setup(ctx, fn, 0),
                lambda: S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 3, 256), [S.make_blob(w.blobs[0])]),
                lambda: S.sage_read_slot(ctx, 10 ** 6)):
        with pytest.raises(S.SageError):
            bad()
    after = S.sage_get_stats(ctx)
    assert {k: v for k, v in after.items() if not k.startswith("t_")} == \
           {k: v for k, v in before.items() if not k.startswith("t_")}


def test_zero_length_kernels_are_no_ops(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    out = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    S.sage_fingerprint(ctx, out.data_ptr(), 0, out.data_ptr())
    S.sage_blkcopy(ctx, out.data_ptr(), 0, out.data_ptr())
    torch.cuda.synchronize()
    assert int(out.item()) == 7


def test_setup_batch_times_each_request(sage_ctx_factory, torch_cuda):
    """fn_setup_batch with per-request times: one positive time per request,
    their sum within the call's own wall time; a failing request stops the
    batch with the earlier ones set up."""
    import time
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=2, width=256, share_frac=0.0, seed=33)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, 2, 256)
    fns = [S.fn_register(ctx, desc, [S.make_blob(b)]) for b in w.blobs]
    t0 = time.perf_counter()
    invs, ms = S.fn_setup_batch(ctx, [fns[0], fns[1], fns[0]], [3, 5, 1], timed=True)
    wall = (time.perf_counter() - t0) * 1e3
    assert len(invs) == len(set(invs)) == 3 and len(ms) == 3
    assert all(m > 0 for m in ms) and sum(ms) <= wall
    assert S.sage_get_stats(ctx)["live_setups"] == 3
    S.fn_release_batch(ctx, invs)
    assert _status(S.fn_setup_batch, ctx, [fns[1], fns[0]], [2, 0]) == S.SAGE_EINVAL
    assert S.sage_get_stats(ctx)["live_setups"] == 1  # the first request of the failed batch


def test_batch_calls_take_arrays(sage_ctx_factory, torch_cuda):
    """Handles and device I/O descriptors passed as numpy arrays give the
    same outputs as the per-request lists."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=2, width=256, share_frac=0.0, seed=34)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, 2, 256)
    fns = [S.fn_register(ctx, desc, [S.make_blob(b)]) for b in w.blobs]
    batches = [3, 1, 4]
    rows = sum(batches)
    x = torch.from_numpy(synth.bf16_inputs(rows, 256, 34, 0).view(np.int16)).cuda()
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    offs = np.concatenate([[0], np.cumsum(batches)[:-1]])
    ins = [(x.data_ptr() + int(o) * 512, b * 512) for o, b in zip(offs, batches)]
    results = []
    for arrays in (False, True):
        y = torch.zeros((rows, 256), dtype=torch.float32, device="cuda")
        outs = [(y.data_ptr() + int(o) * 1024, b * 1024) for o, b in zip(offs, batches)]
        f = [fns[0], fns[1], fns[0]]
        if arrays:
            invs, ms = S.fn_setup_batch(ctx, np.array(f, dtype=np.uint64), np.array(batches), timed=True)
            assert isinstance(invs, np.ndarray) and ms.shape == (3,)
            S.fn_invoke_batch(ctx, invs, np.array(ins, dtype=np.uint64), np.array(outs, dtype=np.uint64), io)
        else:
            invs = S.fn_setup_batch(ctx, f, batches)
            S.fn_invoke_batch(ctx, invs, ins, outs, io)
        S.fn_release_batch(ctx, invs)
        results.append(y.cpu().numpy())
    assert np.array_equal(results[0], results[1]) and np.abs(results[0]).sum() > 0
    assert S.sage_get_stats(ctx)["live_setups"] == 0


def test_timing_only_one_kernel(sage_ctx_factory, torch_cuda):
    """With timing restricted to the GEMM, registrations record no fingerprint
    or copy intervals and invocations still record theirs; the restriction
    lifts with None, and an unknown name is rejected."""
    from paper_2404_14691_amd import sage as S
    layers, width = 2, 256
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=layers, width=width, share_frac=0.0, seed=41)
    x = synth.bf16_inputs(5, width, 41, 0)
    y = np.zeros((5, width), dtype=np.float32)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, layers, width)
    ctx = sage_ctx_factory()
    assert _status(S.sage_timing_only, ctx, "no_such_kernel") == S.SAGE_EINVAL
    S.sage_timing_enable(ctx, True)
    for only, fp_timed in (("ggemm_bf16", False), (None, True)):
        S.sage_timing_reset(ctx)
        S.sage_timing_only(ctx, only)
        fn = S.fn_register(ctx, desc, [S.make_blob(w.blobs[0])])
        inv = S.fn_setup(ctx, fn, 5)
        S.fn_invoke(ctx, inv, x, y)
        S.fn_release(ctx, inv)
        S.fn_unregister(ctx, fn)
        assert (S.sage_timing_get(ctx, "fp64k")[1] > 0) == fp_timed, only
        assert S.sage_timing_get(ctx, "ggemm_bf16")[1] >= layers, only
    S.sage_timing_enable(ctx, False)


def test_mlp_graph_after_stencil_grows_the_flight_metadata(sage_ctx_factory, torch_cuda):
    """With one flight, an MLP group (its graph captured), then a sweep group
    whose per-sweep field tables outgrow the flight's metadata buffer, then
    the MLP group again: the second MLP run re-captures its graph on the new
    buffer and returns the first run's bits."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(inflight_groups=1)
    width, layers, b = 256, 3, 6
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=layers, width=width, share_frac=0.0, seed=33)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(w.blobs[0])])
    x = synth.bf16_inputs(b, width, 33, 0)
    y0 = np.zeros((b, width), dtype=np.float32)
    inv = S.fn_setup(ctx, fn, b)
    S.fn_invoke(ctx, inv, x, y0)
    # 8 fields x 9000 passes of two sweeps x 2 addresses x 8 bytes = 1.15 MB of field tables
    shape = (4, 4, 8)
    relax = S.fn_register(ctx, S.relax_desc(shape[2], shape[1], shape[0], 18000, 0.5), [])
    rinv = S.fn_setup(ctx, relax, 8)
    u0 = np.stack([synth.stencil_field(0, j, seed=33, shape=shape) for j in range(8)])
    u = np.zeros_like(u0)
    S.fn_invoke(ctx, rinv, u0, u)
    assert np.isfinite(u).all()
    y1 = np.full((b, width), np.nan, dtype=np.float32)
    S.fn_invoke(ctx, inv, x, y1)
    assert np.array_equal(y0, y1)
    S.fn_release(ctx, inv)
    S.fn_release(ctx, rinv)


@pytest.mark.parametrize("share", [1, 0])
def test_allocation_failure_gives_enomem_without_side_effects(sage_ctx_factory, torch_cuda, monkeypatch, share):
    """SAGE_FAULT_ALLOC_AFTER=0: every pool-arena and workspace allocation
    fails as if the device were full.  With sharing, registration cannot
    place its blocks and returns ENOMEM leaving no function, class or byte
    behind; without sharing, the private copy of fn_setup fails with ENOMEM
    and no invocation or reference remains.  A context without the knob runs
    the same work."""
    from paper_2404_14691_amd import sage as S
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=2, width=256, share_frac=0.0, seed=34).blobs[0]
    desc = S.mlp_desc(S.SAGE_MLP_BF16, 2, 256)
    monkeypatch.setenv("SAGE_FAULT_ALLOC_AFTER", "0")
    ctx = sage_ctx_factory(share=share)
    st0 = S.sage_get_stats(ctx)
    if share:
        assert _status(S.fn_register, ctx, desc, [S.make_blob(w)]) == S.SAGE_ENOMEM
    else:
        fn = S.fn_register(ctx, desc, [S.make_blob(w)])
        assert _status(S.fn_setup, ctx, fn, 3) == S.SAGE_ENOMEM
        S.fn_unregister(ctx, fn)
    st1 = S.sage_get_stats(ctx)
    for k in ("logical_bytes", "unique_bytes", "classes", "resident_bytes", "refcount_sum", "live_setups",
              "h2d_bytes", "workspace_bytes"):
        assert st1[k] == st0[k], k
    monkeypatch.delenv("SAGE_FAULT_ALLOC_AFTER")
    ok = sage_ctx_factory(share=share)
    fn = S.fn_register(ok, desc, [S.make_blob(w)])
    inv = S.fn_setup(ok, fn, 3)
    y = np.zeros((3, 256), dtype=np.float32)
    S.fn_invoke(ok, inv, synth.bf16_inputs(3, 256, 34, 0), y)
    assert np.isfinite(y).all() and np.abs(y).sum() > 0
    S.fn_release(ok, inv)


def test_host_io_batch_above_a_megabyte_same_bits_as_device_io(sage_ctx_factory, torch_cuda):
    """A batched launch whose host inputs and outputs exceed 1 MiB is staged
    by several host threads: every output equals the same launch's with
    device inputs and outputs bit for bit, and sampled ones the oracle."""
    from paper_2404_14691_amd import sage as S
    from oracle import mlp as OM
    torch = torch_cuda
    W, L = 1024, 2
    ctx = sage_ctx_factory()
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=L, width=W, share_frac=0.2, seed=61).blobs
    fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, L, W), [S.make_blob(b)]) for b in w]
    batches = [int(b) for b in synth.uniform_batches(48, 1, 32, seed=61)]
    xs = [synth.bf16_inputs(b, W, 61, i) for i, b in enumerate(batches)]
    assert sum(x.nbytes for x in xs) > (1 << 20)
    invs = [S.fn_setup(ctx, fns[i % 2], b) for i, b in enumerate(batches)]
    ys = [np.zeros((b, W), dtype=np.float32) for b in batches]
    S.fn_invoke_batch(ctx, invs, xs, ys)
    dx = [torch.from_numpy(x).cuda() for x in xs]
    dy = [torch.zeros((b, W), dtype=torch.float32, device="cuda") for b in batches]
    torch.cuda.synchronize()
    S.fn_invoke_batch(ctx, invs, [(t.data_ptr(), t.numel() * 2) for t in dx],
                      [(t.data_ptr(), t.numel() * 4) for t in dy], S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT)
    S.fn_release_batch(ctx, invs)
    for y, t in zip(ys, dy):
        assert np.array_equal(y, t.cpu().numpy())
    for i in (0, 17, 47):
        Wm = OM.bf16_to_f64(w[i % 2]).reshape(L, W, W)
        assert OM.normwise_error(ys[i], OM.mlp_forward(OM.bf16_to_f64(xs[i]), Wm)) <= 2e-2
