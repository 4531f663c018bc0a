"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (device-resident sources and I/O, one grouped launch):
every fingerprint and the whole dedup partition bit-exact, sampled pool
slots byte-exact, every invocation against the float64 oracle and equal to
its own solo run bit for bit; the 512^3 stencil on every cell and on
sampled cells through their dependency cones."""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle import dedup as OD
from oracle import fingerprint as OF
from oracle import mlp as OM
from oracle import stencil as OS
from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu


def _oracle_outputs(blobs, reqs, xs, width, layers):
    """The float64 oracle output of every invocation; the rows of one
    function's invocations go through the oracle together (rows do not mix)."""
    out = {}
    for f in sorted({f for f, _ in reqs}):
        idx = [i for i, (g, _) in enumerate(reqs) if g == f]
        W = OM.bf16_to_f64(blobs[f]).reshape(layers, width, width)
        ref = OM.mlp_forward(np.concatenate([OM.bf16_to_f64(xs[i]) for i in idx]), W)
        del W
        r = 0
        for i in idx:
            b = reqs[i][1]
            out[i] = ref[r:r + b]
            r += b
    return out


def _run_group(S, ctx, torch, fns, reqs, width, xs):
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    dx = [torch.from_numpy(x).cuda() for x in xs]
    dy = [torch.zeros((b, width), dtype=torch.float32, device="cuda") for _, b in reqs]
    torch.cuda.synchronize()
    invs = [S.fn_setup(ctx, fns[f], b) for f, b in reqs]
    S.fn_invoke_batch(ctx, invs, [(t.data_ptr(), t.numel() * 2) for t in dx],
                      [(t.data_ptr(), t.numel() * 4) for t in dy], io)
    for inv in invs:
        S.fn_release(ctx, inv)
    return [t.cpu().numpy() for t in dy]


def test_sharing_workload_full_size(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory(pool_budget_bytes=2 << 30)
    w = synth.shared_mlp_bf16_functions(n_fns=4, layers=8, width=4096, share_frac=0.3, seed=0)
    dev = [torch.from_numpy(b.view(np.uint8)).cuda() for b in w.blobs]
    torch.cuda.synchronize()
    desc = S.mlp_desc(S.SAGE_MLP_BF16, 8, 4096)
    # one batch call, as the benchmark registers them
    fns, _ = S.fn_register_batch(ctx, [desc] * 4, [[S.make_blob(d.data_ptr(), d.numel(), where=S.SAGE_SRC_DEVICE)]
                                                   for d in dev])
    for f, b in zip(fns, w.blobs):
        assert np.array_equal(S.sage_fn_fingerprints(ctx, f), OF.fp64k_blob(b))
    canon = OD.partition_dict(w.blobs, 65536)
    lib = [[(int(c),) for c in S.sage_fn_block_info(ctx, f)[0]] for f in fns]
    assert OD.same_partition(canon, lib)
    acc = OD.accounting(w.blobs, 65536, canon)
    st = S.sage_get_stats(ctx)
    assert (st["unique_bytes"], st["shared_bytes"], st["private_bytes"]) == (acc["unique"], acc["shared"], acc["private"])
    assert acc["n_classes"] == 1228 + 4 * (4096 - 1228)
    rng = np.random.default_rng(1)
    for _ in range(24):
        f, k = int(rng.integers(0, 4)), int(rng.integers(0, 4096))
        slot = int(S.sage_fn_block_info(ctx, fns[f])[1][k])
        assert np.array_equal(S.sage_read_slot(ctx, slot), w.blobs[f].view(np.uint8)[k * 65536:(k + 1) * 65536])
    batches = synth.uniform_batches(256, 1, 32, seed=0)
    reqs = [(i % 4, int(b)) for i, b in enumerate(batches)]
    xs = [synth.bf16_inputs(b, 4096, 0, 100 + i) for i, (_, b) in enumerate(reqs)]
    ys = _run_group(S, ctx, torch, fns, reqs, 4096, xs)
    refs = _oracle_outputs(w.blobs, reqs, xs, 4096, 8)
    for i in range(len(reqs)):
        assert OM.normwise_error(ys[i], refs[i]) <= 2e-2, i
    for i in range(len(reqs)):  # each alone: the same bits as in the group
        solo = _run_group(S, ctx, torch, fns, [reqs[i]], 4096, [xs[i]])
        assert np.array_equal(solo[0], ys[i]), i


def test_batching_workload_full_size(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory(pool_budget_bytes=1 << 30)
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=8, width=4096, share_frac=0.0, seed=3)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 8, 4096), [S.make_blob(w.blobs[0])])
    batches = synth.lognormal_batches(256, seed=3)
    assert batches.min() >= 1 and batches.max() <= 128
    reqs = [(0, int(b)) for b in batches]
    xs = [synth.bf16_inputs(b, 4096, 3, i) for i, b in enumerate(batches)]
    ys = _run_group(S, ctx, torch, [fn], reqs, 4096, xs)
    refs = _oracle_outputs(w.blobs, reqs, xs, 4096, 8)
    for i in range(len(reqs)):
        assert OM.normwise_error(ys[i], refs[i]) <= 2e-2, i
    for i in range(len(reqs)):
        solo = _run_group(S, ctx, torch, [fn], [reqs[i]], 4096, [xs[i]])
        assert np.array_equal(solo[0], ys[i]), i


def test_stencil_full_size_sampled(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    n, sweeps = 512, 20
    ctx = sage_ctx_factory(pool_budget_bytes=1 << 30)
    c = synth.stencil_coefficients(n, seed=0)
    fn = S.fn_register(ctx, S.stencil_desc(n, n, n, sweeps), [S.make_blob(c)])
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    fields = [synth.stencil_field(n, i, seed=0) for i in range(2)]
    dx = [torch.from_numpy(u).cuda() for u in fields]
    dy = [torch.empty_like(t) for t in dx]
    torch.cuda.synchronize()
    invs = [S.fn_setup(ctx, fn, 1) for _ in fields]
    S.fn_invoke_batch(ctx, invs, [(t.data_ptr(), t.numel() * 4) for t in dx],
                      [(t.data_ptr(), t.numel() * 4) for t in dy], io)
    for inv in invs:
        S.fn_release(ctx, inv)
    rng = np.random.default_rng(2)
    pts = [(0, 0, 0), (1, 1, 1), (511, 300, 7), (256, 256, 256), (3, 510, 509), (20, 20, 20), (491, 20, 255)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(13)]
    for u0, t in zip(fields, dy):
        got = t.cpu().numpy()
        ref = OS.jacobi7_points(u0, c, sweeps, pts)
        vals = np.array([got[p] for p in pts], dtype=np.float64)
        assert np.max(np.abs(vals - ref)) / np.max(np.abs(ref)) <= 1e-5


def test_stencil_full_size_every_cell(sage_ctx_factory, torch_cuda):
    """One full 512^3 invocation (20 sweeps, the 512 MiB shared coefficient
    grid read through its block table, every x-tile seam and the ragged z
    tiles) against the float64 oracle on every cell."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    n, sweeps = 512, 20
    ctx = sage_ctx_factory(pool_budget_bytes=1 << 30)
    c = synth.stencil_coefficients(n, seed=0)
    fn = S.fn_register(ctx, S.stencil_desc(n, n, n, sweeps), [S.make_blob(c)])
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    u0 = synth.stencil_field(n, 1, seed=0)
    dx = torch.from_numpy(u0).cuda()
    dy = torch.empty_like(dx)
    torch.cuda.synchronize()
    inv = S.fn_setup(ctx, fn, 1)
    S.fn_invoke(ctx, inv, (dx.data_ptr(), dx.numel() * 4), (dy.data_ptr(), dy.numel() * 4), io)
    S.fn_release(ctx, inv)
    got = dy.cpu().numpy()
    del dx, dy
    S.fn_unregister(ctx, fn)
    ref = OS.jacobi7(u0, c, sweeps)
    assert OS.normwise_error(got, ref) <= 1e-5
    # the boundary keeps its initial values exactly
    for face in (np.s_[0], np.s_[-1], np.s_[:, 0], np.s_[:, -1], np.s_[:, :, 0], np.s_[:, :, -1]):
        assert np.array_equal(got[face], u0[face])


def test_stencil_32_fields_small_grid(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    n, sweeps = 64, 20
    ctx = sage_ctx_factory()
    c = synth.stencil_coefficients(n, seed=4)
    fn = S.fn_register(ctx, S.stencil_desc(n, n, n, sweeps), [S.make_blob(c)])
    fields = [synth.stencil_field(n, i, seed=4)[None] for i in range(32)]
    invs = [S.fn_setup(ctx, fn, 1) for _ in fields]
    outs = [np.zeros_like(f) for f in fields]
    S.fn_invoke_batch(ctx, invs, fields, outs)
    for inv in invs:
        S.fn_release(ctx, inv)
    for f, o in zip(fields, outs):
        assert OS.normwise_error(o[0], OS.jacobi7(f[0], c, sweeps)) <= 1e-5
