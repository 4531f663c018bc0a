"""Parity of the function bodies run through fn_invoke / fn_invoke_batch:
BF16 and FP32 MLPs and the 7-point stencil against the float64 oracle, exact
special cases, and the invariants shared == private and grouped == solo."""
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)
import numpy as np
import pytest

from oracle import mlp as OM
from oracle import stencil as OS
from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu

BF16_TOL = 2e-2
F32_TOL = 1e-5


def _bf16_fn(S, ctx, layers, width, seed=0):
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=layers, width=width, share_frac=0.0, seed=seed)
    blob = w.blobs[0]
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(blob)])
    return fn, blob


def _run(S, ctx, fn, xs, width, batch_call=True, io=0, torch=None):
    invs = [S.fn_setup(ctx, fn, x.shape[0]) for x in xs]
    ys = [np.zeros((x.shape[0], width), dtype=np.float32) for x in xs]
    if io:
        dx = [torch.from_numpy(x).cuda() for x in xs]
        dy = [torch.zeros((x.shape[0], width), dtype=torch.float32, device="cuda") for x in xs]
        torch.cuda.synchronize()
        S.fn_invoke_batch(ctx, invs, [(t.data_ptr(), t.numel() * t.element_size()) for t in dx],
                          [(t.data_ptr(), t.numel() * 4) for t in dy], io)
        ys = [t.cpu().numpy() for t in dy]
    elif batch_call:
        S.fn_invoke_batch(ctx, invs, xs, ys)
    else:
        for inv, x, y in zip(invs, xs, ys):
            S.fn_invoke(ctx, inv, x, y)
    for inv in invs:
        S.fn_release(ctx, inv)
    return ys


BATCHES = [1, 7, 16, 33, 100]


def test_bf16_mlp_ragged_group_vs_oracle(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    layers, width = 3, 256
    fn, blob = _bf16_fn(S, ctx, layers, width)
    xs = [synth.bf16_inputs(b, width, 0, i) for i, b in enumerate(BATCHES)]
    ys = _run(S, ctx, fn, xs, width)
    W = OM.bf16_to_f64(blob).reshape(layers, width, width)
    for x, y in zip(xs, ys):
        ref = OM.mlp_forward(OM.bf16_to_f64(x), W)
        assert OM.normwise_error(y, ref) <= BF16_TOL
        # the GPU rounds hidden layers to BF16: it must sit much closer to the mirror
        assert OM.normwise_error(y, OM.mlp_forward_mirror(OM.bf16_to_f64(x), W)) <= 2e-3


def test_bf16_grouped_equals_solo_and_device_io(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    layers, width = 2, 512
    fn, _ = _bf16_fn(S, ctx, layers, width, seed=1)
    xs = [synth.bf16_inputs(b, width, 1, i) for i, b in enumerate(BATCHES)]
    grouped = _run(S, ctx, fn, xs, width, batch_call=True)
    solo = _run(S, ctx, fn, xs, width, batch_call=False)
    dev = _run(S, ctx, fn, xs, width, io=S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT, torch=torch_cuda)
    for g, s, d in zip(grouped, solo, dev):
        assert np.array_equal(g, s)
        assert np.array_equal(g, d)


def test_bf16_shared_equals_private_and_eager(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    layers, width = 3, 256
    xs = [synth.bf16_inputs(b, width, 2, i) for i, b in enumerate(BATCHES)]
    outs = []
    for over in ({}, {"share": 0}, {"batch": 0}):
        ctx = sage_ctx_factory(**over)
        fn, _ = _bf16_fn(S, ctx, layers, width, seed=2)
        outs.append(_run(S, ctx, fn, xs, width))
    for a, b, c in zip(*outs):
        assert np.array_equal(a, b)
        assert np.array_equal(a, c)


TILES = ["ggemm6p_bf16_256x256", "ggemm6_bf16_256x128", "ggemm2_bf16_128x256", "ggemm_bf16_128x128",
         "ggemm3_bf16_128x64", "ggemm_bf16_64x128", "ggemm_bf16_32x128", "ggemm3g4_bf16_64x64",
         "ggemm3g4_bf16_32x64", "ggemm3g4_bf16_16x64", "ggemm3t_bf16_32x32", "ggemm3t_bf16_16x32",
         "ggemm3t_bf16_16x16",
         # a large shape over full row tiles + a thin shape over the ragged last ones
         "ggemm6p_bf16_256x256+ggemm3t_bf16_32x32", "ggemm6p_bf16_256x256+ggemm3g4_bf16_16x64",
         "ggemm6_bf16_256x128+ggemm3t_bf16_16x16", "ggemm2_bf16_128x256+ggemm3g4_bf16_64x64"]


def test_bf16_every_tile_shape_same_bits(sage_ctx_factory, torch_cuda, monkeypatch):
    """Every tile shape (forced, autotuner bypassed) walks K in the same order
    with the same MFMA: all give identical bits, and match the oracle; more
    than 256 rows in a group exercise several m-tiles of the largest tiles.
    "main+tail" forces a split launch: the ragged last row tile of every
    group runs in a second, thin-tile launch of each layer."""
    from paper_2404_14691_amd import sage as S
    layers, width = 2, 512
    batches = [300, 5, 70, 1]
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=layers, width=width, share_frac=0.3, seed=9)
    xs = [synth.bf16_inputs(b, width, 9, i) for i, b in enumerate(batches)]
    first = None
    for tile in TILES:
        monkeypatch.setenv("SAGE_TILE", tile)
        ctx = sage_ctx_factory()
        monkeypatch.delenv("SAGE_TILE")
        fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(b)]) for b in w.blobs]
        invs = [S.fn_setup(ctx, fns[i % 2], b) for i, b in enumerate(batches)]
        ys = [np.zeros((b, width), dtype=np.float32) for b in batches]
        S.fn_invoke_batch(ctx, invs, xs, ys)
        S.fn_release_batch(ctx, invs)
        plan = S.sage_last_launch(ctx)
        assert plan.split("+")[0].split(":")[0] == tile.split("+")[0], plan
        assert ("+" in plan) == ("+" in tile), plan
        if first is None:
            first = ys
            for i, (x, y) in enumerate(zip(xs, ys)):
                W = OM.bf16_to_f64(w.blobs[i % 2]).reshape(layers, width, width)
                assert OM.normwise_error(y, OM.mlp_forward(OM.bf16_to_f64(x), W)) <= BF16_TOL
        else:
            for a, b in zip(first, ys):
                assert np.array_equal(a, b), tile


@pytest.mark.parametrize("width,layers", [(128, 3), (8192, 1)])
def test_bf16_mlp_width_limits(sage_ctx_factory, torch_cuda, width, layers):
    """The narrowest BF16 layer (width 128: only the shapes at most 128 wide
    fit; 3 layers are 96 KiB, so the blob ends in a partial block) and a wide
    one (8192: a K walk of 256 slices, 128 MiB per layer), 5 and 11 rows
    batched and alone, against the float64 oracle and each other."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(pool_budget_bytes=(1 << 30))
    rng = np.random.default_rng(width)
    blob = synth.f32_to_bf16_bits(rng.standard_normal((layers, width, width), dtype=np.float32)
                                  / np.float32(np.sqrt(width))).reshape(-1)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(blob)])
    xs = [synth.bf16_inputs(b, width, width, i) for i, b in enumerate((5, 11))]
    ys = _run(S, ctx, fn, xs, width)
    W = OM.bf16_to_f64(blob).reshape(layers, width, width)
    for x, y in zip(xs, ys):
        assert OM.normwise_error(y, OM.mlp_forward(OM.bf16_to_f64(x), W)) <= BF16_TOL
    solo = _run(S, ctx, fn, xs, width, batch_call=False)
    for a, b in zip(ys, solo):
        assert np.array_equal(a, b)
    S.fn_unregister(ctx, fn)


def test_bf16_permutation_weights_exact(sage_ctx_factory, torch_cuda):
    """Permutation-matrix weights: every output is one input value, passed
    through ReLU: the block-table indexing and the MFMA fragment layout must
    put every element in its place, bit for bit."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    layers, width = 3, 256
    rng = np.random.default_rng(0)
    perms = [rng.permutation(width) for _ in range(layers)]
    W = np.zeros((layers, width, width), dtype=np.uint16)
    for l, p in enumerate(perms):
        W[l, np.arange(width), p] = 0x3F80                       # bf16 1.0
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, layers, width), [S.make_blob(W.reshape(-1))])
    xs = [synth.bf16_inputs(b, width, 3, i) for i, b in enumerate([3, 40])]
    ys = _run(S, ctx, fn, xs, width)
    for x, y in zip(xs, ys):
        ref = OM.mlp_forward(OM.bf16_to_f64(x), OM.bf16_to_f64(W))
        assert np.array_equal(y.astype(np.float64), ref)


def test_f32_mlp_vs_oracle(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    wl = synth.mlp_f32_workload(width=256, layers=2, batch=8, invocations=3, seed=4)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, 2, 256), [S.make_blob(wl.weights.reshape(-1))])
    xs = wl.inputs + [np.random.default_rng(1).standard_normal((13, 256)).astype(np.float32)]
    ys = _run(S, ctx, fn, xs, 256)
    for x, y in zip(xs, ys):
        assert OM.normwise_error(y, OM.mlp_forward(x, wl.weights)) <= F32_TOL
    solo = _run(S, ctx, fn, xs, 256, batch_call=False)
    for a, b in zip(ys, solo):
        assert np.array_equal(a, b)


def test_f32_scattered_block_table_same_bits(sage_ctx_factory, torch_cuda):
    """FP32 weights read through a scattered block table: a second function
    whose every other block repeats the first function's blocks points half
    its table at the first function's slots.  Both functions alone, together
    in one launch (two groups; rows staged back to back, or from separate
    device buffers), with device and host I/O, and from private copies
    (share=0) give the same bits, within tolerance of the float64 oracle."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    W, L = 512, 3
    rng = np.random.default_rng(7)
    w0 = (rng.standard_normal((L, W, W)) / np.sqrt(W)).astype(np.float32)
    w1 = (rng.standard_normal((L, W, W)) / np.sqrt(W)).astype(np.float32)
    per = 65536 // 4
    f0, f1 = w0.reshape(-1, per), w1.reshape(-1, per)
    f1[::2] = f0[::2]                               # shared blocks: f1's slots are not back to back
    xs = [rng.standard_normal((b, W)).astype(np.float32) for b in (8, 5)]
    outs = {}
    for share in (1, 0):
        ctx = sage_ctx_factory(share=share, pool_budget_bytes=64 << 20)
        fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, L, W), [S.make_blob(w)]) for w in (w0, w1)]
        solo = []
        for fn, x in zip(fns, xs):
            inv = S.fn_setup(ctx, fn, len(x))
            y = np.zeros((len(x), W), dtype=np.float32)
            S.fn_invoke(ctx, inv, x, y)
            dx = torch.from_numpy(x).cuda()
            dy = torch.zeros((len(x), W), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            S.fn_invoke(ctx, inv, (dx.data_ptr(), dx.numel() * 4), (dy.data_ptr(), dy.numel() * 4),
                        S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT)
            assert np.array_equal(dy.cpu().numpy(), y)
            S.fn_release(ctx, inv)
            solo.append(y)
        invs = [S.fn_setup(ctx, fn, len(x)) for fn, x in zip(fns, xs)]
        ys = [np.zeros((len(x), W), dtype=np.float32) for x in xs]
        S.fn_invoke_batch(ctx, invs, xs, ys)
        # device I/O from separate buffers: rows not back to back, read through the row tables
        dxs = [torch.from_numpy(x).cuda() for x in xs]
        dys = [torch.zeros((len(x), W), dtype=torch.float32, device="cuda") for x in xs]
        torch.cuda.synchronize()
        S.fn_invoke_batch(ctx, invs, [(t.data_ptr(), t.numel() * 4) for t in dxs],
                          [(t.data_ptr(), t.numel() * 4) for t in dys], S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT)
        for inv in invs:
            S.fn_release(ctx, inv)
        for a, b, c in zip(solo, ys, dys):
            assert np.array_equal(a, b) and np.array_equal(a, c.cpu().numpy())
        outs[share] = solo
    for a, b in zip(outs[1], outs[0]):
        assert np.array_equal(a, b)
    for w, x, y in zip((w0, w1), xs, outs[1]):
        assert OM.normwise_error(y, OM.mlp_forward(x, w.astype(np.float64))) <= F32_TOL


def test_f32_mlp_two_k_chunks(sage_ctx_factory, torch_cuda):
    """Width 4096: each column's K is walked as two 2048-wide chunks whose
    partial sums accumulate before the lanes and waves are combined; 3 and 9
    rows alone (ragged row blocks) and together (8 + 4), against the float64
    oracle and each other."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(pool_budget_bytes=512 << 20)
    W, L = 4096, 2
    rng = np.random.default_rng(12)
    w = (rng.standard_normal((L, W, W)) / np.sqrt(W)).astype(np.float32)
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, L, W), [S.make_blob(w.reshape(-1))])
    xs = [rng.standard_normal((b, W)).astype(np.float32) for b in (3, 9)]
    ys = _run(S, ctx, fn, xs, W)
    for x, y in zip(xs, ys):
        assert OM.normwise_error(y, OM.mlp_forward(x, w.astype(np.float64))) <= F32_TOL
    solo = _run(S, ctx, fn, xs, W, batch_call=False)
    for a, b in zip(ys, solo):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("W,L", [(128, 3), (16384, 1)])
def test_f32_mlp_width_limits(sage_ctx_factory, torch_cuda, W, L):
    """The narrowest FP32 layer (width 128: a 32-wide quarter of K per wave,
    8 of its 64 lanes loading) and the widest (16384: rows of 64 KiB, eight
    K chunks), 5 and 11 rows, batched and alone, against the float64 oracle
    and each other."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(pool_budget_bytes=(2 << 30))
    rng = np.random.default_rng(W + L)
    w = (rng.standard_normal((L, W, W), dtype=np.float32) / np.float32(np.sqrt(W)))
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, L, W), [S.make_blob(w.reshape(-1))])
    xs = [rng.standard_normal((b, W), dtype=np.float32) for b in (5, 11)]
    ys = _run(S, ctx, fn, xs, W)
    for x, y in zip(xs, ys):
        assert OM.normwise_error(y, OM.mlp_forward(x, w.astype(np.float64))) <= F32_TOL
    solo = _run(S, ctx, fn, xs, W, batch_call=False)
    for a, b in zip(ys, solo):
        assert np.array_equal(a, b)
    S.fn_unregister(ctx, fn)


def test_f32_mlp_full_size_sixteen_invocations(sage_ctx_factory, torch_cuda):
    """2-layer FP32 MLP of width 2048, 16 sequential invocations of 8 rows,
    each with its own input: every output element vs the float64 oracle."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(share=0)
    wl = synth.mlp_f32_workload()
    fn = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, 2, 2048), [S.make_blob(wl.weights.reshape(-1))])
    for x in wl.inputs:
        inv = S.fn_setup(ctx, fn, 8)
        y = np.zeros((8, 2048), dtype=np.float32)
        S.fn_invoke(ctx, inv, x, y)
        S.fn_release(ctx, inv)
        assert OM.normwise_error(y, OM.mlp_forward(x, wl.weights)) <= F32_TOL
    assert S.sage_get_stats(ctx)["h2d_bytes"] == 16 * wl.weights.nbytes


@pytest.mark.parametrize("shape,sweeps", [((18, 20, 32), 5), ((9, 7, 64), 4), ((5, 3, 128), 1), ((6, 6, 16), 0),
                                          ((70, 45, 64), 3)])
def test_stencil_vs_oracle(sage_ctx_factory, torch_cuda, shape, sweeps):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    nz, ny, nx = shape
    c = synth.stencil_coefficients(0, seed=1, shape=shape)
    fn = S.fn_register(ctx, S.stencil_desc(nx, ny, nz, sweeps), [S.make_blob(c)])
    fields = [np.stack([synth.stencil_field(0, 10 * i + j, seed=1, shape=shape) for j in range(b)])
              for i, b in enumerate([3, 1])]
    invs = [S.fn_setup(ctx, fn, f.shape[0]) for f in fields]
    outs = [np.zeros_like(f) for f in fields]
    S.fn_invoke_batch(ctx, invs, fields, outs)
    for inv in invs:
        S.fn_release(ctx, inv)
    for f, o in zip(fields, outs):
        for j in range(f.shape[0]):
            ref = OS.jacobi7(f[j], c, sweeps)
            assert OS.normwise_error(o[j], ref) <= F32_TOL
            if sweeps == 0:
                assert np.array_equal(o[j], f[j])


@pytest.mark.parametrize("shape,sweeps", [((70, 33, 300), 4), ((9, 20, 64), 5), ((66, 17, 260), 2), ((4, 5, 8), 3)])
def test_stencil_two_sweeps_per_pass_same_bits(sage_ctx_factory, torch_cuda, monkeypatch, shape, sweeps):
    """Sweeps fused in passes of two (u1 kept on chip, tiles overlapping by a
    row and a cell) give the bits of one sweep per pass, across x tiles
    (ragged at nx = 300, 260), y tiles of 14 rows and z tiles of 64 planes,
    with a coefficient grid and with a constant coefficient."""
    from paper_2404_14691_amd import sage as S
    nz, ny, nx = shape
    c = np.random.default_rng(6).uniform(0.1, 1.0, shape).astype(np.float32)
    fields = np.stack([synth.stencil_field(0, j, seed=6, shape=shape) for j in range(2)])
    outs = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("SAGE_STENCIL_FUSE", fuse)
        ctx = sage_ctx_factory(pool_budget_bytes=64 << 20)
        res = []
        kinds = [(S.relax_desc(nx, ny, nz, sweeps, 0.6), [])]
        if nx & (nx - 1) == 0:  # the coefficient-grid kind needs a power-of-two nx
            kinds.insert(0, (S.stencil_desc(nx, ny, nz, sweeps), [S.make_blob(c)]))
        for desc, blobs in kinds:
            fn = S.fn_register(ctx, desc, blobs)
            inv = S.fn_setup(ctx, fn, 2)
            out = np.zeros_like(fields)
            S.fn_invoke(ctx, inv, fields, out)
            S.fn_release(ctx, inv)
            S.fn_unregister(ctx, fn)
            res.append(out)
        outs[fuse] = res
    for a, b in zip(outs["1"], outs["0"]):
        assert np.array_equal(a, b)
    cg = np.full(shape, 0.6, dtype=np.float32)
    for j in range(2):
        assert OS.normwise_error(outs["1"][-1][j], OS.jacobi7(fields[j], cg, sweeps)) <= F32_TOL


def test_stencil_zero_coefficient_identity(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    shape = (10, 12, 64)
    c = np.zeros(shape, dtype=np.float32)
    fn = S.fn_register(ctx, S.stencil_desc(64, 12, 10, 3), [S.make_blob(c)])
    u = synth.stencil_field(0, 0, seed=2, shape=shape)
    inv = S.fn_setup(ctx, fn, 1)
    out = np.zeros_like(u)
    S.fn_invoke(ctx, inv, u, out)
    S.fn_release(ctx, inv)
    assert np.array_equal(out, u)


@pytest.mark.parametrize("shape,sweeps,coef", [((7, 9, 20), 3, 0.7), ((4, 5, 8), 1, 1.0), ((18, 20, 300), 4, 0.35),
                                               ((66, 33, 260), 2, 0.5)])
def test_relax_vs_oracle_and_plain(sage_ctx_factory, torch_cuda, shape, sweeps, coef):
    """The relaxation kind has no read-only data: it registers with no blobs
    and its sweep uses one constant coefficient.  Shared and plain contexts
    run the same work and return the same bits; both match the oracle's
    Jacobi sweeps with a constant coefficient grid (nx = 300 spans two
    256-cell x tiles and a ragged one)."""
    from paper_2404_14691_amd import sage as S
    nz, ny, nx = shape
    desc = S.relax_desc(nx, ny, nz, sweeps, coef)
    fields = np.stack([synth.stencil_field(0, j, seed=3, shape=shape) for j in range(2)])
    results = []
    for share in (1, 0):
        ctx = sage_ctx_factory(share=share)
        fn = S.fn_register(ctx, desc, [])
        assert S.sage_fn_block_count(ctx, fn) == 0
        inv = S.fn_setup(ctx, fn, 2)
        out = np.zeros_like(fields)
        S.fn_invoke(ctx, inv, fields, out)
        S.fn_release(ctx, inv)
        S.fn_unregister(ctx, fn)
        results.append(out)
    assert np.array_equal(results[0], results[1])
    cgrid = np.full(shape, coef, dtype=np.float32)
    for j in range(2):
        assert OS.normwise_error(results[0][j], OS.jacobi7(fields[j], cgrid, sweeps)) <= F32_TOL


def test_relax_rejects_read_only_blobs(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    blob = np.zeros(1024, dtype=np.float32)
    with pytest.raises(S.SageError):
        S.fn_register(ctx, S.relax_desc(8, 4, 4, 1, 0.5), [S.make_blob(blob)])
    with pytest.raises(S.SageError):
        S.fn_register(ctx, S.relax_desc(6, 4, 4, 1, 0.5), [])  # nx not a multiple of 4


def test_f32_four_and_eight_columns_per_workgroup_same_bits(sage_ctx_factory, torch_cuda, monkeypatch):
    """The FP32 layer with four output columns per workgroup (SAGE_F32_COLS=4)
    splits each column's K over the lanes and waves as with eight and sums
    the partial sums along the same exchange tree: the same bits, one group
    and two groups (the last column of the last layer included).  A one-group
    launch passes its group by value, a two-group one reads the groups from
    the launch header: the solo run against the batch compares the two."""
    from paper_2404_14691_amd import sage as S
    W, L = 1024, 2
    rng = np.random.default_rng(8)
    ws = [(rng.standard_normal((L, W, W)) / np.sqrt(W)).astype(np.float32) for _ in range(2)]
    xs = [rng.standard_normal((b, W)).astype(np.float32) for b in (8, 11)]
    outs = {}
    for cols in ("8", "4"):
        monkeypatch.setenv("SAGE_F32_COLS", cols)
        ctx = sage_ctx_factory(pool_budget_bytes=64 << 20)
        fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_F32, L, W), [S.make_blob(w)]) for w in ws]
        invs = [S.fn_setup(ctx, f, len(x)) for f, x in zip(fns, xs)]
        ys = [np.zeros((len(x), W), dtype=np.float32) for x in xs]
        S.fn_invoke_batch(ctx, invs, xs, ys)
        solo = np.zeros((len(xs[0]), W), dtype=np.float32)
        S.fn_invoke(ctx, invs[0], xs[0], solo)
        for inv in invs:
            S.fn_release(ctx, inv)
        assert np.array_equal(solo, ys[0])
        outs[cols] = ys
    for a, b in zip(outs["8"], outs["4"]):
        assert np.array_equal(a, b)
    for w, x, y in zip(ws, xs, outs["4"]):
        assert OM.normwise_error(y, OM.mlp_forward(x, w.astype(np.float64))) <= F32_TOL
