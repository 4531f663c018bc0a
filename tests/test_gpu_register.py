"""Parity of fn_register's data path: fingerprints, the dedup partition and
the bytes in the pool are bit-exact against the oracle; the byte accounting
matches its closed forms; host (pageable, pinned) and device sources agree;
forced fingerprint collisions still give the byte-exact partition."""
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)
import os

import numpy as np
import pytest

from oracle import dedup as OD
from oracle import fingerprint as OF
from paper_2404_14691_amd import synth

pytestmark = pytest.mark.gpu

WIDTH, LAYERS = 512, 4          # 2 MiB blobs = 32 blocks


def _blobs():
    w = synth.shared_mlp_bf16_functions(n_fns=3, layers=LAYERS, width=WIDTH, share_frac=0.3, seed=5)
    blobs = [b.copy() for b in w.blobs]
    per = 65536 // 2
    blobs[1][5 * per:6 * per] = blobs[1][2 * per:3 * per]     # duplicate inside one chunk pair
    blobs[1][3 * per:4 * per] = blobs[1][2 * per:3 * per]     # same chunk as block 2 (chunk = 4 blocks)
    blobs[2][7 * per:8 * per] = 0
    blobs[0][30 * per:31 * per] = 0                           # zero block in two functions
    blobs[2][31 * per:32 * per] = blobs[0][1 * per:2 * per]   # cross-function duplicate
    return blobs


def _register(S, ctx, blobs, where, torch=None, keep=None):
    fns = []
    for b in blobs:
        if where == "host":
            blob = S.make_blob(b)
        elif where == "pinned":
            arr = S.pinned_array(ctx, b.shape, b.dtype)
            arr[:] = b
            keep.append(arr)
            blob = S.make_blob(arr)
        else:
            d = torch.from_numpy(b.view(np.uint8)).cuda()
            torch.cuda.synchronize()
            keep.append(d)
            blob = S.make_blob(d.data_ptr(), b.nbytes, where=S.SAGE_SRC_DEVICE)
        fns.append(S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH), [blob]))
    return fns


def _check_against_oracle(S, ctx, fns, blobs, read_bytes=True):
    for f, b in zip(fns, blobs):
        assert np.array_equal(S.sage_fn_fingerprints(ctx, f), OF.fp64k_blob(b))
    canon = OD.partition_dict(blobs, 65536)
    lib_canon = []
    for f in fns:
        cls, slot, refs = S.sage_fn_block_info(ctx, f)
        lib_canon.append([(int(c),) for c in cls])
        assert np.all(slot != 0xFFFFFFFF) and np.all(refs == 0)
    assert OD.same_partition(canon, lib_canon)
    if read_bytes:
        for f, b in zip(fns, blobs):
            raw = b.view(np.uint8)
            _, slot, _ = S.sage_fn_block_info(ctx, f)
            for k, s in enumerate(slot):
                assert np.array_equal(S.sage_read_slot(ctx, int(s)), raw[k * 65536:(k + 1) * 65536]), (f, k)
    acc = OD.accounting(blobs, 65536, canon)
    st = S.sage_get_stats(ctx)
    assert st["logical_bytes"] == acc["logical"]
    assert st["unique_bytes"] == acc["unique"]
    assert st["shared_bytes"] == acc["shared"]
    assert st["private_bytes"] == acc["private"]
    assert st["shared_bytes"] + st["private_bytes"] == st["logical_bytes"]
    assert st["classes"] == acc["n_classes"]
    assert st["resident_bytes"] == acc["unique"]
    assert st["h2d_bytes"] == acc["logical"]


@pytest.mark.parametrize("where", ["host", "pinned", "device"])
def test_register_partition_and_bytes(sage_ctx_factory, torch_cuda, where):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory(chunk_bytes=256 << 10, ring_slots=3, streams=2)
    blobs = _blobs()
    keep = []
    fns = _register(S, ctx, blobs, where, torch_cuda, keep)
    _check_against_oracle(S, ctx, fns, blobs)
    for f in fns:
        S.fn_unregister(ctx, f)
    st = S.sage_get_stats(ctx)
    assert st["classes"] == 0 and st["resident_slots"] == 0 and st["logical_bytes"] == 0
    for a in keep:
        if isinstance(a, np.ndarray):
            S.sage_host_free(ctx, a.ctypes.data)


def test_register_serial_and_unpipelined_agree(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    blobs = _blobs()
    results = []
    for over in ({"serial_setup": 1}, {"ring_slots": 1, "streams": 1, "chunk_bytes": 65536}):
        ctx = sage_ctx_factory(**over)
        fns = _register(S, ctx, blobs, "host")
        _check_against_oracle(S, ctx, fns, blobs, read_bytes=False)
        results.append([S.sage_fn_fingerprints(ctx, f) for f in fns])
    for a, b in zip(*results):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("where", ["host", "device", "device-batch"])
def test_forced_fingerprint_collisions(sage_ctx_factory, torch_cuda, monkeypatch, where):
    """Every fingerprint forced to one value: only byte verification keeps
    blocks apart, and the partition is still the byte-exact one (staged
    chunks settle their VERIFYs chunk by chunk; device sources at the end of
    the registration, after counting the blocks in optimistically; in one
    fn_register_batch call, while the next function's fingerprints are
    already out)."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    monkeypatch.setenv("SAGE_TEST_FP_CONST", "12345")
    # three slots for the batch: one function's chunk in flight, the next one's fingerprinted ahead, one free
    ctx = sage_ctx_factory(chunk_bytes=256 << 10, ring_slots=3 if where == "device-batch" else 2)
    monkeypatch.delenv("SAGE_TEST_FP_CONST")
    # BF16 MLP of width 256 and 8 layers: 1 MiB = the first 16 blocks of each blob
    blobs = [np.ascontiguousarray(b[: 8 * 256 * 256]) for b in _blobs()]
    dev = where.startswith("device")
    keep = [torch.from_numpy(b.view(np.uint8)).cuda() for b in blobs] if dev else []
    torch.cuda.synchronize()
    srcs = [S.make_blob(d.data_ptr(), d.numel(), where=S.SAGE_SRC_DEVICE) for d in keep] if dev \
        else [S.make_blob(b) for b in blobs]
    desc = S.mlp_desc(S.SAGE_MLP_BF16, 8, 256)
    if where == "device-batch":
        fns, _ = S.fn_register_batch(ctx, [desc] * len(srcs), [[s_] for s_ in srcs])
    else:
        fns = [S.fn_register(ctx, desc, [s_]) for s_ in srcs]
    canon = OD.partition_dict(blobs, 65536)
    lib = [[(int(c),) for c in S.sage_fn_block_info(ctx, f)[0]] for f in fns]
    assert OD.same_partition(canon, lib)
    st = S.sage_get_stats(ctx)
    assert st["verify_mismatches"] > 0
    for f, b in zip(fns, blobs):
        raw = b.view(np.uint8)
        _, slot, _ = S.sage_fn_block_info(ctx, f)
        for k, s in enumerate(slot):
            assert np.array_equal(S.sage_read_slot(ctx, int(s)), raw[k * 65536:(k + 1) * 65536])


def test_register_rejects_bad_layouts(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    b = np.zeros(256 * 256, dtype=np.uint16)
    with pytest.raises(S.SageError) as e:
        S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 2, 256), [S.make_blob(b)])
    assert e.value.status == S.SAGE_EINVAL
    with pytest.raises(S.SageError) as e:
        S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 1, 384), [S.make_blob(np.zeros(384 * 384, np.uint16))])
    assert e.value.status == S.SAGE_EINVAL
    with pytest.raises(S.SageError) as e:
        S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 1, 256), [S.make_blob(b, access=S.SAGE_RW)])
    assert e.value.status == S.SAGE_EINVAL
    with pytest.raises(S.SageError) as e:
        S.fn_setup(ctx, 999999, 1)
    assert e.value.status == S.SAGE_ENOTFOUND


@pytest.mark.parametrize("chunk", [64 << 20, None])
def test_device_source_across_chunks(sage_ctx_factory, torch_cuda, monkeypatch, chunk):
    """A 160 MiB device source is fingerprinted in three 64 MiB chunks (or in
    one, the default chunk size); blocks equal
    to blocks of earlier chunks (still being copied from the source) and to
    another function's blocks join their classes; fingerprints, partition,
    accounting and sampled slot bytes match the oracle."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    layers, width = 5, 4096                      # 5 x 32 MiB = 2560 blocks
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=layers, width=width, share_frac=0.1, seed=9)
    blobs = [b.copy() for b in w.blobs]
    per = 65536 // 2
    planted = [(1500, 10), (2100, 10), (2500, 1100), (1030, 1029)]   # (copy, original): across chunks
    for dst, src in planted:
        blobs[0][dst * per:(dst + 1) * per] = blobs[0][src * per:(src + 1) * per]
    blobs[0][30 * per:31 * per] = 0
    blobs[0][2300 * per:2301 * per] = 0
    blobs[1][700 * per:701 * per] = blobs[0][2200 * per:2201 * per]    # the second function joins a late class
    if chunk:
        monkeypatch.setenv("SAGE_DEV_CHUNK_BYTES", str(chunk))
    ctx = sage_ctx_factory(pool_budget_bytes=1 << 30)
    dev = [torch.from_numpy(b.view(np.uint8)).cuda() for b in blobs]
    torch.cuda.synchronize()
    desc = S.mlp_desc(S.SAGE_MLP_BF16, layers, width)
    fns = [S.fn_register(ctx, desc, [S.make_blob(d.data_ptr(), d.numel(), where=S.SAGE_SRC_DEVICE)]) for d in dev]
    for f, b in zip(fns, blobs):
        assert np.array_equal(S.sage_fn_fingerprints(ctx, f), OF.fp64k_blob(b))
    canon = OD.partition_dict(blobs, 65536)
    info = [S.sage_fn_block_info(ctx, f) for f in fns]
    assert OD.same_partition(canon, [[(int(c),) for c in cls] for cls, _, _ in info])
    cls0 = info[0][0]
    for dst, src in planted:
        assert cls0[dst] == cls0[src]
    assert cls0[30] == cls0[2300] and info[1][0][700] == cls0[2200]
    acc = OD.accounting(blobs, 65536, canon)
    st = S.sage_get_stats(ctx)
    assert st["unique_bytes"] == acc["unique"] and st["classes"] == acc["n_classes"]
    rng = np.random.default_rng(9)
    for fi, b in enumerate(blobs):
        raw = b.view(np.uint8)
        slots = info[fi][1]
        picks = sorted(set(rng.choice(len(slots), 48, replace=False).tolist()) | {d for d, _ in planted} | {30, 2300})
        for k in picks:
            assert np.array_equal(S.sage_read_slot(ctx, int(slots[k])), raw[k * 65536:(k + 1) * 65536]), (fi, k)
    for f in fns:
        S.fn_unregister(ctx, f)



def _source(S, ctx, b, where, torch, keep):
    if where == "host":
        return S.make_blob(b)
    if where == "pinned":
        arr = S.pinned_array(ctx, b.shape, b.dtype)
        arr[:] = b
        keep.append(arr)
        return S.make_blob(arr)
    d = torch.from_numpy(b.view(np.uint8)).cuda()
    torch.cuda.synchronize()
    keep.append(d)
    return S.make_blob(d.data_ptr(), b.nbytes, where=S.SAGE_SRC_DEVICE)


@pytest.mark.parametrize("mix,dev_chunk", [("device", None), ("device", "524288"), ("mixed", None)])
def test_register_batch_matches_oracle_and_one_by_one(sage_ctx_factory, torch_cuda, monkeypatch, mix, dev_chunk):
    """fn_register_batch: fingerprints, the dedup partition, the pool bytes and
    the accounting bit-exact against the oracle, and every function's outputs
    the same bits as after one-by-one registration.  Device sources are
    fingerprinted ahead of the previous function's classification (with
    512 KiB device chunks the later functions find too few free ring slots
    and go one by one); a mix of device, pinned and pageable sources."""
    from paper_2404_14691_amd import sage as S
    from oracle import mlp as OM
    torch = torch_cuda
    if dev_chunk:
        monkeypatch.setenv("SAGE_DEV_CHUNK_BYTES", dev_chunk)
    blobs = _blobs()
    wheres = ["device"] * 3 if mix == "device" else ["device", "pinned", "host"]
    desc = S.mlp_desc(S.SAGE_MLP_BF16, LAYERS, WIDTH)
    outs = []
    for batch in (True, False):
        ctx = sage_ctx_factory(chunk_bytes=256 << 10, ring_slots=8 if dev_chunk else 3, streams=2)
        keep = []
        srcs = [[_source(S, ctx, b, w, torch, keep)] for b, w in zip(blobs, wheres)]
        if batch:
            fns, ms = S.fn_register_batch(ctx, [desc] * 3, srcs)
            assert len(set(fns)) == 3 and all(m > 0 for m in ms)
            _check_against_oracle(S, ctx, fns, blobs)
        else:
            fns = [S.fn_register(ctx, desc, s) for s in srcs]
        ys = []
        for i, f in enumerate(fns):
            x = synth.bf16_inputs(5, WIDTH, 6, i)
            inv = S.fn_setup(ctx, f, 5)
            y = np.zeros((5, WIDTH), dtype=np.float32)
            S.fn_invoke(ctx, inv, x, y)
            S.fn_release(ctx, inv)
            W = OM.bf16_to_f64(blobs[i]).reshape(LAYERS, WIDTH, WIDTH)
            assert OM.normwise_error(y, OM.mlp_forward(OM.bf16_to_f64(x), W)) <= 2e-2
            ys.append(y)
        outs.append(ys)
        for f in fns:
            S.fn_unregister(ctx, f)
        st = S.sage_get_stats(ctx)
        assert st["classes"] == 0 and st["logical_bytes"] == 0
        for a in keep:
            if isinstance(a, np.ndarray):
                S.sage_host_free(ctx, a.ctypes.data)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def _status(fn, *args):
    from paper_2404_14691_amd import sage as S
    try:
        fn(*args)
    except S.SageError as e:
        return e.status
    return S.SAGE_OK


def test_register_batch_all_or_nothing(sage_ctx_factory, torch_cuda):
    """A batch whose second function cannot be placed (the pool is held by a
    live setup of another function) fails with ENOMEM and leaves no function
    of the batch behind: the first one, already registered, is taken out
    again.  The held function is untouched and still computes; a batch that
    fits registers afterwards (the ring slots held for fingerprints taken
    ahead were given back)."""
    from paper_2404_14691_amd import sage as S
    from oracle import mlp as OM
    torch = torch_cuda
    ctx = sage_ctx_factory(pool_budget_bytes=48 * 65536)
    mk = lambda width, seed: synth.shared_mlp_bf16_functions(n_fns=1, layers=2, width=width, share_frac=0.0,
                                                             seed=seed).blobs[0]
    wa, wb, wc, wd = mk(512, 41), mk(256, 42), mk(1024, 43), mk(256, 44)  # 16, 4, 64 and 4 blocks
    fa = S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, 2, 512), [S.make_blob(wa)])
    inv = S.fn_setup(ctx, fa, 2)  # holds its 16 blocks: 32 of the 48 slots are left
    st0 = S.sage_get_stats(ctx)
    keep = []
    src = lambda w: [_source(S, ctx, w, "device", torch, keep)]
    descs = [S.mlp_desc(S.SAGE_MLP_BF16, 2, 256), S.mlp_desc(S.SAGE_MLP_BF16, 2, 1024)]
    assert _status(S.fn_register_batch, ctx, descs, [src(wb), src(wc)]) == S.SAGE_ENOMEM
    st1 = S.sage_get_stats(ctx)
    for k in ("logical_bytes", "unique_bytes", "classes", "resident_bytes", "refcount_sum", "live_setups"):
        assert st1[k] == st0[k], k
    x = synth.bf16_inputs(2, 512, 41, 0)
    y = np.zeros((2, 512), dtype=np.float32)
    S.fn_invoke(ctx, inv, x, y)
    W = OM.bf16_to_f64(wa).reshape(2, 512, 512)
    assert OM.normwise_error(y, OM.mlp_forward(OM.bf16_to_f64(x), W)) <= 2e-2
    fns, _ = S.fn_register_batch(ctx, [descs[0]] * 2, [src(wb), src(wd)])
    for f, w in zip(fns, (wb, wd)):
        assert np.array_equal(S.sage_fn_fingerprints(ctx, f), OF.fp64k_blob(w))
        S.fn_unregister(ctx, f)
    S.fn_release(ctx, inv)
    S.fn_unregister(ctx, fa)


def test_register_batch_evicts_an_earlier_function_of_the_batch(sage_ctx_factory, torch_cuda):
    """A batch whose last function only fits by evicting blocks of the
    functions registered before it in the same batch (48 slots for 16 + 16 +
    32 blocks from device sources): the copies gathered so far go out before
    that function is placed, so the evicted blocks are reloaded from their
    sources at setup.  Every fingerprint matches the oracle and every output
    equals the same function's output in a context whose pool holds all of
    them, within tolerance of the float64 oracle."""
    from paper_2404_14691_amd import sage as S
    from oracle import mlp as OM
    torch = torch_cuda
    mk = lambda layers, seed: synth.shared_mlp_bf16_functions(n_fns=1, layers=layers, width=512, share_frac=0.0,
                                                               seed=seed).blobs[0]
    ws = [(2, mk(2, 51)), (2, mk(2, 52)), (4, mk(4, 53))]  # 16, 16 and 32 blocks
    outs = {}
    for budget in (1 << 30, 48 * 65536):
        ctx = sage_ctx_factory(pool_budget_bytes=budget)
        keep = []
        descs = [S.mlp_desc(S.SAGE_MLP_BF16, L, 512) for L, _ in ws]
        fns, _ = S.fn_register_batch(ctx, descs, [[_source(S, ctx, w, "device", torch, keep)] for _, w in ws])
        for f, (_, w) in zip(fns, ws):
            assert np.array_equal(S.sage_fn_fingerprints(ctx, f), OF.fp64k_blob(w))
        ys = []
        for i, (f, (L, w)) in enumerate(zip(fns, ws)):
            x = synth.bf16_inputs(3, 512, 60 + i, 0)
            inv = S.fn_setup(ctx, f, 3)
            y = np.zeros((3, 512), dtype=np.float32)
            S.fn_invoke(ctx, inv, x, y)
            S.fn_release(ctx, inv)
            W = OM.bf16_to_f64(w).reshape(L, 512, 512)
            assert OM.normwise_error(y, OM.mlp_forward(OM.bf16_to_f64(x), W)) <= 2e-2
            ys.append(y)
        outs[budget] = ys
        if budget < (1 << 30):
            assert S.sage_get_stats(ctx)["evictions"] > 0
        for f in fns:
            S.fn_unregister(ctx, f)
    for a, b in zip(outs[1 << 30], outs[48 * 65536]):
        assert np.array_equal(a, b)


def test_register_batch_empty_and_null(sage_ctx_factory, torch_cuda):
    import ctypes as C
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    assert S.fn_register_batch(ctx, [], []) == ([], [])
    out = (C.c_uint64 * 1)()
    assert S._lib.fn_register_batch(ctx, 1, None, None, None, out, None) == S.SAGE_EINVAL
