"""Parity of the data-movement kernels called through the C ABI: FP64K-v1
fingerprints (bit-exact vs the oracle) and block COPY / VERIFY."""
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)
import numpy as np
import pytest

from oracle import fingerprint as OF

pytestmark = pytest.mark.gpu


def _dev(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


@pytest.mark.parametrize("nbytes", [1, 7, 8, 9, 4095, 65535, 65536, 65537, 3 * 65536 + 1000, 300 * 65536])
def test_fingerprint_parity(sage_ctx_factory, torch_cuda, nbytes):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    rng = np.random.default_rng(nbytes)
    data = rng.integers(0, 256, nbytes, dtype=np.uint8)
    if nbytes >= 3 * 65536:
        data[65536:2 * 65536] = 0                  # a zero block
        data[2 * 65536:3 * 65536] = np.arange(65536) & 0xFF
    nblk = -(-nbytes // 65536)
    d = _dev(torch, data)
    out = torch.zeros(nblk, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    S.sage_fingerprint(ctx, d.data_ptr(), nbytes, out.data_ptr(), s)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, OF.fp64k_blob(data))


def test_fingerprint_equal_blocks_equal_values(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    rng = np.random.default_rng(9)
    blk = rng.integers(0, 256, 65536, dtype=np.uint8)
    data = np.concatenate([blk, blk, blk ^ np.uint8(1), blk])
    d = _dev(torch, data)
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    S.sage_fingerprint(ctx, d.data_ptr(), data.size, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    fp = out.cpu().numpy().view(np.uint64)
    assert fp[0] == fp[1] == fp[3] and fp[2] != fp[0]


def test_blkcopy_copy_and_verify(sage_ctx_factory, torch_cuda):
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    rng = np.random.default_rng(3)
    nsrc = 6
    src = rng.integers(0, 256, nsrc * 65536, dtype=np.uint8)
    src[65536 + 1000] = 0x5A                       # differs from the 0xA5 fill below
    dsrc = _dev(torch, src)
    dst = torch.full((nsrc * 65536,), 0xA5, dtype=torch.uint8, device="cuda")
    lens = [65536, 1000, 17, 65535, 65536, 16]
    ops = np.zeros(nsrc, dtype=[("src", "<u8"), ("dst", "<u8"), ("len", "<u4"), ("op", "<u4")])
    for i, L in enumerate(lens):
        ops[i] = (dsrc.data_ptr() + i * 65536, dst.data_ptr() + ((i + 2) % nsrc) * 65536, L, S.SAGE_OP_COPY)
    dops = _dev(torch, ops.view(np.uint8))
    res = torch.zeros(nsrc, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    S.sage_blkcopy(ctx, dops.data_ptr(), nsrc, res.data_ptr(), stream)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    for i, L in enumerate(lens):
        o = ((i + 2) % nsrc) * 65536
        assert np.array_equal(out[o:o + L], src[i * 65536:i * 65536 + L])
        assert np.all(out[o + L:o + 65536] == 0xA5)
    # VERIFY: equal spans -> 0, a one-byte difference -> 1 (also in a short tail)
    vops = np.zeros(4, dtype=ops.dtype)
    vops[0] = (dsrc.data_ptr(), dst.data_ptr() + 2 * 65536, 65536, S.SAGE_OP_VERIFY)
    vops[1] = (dsrc.data_ptr() + 65536, dst.data_ptr() + 3 * 65536, 1000, S.SAGE_OP_VERIFY)
    vops[2] = (dsrc.data_ptr() + 65536, dst.data_ptr() + 3 * 65536, 1001, S.SAGE_OP_VERIFY)
    vops[3] = (dsrc.data_ptr(), dst.data_ptr() + 3 * 65536, 65536, S.SAGE_OP_VERIFY)
    dv = _dev(torch, vops.view(np.uint8))
    res = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    S.sage_blkcopy(ctx, dv.data_ptr(), 4, res.data_ptr(), stream)
    torch.cuda.synchronize()
    assert res.cpu().tolist() == [0, 0, 1, 1]


def test_blkcopy_launch_larger_than_one_wave(sage_ctx_factory, torch_cuda):
    """More operations than one wave of workgroups (32 per CU): the launch
    takes blocks two at a time, full-block COPY pairs on the fast path and
    partial COPYs and VERIFYs mixed in; every destination block is checked."""
    from paper_2404_14691_amd import sage as S
    torch = torch_cuda
    ctx = sage_ctx_factory()
    n = torch.cuda.get_device_properties(0).multi_processor_count * 32 + 37
    rng = np.random.default_rng(11)
    nsrc = 64
    src = rng.integers(0, 256, nsrc * 65536, dtype=np.uint8)
    dsrc = _dev(torch, src)
    dst = torch.full((n * 65536,), 0xA5, dtype=torch.uint8, device="cuda")
    ops = np.zeros(n, dtype=[("src", "<u8"), ("dst", "<u8"), ("len", "<u4"), ("op", "<u4")])
    kind = np.zeros(n, dtype=np.int64)  # 0 full COPY, 1 partial COPY, 2 VERIFY equal, 3 VERIFY different
    for i in range(n):
        j = i % nsrc
        if i % 97 == 5:
            kind[i] = 2
            ops[i] = (dsrc.data_ptr() + j * 65536, dsrc.data_ptr() + j * 65536, 65536, S.SAGE_OP_VERIFY)
        elif i % 97 == 6:
            kind[i] = 3
            ops[i] = (dsrc.data_ptr() + j * 65536, dsrc.data_ptr() + ((j + 1) % nsrc) * 65536, 65536,
                      S.SAGE_OP_VERIFY)
        elif i % 89 == 7:
            kind[i] = 1
            ops[i] = (dsrc.data_ptr() + j * 65536, dst.data_ptr() + i * 65536, 1000, S.SAGE_OP_COPY)
        else:
            ops[i] = (dsrc.data_ptr() + j * 65536, dst.data_ptr() + i * 65536, 65536, S.SAGE_OP_COPY)
    dops = _dev(torch, ops.view(np.uint8))
    res = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    S.sage_blkcopy(ctx, dops.data_ptr(), n, res.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = dst.cpu().numpy().reshape(n, 65536)
    blocks = src.reshape(nsrc, 65536)
    r = res.cpu().numpy()
    for i in range(n):
        j = i % nsrc
        if kind[i] == 0:
            assert np.array_equal(out[i], blocks[j]), i
        elif kind[i] == 1:
            assert np.array_equal(out[i, :1000], blocks[j, :1000]) and np.all(out[i, 1000:] == 0xA5), i
        else:
            assert np.all(out[i] == 0xA5), i
            assert r[i] == (0 if kind[i] == 2 else 1), i


def test_mfma_ceiling_measurement(sage_ctx_factory, torch_cuda):
    """The compute-side ceiling measurement of the main GEMM tile runs,
    reports a positive time and a plausible shader clock, and scales with K;
    bad arguments are EINVAL."""
    from paper_2404_14691_amd import sage as S
    ctx = sage_ctx_factory()
    us_4k, ghz = S.sage_mfma_ceiling(ctx, 4096, 5)
    us_1k, _ = S.sage_mfma_ceiling(ctx, 1024, 5)
    assert us_4k > 0 and us_1k > 0
    assert 0.5 < ghz < 3.0, ghz
    assert us_4k > 2 * us_1k  # four times the MFMAs: well over twice the time
    for k, reps in ((0, 1), (33, 1), (4096, 0), (4096, 1001)):
        with pytest.raises(S.SageError) as e:
            S.sage_mfma_ceiling(ctx, k, reps)
        assert e.value.status == S.SAGE_EINVAL
