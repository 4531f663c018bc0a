"""Pins for the FP64K-v1 oracle: published splitmix64 values, closed forms on
constructed blocks, agreement of two implementations, and sensitivity."""
import json
import os

import numpy as np
import pytest

from oracle import fingerprint as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_mix64_reproduces_published_splitmix64():
    ref = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))["outputs_hex"]
    got = ["%016x" % v for v in F.splitmix64(0, len(ref))]
    assert got == ref


def test_keys_are_odd_and_sized():
    for k in (F.K0, F.K1, F.K2, F.K3):
        assert 0 < k < 2**32 and k & 1
    assert 0 < F.K4 < 2**64 and F.K4 & 1


def _block_with_keyed_halves(n_words, lo_target, hi_target):
    """Block whose keyed halves (lo_j + a_j) and (hi_j + c_j) equal the given
    per-word targets mod 2^32, built by subtracting the keys."""
    out = bytearray()
    for j in range(n_words):
        a = (F.K0 + j * F.K1) & F.M32
        c = (F.K2 + j * F.K3) & F.M32
        lo = (lo_target(j) - a) & F.M32
        hi = (hi_target(j) - c) & F.M32
        out += ((hi << 32) | lo).to_bytes(8, "little")
    return bytes(out)


@pytest.mark.parametrize("n_words", [1, 3, 8192])
def test_closed_form_zero_sum(n_words):
    # keyed low half 0 for every word -> S = 0 whatever the high halves
    blk = _block_with_keyed_halves(n_words, lambda j: 0, lambda j: (j * 2654435761) & F.M32)
    L = 8 * n_words
    assert F.nh_sum_py(blk) == 0
    assert F.fp64k_py(blk) == F.mix64((L * F.K4) & F.M64)


@pytest.mark.parametrize("n_words", [1, 5, 8192])
def test_closed_form_unit_products(n_words):
    blk = _block_with_keyed_halves(n_words, lambda j: 1, lambda j: 1)
    assert F.nh_sum_py(blk) == n_words


def test_closed_form_distinguishes_halves():
    # keyed (lo, hi) = (2, 3): S = 6n.  Building it with the roles of the two
    # halves swapped must not give 6n, so a swapped key assignment fails.
    n = 64
    blk = _block_with_keyed_halves(n, lambda j: 2, lambda j: 3)
    assert F.nh_sum_py(blk) == 6 * n
    swapped = bytearray()
    for j in range(n):
        a = (F.K0 + j * F.K1) & F.M32
        c = (F.K2 + j * F.K3) & F.M32
        lo = (2 - c) & F.M32
        hi = (3 - a) & F.M32
        swapped += ((hi << 32) | lo).to_bytes(8, "little")
    assert F.nh_sum_py(bytes(swapped)) != 6 * n


def test_closed_form_wraps_mod_2_64():
    # every keyed product is (2^32-1)^2; 8192 of them wrap mod 2^64
    n = 8192
    m = F.M32
    blk = _block_with_keyed_halves(n, lambda j: m, lambda j: m)
    assert F.nh_sum_py(blk) == (n * m * m) & F.M64


def test_single_word_delta():
    # changing word j changes S by exactly the difference of its keyed product
    rng = np.random.default_rng(1)
    blk = bytearray(rng.integers(0, 256, 4096, dtype=np.uint8).tobytes())
    j = 137
    w_old = int.from_bytes(blk[8 * j:8 * j + 8], "little")
    w_new = w_old ^ (1 << 45)
    a = (F.K0 + j * F.K1) & F.M32
    c = (F.K2 + j * F.K3) & F.M32

    def prod(w):
        return (((w & F.M32) + a) & F.M32) * (((w >> 32) + c) & F.M32)
    s0 = F.nh_sum_py(bytes(blk))
    blk[8 * j:8 * j + 8] = w_new.to_bytes(8, "little")
    assert F.nh_sum_py(bytes(blk)) == (s0 - prod(w_old) + prod(w_new)) & F.M64


@pytest.mark.parametrize("L", [1, 7, 8, 9, 15, 16, 17, 4095, 65535, 65536])
def test_python_and_numpy_agree_edge_lengths(L):
    rng = np.random.default_rng(L)
    b = rng.integers(0, 256, L, dtype=np.uint8)
    ref = F.fp64k_py(b.tobytes())
    assert int(F.fp64k_blob(b)[0]) == ref


def test_python_and_numpy_agree_multi_block_with_tail():
    rng = np.random.default_rng(7)
    b = rng.integers(0, 256, 3 * 65536 + 1000, dtype=np.uint8)
    b[65536:2 * 65536] = 0                       # a zero block
    got = F.fp64k_blob(b)
    want = [F.fp64k_py(b[o:o + 65536].tobytes()) for o in range(0, b.size, 65536)]
    assert [int(x) for x in got] == want


def test_ramp_block():
    b = (np.arange(65536) & 0xFF).astype(np.uint8)
    assert int(F.fp64k_blob(b)[0]) == F.fp64k_py(b.tobytes())


def test_length_is_mixed_in():
    # same padded words, different lengths -> different fingerprints
    base = bytes(range(1, 8)) + b"\0"
    assert F.nh_sum_py(base[:7]) == F.nh_sum_py(base)
    assert F.fp64k_py(base[:7]) != F.fp64k_py(base)
    z = bytes(65536)
    assert F.fp64k_py(z[:65528]) != F.fp64k_py(z)


def test_equal_content_equal_fp():
    rng = np.random.default_rng(3)
    b = rng.integers(0, 256, 65536, dtype=np.uint8)
    two = np.concatenate([b, b])
    fp = F.fp64k_blob(two)
    assert fp[0] == fp[1]


def test_single_bit_flips_change_fp():
    rng = np.random.default_rng(4)
    base = rng.integers(0, 256, 65536, dtype=np.uint8)
    n = 10000
    blocks = np.repeat(base[None, :], 64, axis=0)
    ref = F.fp64k_blob(base)[0]
    changed = 0
    for start in range(0, n, 64):
        m = min(64, n - start)
        bb = blocks[:m].copy()
        pos = rng.integers(0, 65536 * 8, m)
        for i, p in enumerate(pos):
            bb[i, p // 8] ^= np.uint8(1 << (p % 8))
        fps = F.fp64k_full_blocks(bb.view(np.uint64).reshape(m, 8192))
        changed += int(np.sum(fps != ref))
    assert changed == n


def test_reduction_order_irrelevant():
    rng = np.random.default_rng(5)
    w = rng.integers(0, 2**63, 8192, dtype=np.int64).astype(np.uint64)
    lo, hi = w & np.uint64(F.M32), w >> np.uint64(32)
    with np.errstate(over="ignore"):
        p = ((lo + F._A) & np.uint64(F.M32)) * ((hi + F._C) & np.uint64(F.M32))
        s1 = int(p.sum(dtype=np.uint64))
        s2 = int(p[rng.permutation(8192)].reshape(64, 128).sum(axis=0, dtype=np.uint64).sum(dtype=np.uint64))
    assert s1 == s2
