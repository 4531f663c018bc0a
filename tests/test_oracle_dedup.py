"""Pins for the dedup oracle: brute-force byte comparison (no fingerprint)
against the indexed method, planted duplicates with closed-form counts, and
forced fingerprint collisions."""
import numpy as np
import pytest

from oracle import dedup as D
from oracle import fingerprint as F
from paper_2404_14691_amd import synth


def _fp_py(data: bytes) -> int:
    return F.fp64k_py(data)


def test_planted_duplicates_closed_form():
    B = 64
    # fn0: 10 blocks, block 7 = block 2, block 9 = block 2; zero blocks 4 and 5
    a = synth.blob_with_duplicates(10, B, [(7, 2), (9, 2)], seed=1, zero_blocks=(4, 5))
    # fn1: 6 blocks + 10-byte tail; block 1 = fn0 block 3 (planted below), block 5 zero
    b = synth.blob_with_duplicates(6, B, [], seed=2, tail=10, zero_blocks=(5,))
    b[1 * B:2 * B] = a[3 * B:4 * B]
    canon = D.partition_bruteforce([a, b], B)
    assert canon[0][7] == (0, 2) and canon[0][9] == (0, 2)
    assert canon[0][5] == (0, 4) and canon[1][5] == (0, 4)
    assert canon[1][1] == (0, 3)
    acc = D.accounting([a, b], B, canon)
    n_logical_blocks = 10 + 7
    assert acc["n_blocks"] == n_logical_blocks
    # classes: fn0 has 10 - 2 (dups of 2) - 1 (zero 5 joins 4) = 7 classes;
    # fn1 adds 7 blocks - 1 (block1) - 1 (zero) = 5 new classes
    assert acc["n_classes"] == 12
    assert acc["logical"] == 16 * B + 10
    assert acc["unique"] == 11 * B + 10
    # shared blocks: {2,7,9}, {4,5,fn1:5}, {3, fn1:1}
    assert acc["shared"] == 8 * B
    assert acc["shared"] + acc["private"] == acc["logical"]


@pytest.mark.parametrize("seed", range(5))
def test_indexed_equals_bruteforce_random(seed):
    rng = np.random.default_rng(seed)
    B = 64
    blobs = []
    pool = [rng.integers(0, 256, B, dtype=np.uint8) for _ in range(6)]
    for f in range(3):
        nb = int(rng.integers(1, 12))
        tail = int(rng.integers(0, B))
        buf = rng.integers(0, 256, nb * B + tail, dtype=np.uint8)
        for k in range(nb):
            if rng.random() < 0.5:
                buf[k * B:(k + 1) * B] = pool[int(rng.integers(0, len(pool)))]
        blobs.append(buf)
    brute = D.partition_bruteforce(blobs, B)
    assert D.partition_indexed(blobs, B, _fp_py) == brute
    assert D.partition_dict(blobs, B) == brute
    acc = D.accounting(blobs, B, brute)
    assert acc["shared"] + acc["private"] == acc["logical"]


def test_forced_collisions_keep_partition():
    rng = np.random.default_rng(11)
    B = 32
    blobs = [rng.integers(0, 4, 8 * B, dtype=np.uint8) for _ in range(3)]
    blobs[1][:B] = blobs[0][B:2 * B]
    brute = D.partition_bruteforce(blobs, B)
    # every block gets the same fingerprint: only byte verification separates them
    assert D.partition_indexed(blobs, B, lambda d: 42) == brute
    # two-valued fingerprint: chains of length > 1 on both values
    assert D.partition_indexed(blobs, B, lambda d: d[0] & 1) == brute


def test_tail_blocks_compare_length_and_bytes():
    B = 16
    a = np.zeros(B + 4, dtype=np.uint8)       # full zero block + 4-byte zero tail
    b = np.zeros(4, dtype=np.uint8)           # a lone 4-byte zero block
    canon = D.partition_bruteforce([a, b], B)
    assert canon[0][1] == (0, 1) and canon[1][0] == (0, 1)
    assert canon[0][0] == (0, 0)
    assert D.accounting([a, b], B, canon)["unique"] == B + 4


def test_empty_blob_has_no_blocks():
    canon = D.partition_bruteforce([np.zeros(0, dtype=np.uint8)], 64)
    assert canon == [[]]
    acc = D.accounting([np.zeros(0, dtype=np.uint8)], 64, canon)
    assert acc["logical"] == acc["unique"] == acc["n_blocks"] == 0


def test_shared_mlp_functions_closed_form_small():
    # generator plants floor(0.3 * n_blocks) common block indices
    w = synth.shared_mlp_bf16_functions(n_fns=4, layers=2, width=512, share_frac=0.3, seed=0)
    n = w.n_blocks
    assert n == 2 * 512 * 512 * 2 // 65536
    k = int(np.floor(0.3 * n))
    canon = D.partition_dict(w.blobs, 65536)
    acc = D.accounting(w.blobs, 65536, canon)
    assert acc["n_classes"] == k + 4 * (n - k)
    assert acc["unique"] == (k + 4 * (n - k)) * 65536
    assert acc["shared"] == 4 * k * 65536
    assert D.partition_indexed(w.blobs, 65536, lambda d: int(F.fp64k_blob(np.frombuffer(d, np.uint8))[0])) == canon
