"""Per-layer readiness of a reload, checked on the host against brute force:
layer l of an MLP body may start once every reloaded class used by a block
overlapping layers 0..l has landed.  The library reports, per layer, a prefix
of the reload order (classes by first block); the prefix must be exactly the
shortest one that holds all those classes."""
import numpy as np
import pytest

from paper_2404_14691_amd import sage as S

BLOCK = 65536


def _brute(block_class, missing, layers, layer_bytes):
    """Reload order and, per layer, the shortest prefix of it holding every
    missing class that a block of layers 0..l uses (by enumeration)."""
    first = {}
    for b, c in enumerate(block_class):
        first.setdefault(c, b)
    order = sorted(missing, key=lambda c: (first[c], c))
    rank = {c: i for i, c in enumerate(order)}
    ends = []
    need = set()
    for l in range(layers):
        lo = (l * layer_bytes) // BLOCK
        hi = ((l + 1) * layer_bytes - 1) // BLOCK
        need |= {block_class[b] for b in range(lo, hi + 1) if block_class[b] in rank}
        ends.append(max((rank[c] + 1 for c in need), default=0))
    ends[-1] = len(order)  # the last layer waits for the whole reload
    return [first[c] for c in order], ends


@pytest.mark.parametrize("seed", range(40))
def test_segments_match_brute_force(seed):
    rng = np.random.default_rng(seed)
    layers = int(rng.integers(1, 9))
    # layer sizes below, at and across block boundaries (small widths share blocks)
    layer_bytes = int(rng.choice([8 * 1024, 40 * 1024, BLOCK, 96 * 1024, 3 * BLOCK, 5 * BLOCK + 4096]))
    n_blocks = -(-layers * layer_bytes // BLOCK)
    # classes repeat within and across layers (equal blocks deduplicated)
    n_classes = int(rng.integers(1, n_blocks + 1))
    block_class = [int(c) for c in rng.integers(0, n_classes, n_blocks)]
    used = sorted(set(block_class))
    missing = [c for c in used if rng.random() < rng.choice([0.2, 0.6, 1.0])]
    first, ends = _brute(block_class, missing, layers, layer_bytes)
    got = S.sage_selftest_segments(first, layers, layer_bytes)
    assert got == ends, (layers, layer_bytes, block_class, missing)
    assert all(a <= b for a, b in zip(got, got[1:]))


def test_segments_of_a_4096_wide_bf16_function():
    """8 layers of 4096 x 4096 BF16 (32 MiB, 512 blocks each), every block its
    own class: layer l waits for exactly the first 512 (l + 1) classes."""
    first = list(range(8 * 512))
    assert S.sage_selftest_segments(first, 8, 4096 * 4096 * 2) == [512 * (l + 1) for l in range(8)]


def test_segments_reject_bad_input():
    with pytest.raises(S.SageError):
        S.sage_selftest_segments([3, 1], 2, BLOCK)
    with pytest.raises(S.SageError):
        S.sage_selftest_segments([0], 0, BLOCK)
    assert S.sage_selftest_segments([], 3, BLOCK) == [0, 0, 0]
