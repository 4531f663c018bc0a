"""Oracle: block deduplication partition and byte accounting (test
infrastructure only).

The paper loads a function's read-only data once and lets every invocation
of that function use the same copy (Design Overview, "SAGE Architecture";
Sharing-based Memory Management, "Read-only Memory Sharing").  This build
generalises sharing to identical 64 KiB blocks across functions.  Readings
fixed here, where the paper is silent:

* Blocks: a blob of n bytes has ceil(n / B) blocks; the last one is short
  when B does not divide n; n = 0 gives no blocks.
* Logical blocks are ordered by registration order of functions, then block
  index.  Every block belongs to the class of the earliest logical block with
  the same length and the same bytes; that earliest block is the class's
  canonical representative.
* A fingerprint is only an index: blocks with equal fingerprints but
  different bytes are different classes.
* Accounting: logical = sum of blob sizes; unique = sum of class lengths;
  shared = bytes of blocks in classes of two or more members; private =
  bytes of blocks in singleton classes.  shared + private = logical.

Pins (tests/test_oracle_dedup.py): ``partition_bruteforce`` compares every
pair of blocks byte by byte and uses no fingerprint; ``partition_indexed``
(fingerprint map plus byte verification, the GPU path's method) must give the
same partition, also under a fingerprint that collides on purpose; planted
duplicates give closed-form counts.
"""
from __future__ import annotations

import numpy as np


def as_bytes(blob) -> np.ndarray:
    return np.frombuffer(memoryview(np.ascontiguousarray(blob)).cast("B"), dtype=np.uint8)


def block_spans(nbytes: int, block: int):
    """(offset, length) of every block of an ``nbytes`` blob."""
    return [(o, min(block, nbytes - o)) for o in range(0, nbytes, block)]


def logical_blocks(blobs, block: int):
    """List of (fn, blk, bytes) in canonical order."""
    out = []
    for f, blob in enumerate(blobs):
        b = as_bytes(blob)
        for k, (o, L) in enumerate(block_spans(b.size, block)):
            out.append((f, k, b[o:o + L].tobytes()))
    return out


def partition_bruteforce(blobs, block: int):
    """canon[f][k] = (f0, k0), the earliest logical block with equal bytes.
    O(n^2) byte comparisons, no hashing."""
    blocks = logical_blocks(blobs, block)
    reps = []                      # canonical (f, k, bytes)
    canon = [[None] * len(block_spans(as_bytes(b).size, block)) for b in blobs]
    for f, k, data in blocks:
        for rf, rk, rdata in reps:
            if len(rdata) == len(data) and rdata == data:
                canon[f][k] = (rf, rk)
                break
        else:
            reps.append((f, k, data))
            canon[f][k] = (f, k)
    return canon


def partition_dict(blobs, block: int):
    """Same partition via a dictionary keyed by the block's bytes (exact, no
    fingerprint); linear time, used at full workload sizes."""
    first = {}
    canon = [[None] * len(block_spans(as_bytes(b).size, block)) for b in blobs]
    for f, blob in enumerate(blobs):
        b = as_bytes(blob)
        for k, (o, L) in enumerate(block_spans(b.size, block)):
            canon[f][k] = first.setdefault(b[o:o + L].tobytes(), (f, k))
    return canon


def partition_indexed(blobs, block: int, fp):
    """Same partition, computed the way the GPU path does it: look the block's
    fingerprint up in a map of fingerprint -> candidate classes (in creation
    order), verify bytes, and start a new class when no candidate matches."""
    by_fp = {}
    canon = [[None] * len(block_spans(as_bytes(b).size, block)) for b in blobs]
    for f, k, data in logical_blocks(blobs, block):
        h = fp(data)
        for rf, rk, rdata in by_fp.get(h, []):
            if rdata == data:
                canon[f][k] = (rf, rk)
                break
        else:
            by_fp.setdefault(h, []).append((f, k, data))
            canon[f][k] = (f, k)
    return canon


def classes(canon):
    """Map canonical representative -> list of member (f, k), canonical order."""
    out = {}
    for f, row in enumerate(canon):
        for k, rep in enumerate(row):
            out.setdefault(rep, []).append((f, k))
    return out


def accounting(blobs, block: int, canon) -> dict:
    sizes = [as_bytes(b).size for b in blobs]
    lens = [[L for _, L in block_spans(n, block)] for n in sizes]
    cls = classes(canon)
    logical = sum(sizes)
    unique = sum(lens[f][k] for (f, k) in cls)
    shared = sum(lens[f][k] for members in cls.values() if len(members) >= 2 for (f, k) in members)
    private = sum(lens[f][k] for members in cls.values() if len(members) == 1 for (f, k) in members)
    return {"logical": logical, "unique": unique, "shared": shared, "private": private,
            "n_blocks": sum(len(x) for x in lens), "n_classes": len(cls)}


def same_partition(a, b) -> bool:
    """True when two block->representative maps induce the same partition."""
    if [len(r) for r in a] != [len(r) for r in b]:
        return False
    fwd, bwd = {}, {}
    for ra, rb in zip(a, b):
        for x, y in zip(ra, rb):
            if fwd.setdefault(x, y) != y or bwd.setdefault(y, x) != x:
                return False
    return True
