"""Seeded synthetic workloads for the function-setup path.

This module only draws inputs.  It is shared by the CPU oracle and by the GPU
path and therefore holds none of the method's arithmetic: no fingerprint, no
deduplication, no MLP or stencil maths.  Every array comes from numpy's PCG64
(`default_rng`) keyed by ``(seed, stream, ...)`` so that any piece can be
regenerated on its own.

The workloads stand in for the paper's benchmark functions (Table 1: DNN
inference with read-only weights, scientific kernels with a read-only
coefficient field) and for the production arrival trace (Evaluation,
"Implementation and Experimental Setup"); none of those are available, so
their shapes, sizes and sharing structure are reproduced with random data.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BLOCK = 65536  # bytes per read-only block

# stream ids: keep each workload's random numbers independent
_S_MLP_F32_W, _S_MLP_F32_X = 1, 2
_S_SHARED_IDX, _S_SHARED_CONTENT, _S_FN_CONTENT = 10, 11, 12
_S_BATCH_U, _S_BATCH_LOGN, _S_X_BF16 = 20, 21, 22
_S_STENCIL_C, _S_STENCIL_U = 30, 31
_S_SERVE = 40


def generator(seed: int, *stream: int) -> np.random.Generator:
    """PCG64 generator for ``(seed, *stream)`` (all non-negative ints)."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), *map(int, stream)]))


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 samples to bfloat16 (nearest, ties to even); returns the
    16-bit patterns.  Inputs are finite.  Used only to prepare BF16 inputs."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    bias = np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    return ((u + bias) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns to float32 (exact)."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------- MLP, FP32
@dataclass
class MlpF32Workload:
    """2-layer FP32 ReLU MLP, weights ``[layers][out][in]`` row-major."""
    weights: np.ndarray            # float32 [layers, width, width]
    inputs: list                   # float32 [batch, width] per invocation

    @property
    def width(self) -> int:
        return self.weights.shape[1]

    @property
    def layers(self) -> int:
        return self.weights.shape[0]


def mlp_f32_workload(width: int = 2048, layers: int = 2, batch: int = 8,
                     invocations: int = 16, seed: int = 0) -> MlpF32Workload:
    g = generator(seed, _S_MLP_F32_W)
    w = g.standard_normal((layers, width, width), dtype=np.float32)
    w *= np.float32(1.0 / np.sqrt(width))
    xs = [generator(seed, _S_MLP_F32_X, i).standard_normal((batch, width), dtype=np.float32)
          for i in range(invocations)]
    return MlpF32Workload(weights=w, inputs=xs)


# ---------------------------------------------------------------- MLP, BF16
@dataclass
class SharedMlpFunctions:
    """``n_fns`` BF16 MLPs whose weight blobs hold the same content at a
    common set of 64 KiB block indices (``shared_idx``) and independent
    content everywhere else."""
    width: int
    layers: int
    blobs: list                    # uint16 [layers*width*width] per function
    shared_idx: np.ndarray         # sorted block indices identical across fns

    @property
    def blob_bytes(self) -> int:
        return self.layers * self.width * self.width * 2

    @property
    def n_blocks(self) -> int:
        return -(-self.blob_bytes // BLOCK)


def shared_mlp_bf16_functions(n_fns: int = 4, layers: int = 8, width: int = 4096,
                              share_frac: float = 0.3, seed: int = 0) -> SharedMlpFunctions:
    """Weights ~ N(0, 1/width) rounded to BF16.  floor(share_frac * n_blocks)
    block indices, drawn without replacement, carry one common content stream
    in every function; the other blocks are drawn per function."""
    nbytes = layers * width * width * 2
    if nbytes % BLOCK:
        raise ValueError("blob must be a whole number of 64 KiB blocks")
    n_blocks = nbytes // BLOCK
    per_block = BLOCK // 2
    n_shared = int(np.floor(share_frac * n_blocks))
    shared_idx = np.sort(generator(seed, _S_SHARED_IDX).choice(n_blocks, size=n_shared, replace=False))
    mask = np.zeros(n_blocks, dtype=bool)
    mask[shared_idx] = True
    own_idx = np.nonzero(~mask)[0]
    std = np.float32(1.0 / np.sqrt(width))
    shared = f32_to_bf16_bits(
        generator(seed, _S_SHARED_CONTENT).standard_normal((n_shared, per_block), dtype=np.float32) * std)
    blobs = []
    for f in range(n_fns):
        blob = np.empty((n_blocks, per_block), dtype=np.uint16)
        blob[shared_idx] = shared
        own = generator(seed, _S_FN_CONTENT, f).standard_normal((own_idx.size, per_block), dtype=np.float32)
        own *= std
        blob[own_idx] = f32_to_bf16_bits(own)
        blobs.append(blob.reshape(-1))
    return SharedMlpFunctions(width=width, layers=layers, blobs=blobs, shared_idx=shared_idx)


def uniform_batches(n: int, lo: int = 1, hi: int = 32, seed: int = 0, stream: int = 0) -> np.ndarray:
    """Batch sizes uniform on the integers lo..hi."""
    return generator(seed, _S_BATCH_U, stream).integers(lo, hi + 1, size=n).astype(np.int64)


def lognormal_batches(n: int, median: float = 8.0, sigma: float = 1.0, lo: int = 1,
                      hi: int = 128, seed: int = 0) -> np.ndarray:
    """Batch sizes clip(round(lognormal(ln median, sigma)), lo, hi)."""
    b = generator(seed, _S_BATCH_LOGN).lognormal(np.log(median), sigma, size=n)
    return np.clip(np.rint(b), lo, hi).astype(np.int64)


def bf16_inputs(batch: int, width: int, seed: int = 0, *key: int) -> np.ndarray:
    """One invocation's input rows, N(0,1) rounded to BF16 (uint16 bits)."""
    x = generator(seed, _S_X_BF16, *key).standard_normal((batch, width), dtype=np.float32)
    return f32_to_bf16_bits(x)


# ---------------------------------------------------------------- stencil
def stencil_coefficients(n: int, seed: int = 0, lo: float = 0.1, hi: float = 1.0,
                         shape=None) -> np.ndarray:
    """Read-only coefficient grid c[z][y][x] ~ U[lo, hi) as float32."""
    shape = (n, n, n) if shape is None else shape
    c = generator(seed, _S_STENCIL_C).random(shape, dtype=np.float32)
    return (c * np.float32(hi - lo) + np.float32(lo)).astype(np.float32)


def stencil_field(n: int, inv: int, seed: int = 0, shape=None) -> np.ndarray:
    """Initial field u0[z][y][x] ~ N(0, 1) as float32 for invocation ``inv``."""
    shape = (n, n, n) if shape is None else shape
    return generator(seed, _S_STENCIL_U, inv).standard_normal(shape, dtype=np.float32)


# ---------------------------------------------------------------- small blobs
def blob_with_duplicates(n_blocks: int, block: int, dup_pairs, seed: int = 0,
                         tail: int = 0, zero_blocks=()) -> np.ndarray:
    """Random bytes arranged as ``n_blocks`` blocks of ``block`` bytes plus an
    optional partial tail; ``dup_pairs`` lists (dst, src) block indices whose
    contents are made equal, ``zero_blocks`` are cleared."""
    g = generator(seed, 50, n_blocks, block, tail)
    buf = g.integers(0, 256, size=n_blocks * block + tail, dtype=np.uint8)
    for z in zero_blocks:
        buf[z * block:(z + 1) * block] = 0
    for dst, src in dup_pairs:
        buf[dst * block:(dst + 1) * block] = buf[src * block:(src + 1) * block]
    return buf


# ---------------------------------------------------------------- serving
@dataclass
class ServingWorkload:
    """Open-loop Poisson arrivals over a set of BF16 MLP functions."""
    width: int
    layers: list                   # layers per function
    arrivals: np.ndarray           # float64 seconds, sorted
    fn: np.ndarray                 # int64 function id per request
    batch: np.ndarray              # int64 rows per request
    overlap_frac: float
    extra: dict = field(default_factory=dict)


def serving_workload(rate: float, duration: float, n_fns: int = 16, width: int = 4096,
                     median_bytes: float = 512 * 2**20, sigma: float = 1.0,
                     min_bytes: float = 64 * 2**20, max_bytes: float = 4 * 2**30,
                     max_batch: int = 64, overlap_frac: float = 0.2, seed: int = 0) -> ServingWorkload:
    """Function sizes lognormal(ln median, sigma) clipped to [min, max] and
    rounded to whole layers (width*width BF16 each); popularity Zipf(1) over
    the functions; batch uniform on 1..max_batch; exponential inter-arrival
    times with the given rate."""
    g = generator(seed, _S_SERVE)
    layer_bytes = width * width * 2
    sizes = np.clip(g.lognormal(np.log(median_bytes), sigma, size=n_fns), min_bytes, max_bytes)
    layers = [max(1, int(round(s / layer_bytes))) for s in sizes]
    n_req = max(1, int(rate * duration * 1.5) + 16)
    gaps = g.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps)
    t = t[t < duration]
    w = 1.0 / np.arange(1, n_fns + 1)
    fn = g.choice(n_fns, size=t.size, p=w / w.sum()).astype(np.int64)
    batch = g.integers(1, max_batch + 1, size=t.size).astype(np.int64)
    return ServingWorkload(width=width, layers=layers, arrivals=t, fn=fn, batch=batch,
                           overlap_frac=overlap_frac)


def serving_blobs(layers_per_fn, width: int, overlap_frac: float, seed: int = 0):
    """Weight blobs for the serving functions: a fraction ``overlap_frac`` of
    each function's 64 KiB blocks is copied from one common content pool
    (same pool block at the same block index), the rest is drawn per
    function."""
    per_block = BLOCK // 2
    std = np.float32(1.0 / np.sqrt(width))
    max_blocks = max(layers_per_fn) * width * width * 2 // BLOCK
    g = generator(seed, _S_SERVE, 1)
    pool = f32_to_bf16_bits(g.standard_normal((max_blocks, per_block), dtype=np.float32) * std)
    blobs = []
    for f, nl in enumerate(layers_per_fn):
        nb = nl * width * width * 2 // BLOCK
        gf = generator(seed, _S_SERVE, 2, f)
        share = gf.random(nb) < overlap_frac
        blob = f32_to_bf16_bits(gf.standard_normal((nb, per_block), dtype=np.float32) * std)
        blob[share] = pool[:nb][share]
        blobs.append(blob.reshape(-1))
    return blobs
