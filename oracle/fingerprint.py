"""Oracle: the FP64K-v1 block fingerprint (test infrastructure only).

The paper shares read-only data among invocations of the same function
(Sharing-based Memory Management, "Read-only Memory Sharing") but names no
content fingerprint.  This build shares at 64 KiB block granularity across
functions, so it needs one; FP64K-v1 is the reading this project fixes:

  for a block of L bytes (1 <= L <= 65536): zero-pad to 8*ceil(L/8) bytes,
  read little-endian 64-bit words w_j, split lo_j = w_j mod 2^32,
  hi_j = w_j >> 32, key the halves with a_j = (K0 + j*K1) mod 2^32 and
  c_j = (K2 + j*K3) mod 2^32, and form the NH-style sum (Black et al.,
  "UMAC: Fast and Secure Message Authentication", CRYPTO 1999)

      S = sum_j ((lo_j + a_j) mod 2^32) * ((hi_j + c_j) mod 2^32)   (mod 2^64)

  then fp = mix64(S xor (L * K4 mod 2^64)) with mix64 the splitmix64
  finaliser (Steele, Lea, Flood, "Fast Splittable Pseudorandom Number
  Generators", OOPSLA 2014).

K0..K3 are the low 32 bits of the first four splitmix64 outputs from state 0,
K4 the fifth output, each with its lowest bit set.  The sum is commutative
and associative mod 2^64, so any reduction tree gives the same bits.

Pins (tests/test_oracle_fingerprint.py): mix64 reproduces the published
splitmix64 sequence; closed forms on constructed blocks whose keyed halves
are forced to known values (S = 0, S = number of words, S = 6*words); two
implementations (Python integers, vectorised numpy) agree; length is mixed
in; single-bit flips change the value.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
BLOCK = 65536


def mix64(z: int) -> int:
    """splitmix64 output function (variant "Mix13" of Stafford's finalisers)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64(state: int, n: int) -> list:
    """First ``n`` outputs of splitmix64 started from ``state``."""
    out = []
    for _ in range(n):
        state = (state + GOLDEN_GAMMA) & M64
        out.append(mix64(state))
    return out


def keys() -> tuple:
    """(K0, K1, K2, K3, K4) as defined in the module header."""
    s = splitmix64(0, 5)
    return tuple((v & M32) | 1 for v in s[:4]) + ((s[4] | 1) & M64,)


K0, K1, K2, K3, K4 = keys()


def nh_sum_py(block: bytes) -> int:
    """The keyed sum S of a block, with Python integers (slow, plain)."""
    L = len(block)
    padded = bytes(block) + b"\0" * ((-L) % 8)
    s = 0
    for j in range(len(padded) // 8):
        w = int.from_bytes(padded[8 * j:8 * j + 8], "little")
        lo, hi = w & M32, w >> 32
        a = (K0 + j * K1) & M32
        c = (K2 + j * K3) & M32
        s += ((lo + a) & M32) * ((hi + c) & M32)
    return s & M64


def fp64k_py(block: bytes) -> int:
    """FP64K-v1 of one block (1..65536 bytes), Python integers."""
    L = len(block)
    if not 1 <= L <= BLOCK:
        raise ValueError("block length must be in 1..65536")
    return mix64(nh_sum_py(block) ^ ((L * K4) & M64))


# --------------------------------------------------------------- vectorised
_J = np.arange(BLOCK // 8, dtype=np.uint64)
_A = ((np.uint64(K0) + _J * np.uint64(K1)) & np.uint64(M32))
_C = ((np.uint64(K2) + _J * np.uint64(K3)) & np.uint64(M32))


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def fp64k_full_blocks(words: np.ndarray) -> np.ndarray:
    """FP64K-v1 of full 64 KiB blocks given as uint64 words [n, 8192]."""
    words = np.asarray(words, dtype=np.uint64)
    n, m = words.shape
    lo = words & np.uint64(M32)
    hi = words >> np.uint64(32)
    with np.errstate(over="ignore"):
        prod = ((lo + _A[:m]) & np.uint64(M32)) * ((hi + _C[:m]) & np.uint64(M32))
        s = prod.sum(axis=1, dtype=np.uint64)
        lk = np.uint64((m * 8 * K4) & M64)
        return _mix64_np(s ^ lk)


def fp64k_blob(blob, block: int = BLOCK, chunk_blocks: int = 512) -> np.ndarray:
    """Fingerprints of every block of a byte blob (last block may be short)."""
    buf = np.frombuffer(memoryview(np.ascontiguousarray(blob)).cast("B"), dtype=np.uint8)
    n = buf.size
    if block != BLOCK:
        return np.array([fp64k_py(buf[i:i + block].tobytes()) for i in range(0, n, block)],
                        dtype=np.uint64)
    nfull = n // BLOCK
    out = np.empty(nfull + (1 if n % BLOCK else 0), dtype=np.uint64)
    for s in range(0, nfull, chunk_blocks):
        e = min(nfull, s + chunk_blocks)
        w = buf[s * BLOCK:e * BLOCK].view(np.uint64).reshape(e - s, BLOCK // 8)
        out[s:e] = fp64k_full_blocks(w)
    if n % BLOCK:
        tail = buf[nfull * BLOCK:]
        L = tail.size
        padded = np.zeros(-(-L // 8) * 8, dtype=np.uint8)
        padded[:L] = tail
        w = padded.view(np.uint64)
        lo, hi = w & np.uint64(M32), w >> np.uint64(32)
        m = w.size
        with np.errstate(over="ignore"):
            s_ = (((lo + _A[:m]) & np.uint64(M32)) * ((hi + _C[:m]) & np.uint64(M32))).sum(dtype=np.uint64)
        out[-1] = mix64(int(s_) ^ ((L * K4) & M64))
    return out
