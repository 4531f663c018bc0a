"""Oracle: the MLP function body (test infrastructure only).

The paper's DNN-inference functions keep their weights as read-only data
shared by invocations (Table 1 benchmarks; Table 2 read-only column).  The
trained models are not available, so the body here is a plain ReLU MLP whose
weights are the read-only blob.  Readings fixed where the paper is silent:

* weights W_l stored [out][in] row-major, layers concatenated, no bias;
* H_0 = X, H_l = relu(H_{l-1} W_l^T) for l < L, Y = H_{L-1} W_L^T (no ReLU
  after the last layer);
* the oracle evaluates in float64 on the exact input values (BF16 or FP32);
* error metric per invocation: max|Y - Y_ref| / max|Y_ref| (normwise), since
  elementwise relative error is ill-posed at ReLU zeros.

``mlp_forward_mirror`` additionally rounds every hidden layer to BF16
(nearest, ties to even) as the GPU does between layers; it is a diagnostic,
not the parity reference.

Pins (tests/test_oracle_mlp.py): permutation-matrix weights give an exact
row permutation of the ReLU'd input; identity weights with non-negative
input return the input; a scalar triple loop agrees with the matrix form on
small shapes.
"""
from __future__ import annotations

import numpy as np


def bf16_to_f64(bits) -> np.ndarray:
    """Exact value of BF16 bit patterns."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def mlp_forward(x, weights) -> np.ndarray:
    """x: [b, K] values, weights: [L, N, K] values (any float dtype)."""
    h = np.asarray(x, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    L = w.shape[0]
    for l in range(L):
        h = h @ w[l].T
        if l < L - 1:
            h = np.maximum(h, 0.0)
    return h


def mlp_forward_loops(x, weights) -> np.ndarray:
    """Scalar triple loop, for small shapes."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    L, N, K = w.shape
    h = [list(r) for r in x]
    for l in range(L):
        out = []
        for row in h:
            o = []
            for n in range(N):
                s = 0.0
                for k in range(K):
                    s += row[k] * w[l, n, k]
                o.append(max(s, 0.0) if l < L - 1 else s)
            out.append(o)
        h = out
    return np.array(h, dtype=np.float64)


def round_to_bf16(v) -> np.ndarray:
    """Round float64 values to the nearest BF16 value, ties to even (finite,
    normal-range inputs)."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)                 # v = m * 2^e, 0.5 <= |m| < 1
    scaled = np.ldexp(m, 8)            # 8 significant bits for BF16
    r = np.round(scaled)               # numpy rounds half to even
    return np.ldexp(r, e - 8)


def mlp_forward_mirror(x, weights) -> np.ndarray:
    h = np.asarray(x, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    L = w.shape[0]
    for l in range(L):
        h = h @ w[l].T
        if l < L - 1:
            h = round_to_bf16(np.maximum(h, 0.0))
    return h


def normwise_error(y, y_ref) -> float:
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    denom = np.max(np.abs(y_ref))
    err = np.max(np.abs(y - y_ref))
    return float(err / denom) if denom > 0 else float(err)
