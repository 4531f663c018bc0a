"""Pins for the MLP oracle: exact special cases and a scalar triple loop."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2404_14691_amd import synth


def test_permutation_weights_exact():
    rng = np.random.default_rng(0)
    K = 16
    x = rng.standard_normal((5, K))
    perms = [rng.permutation(K) for _ in range(3)]
    w = np.zeros((3, K, K))
    for l, p in enumerate(perms):
        w[l, np.arange(K), p] = 1.0          # row n picks input p[n]
    y = M.mlp_forward(x, w)
    # layer 0: h[:, n] = x[:, p0[n]] then relu; layer 1: relu again; layer 2 no relu
    h = np.maximum(x[:, perms[0]], 0)
    h = np.maximum(h[:, perms[1]], 0)
    want = h[:, perms[2]]
    assert np.array_equal(y, want)


def test_identity_nonnegative_returns_input():
    rng = np.random.default_rng(1)
    x = np.abs(rng.standard_normal((4, 8)))
    w = np.stack([np.eye(8)] * 4)
    assert np.array_equal(M.mlp_forward(x, w), x)


def test_last_layer_has_no_relu():
    x = np.array([[1.0, -2.0]])
    w = np.stack([np.eye(2), -np.eye(2)])
    # layer0 relu -> [1, 0]; layer1 = -h -> [-1, 0] (negative kept)
    assert np.array_equal(M.mlp_forward(x, w), np.array([[-1.0, 0.0]]))


@pytest.mark.parametrize("shape", [(4, 8, 2), (3, 5, 3), (1, 7, 1)])
def test_loops_equal_matrix_form(shape):
    b, K, L = shape
    rng = np.random.default_rng(b * 100 + K)
    x = rng.standard_normal((b, K))
    w = rng.standard_normal((L, K, K)) / np.sqrt(K)
    np.testing.assert_allclose(M.mlp_forward_loops(x, w), M.mlp_forward(x, w), rtol=1e-13, atol=1e-13)


def test_bf16_widening_exact():
    x = np.array([1.0, -2.5, 3.140625, 1e-3, 65504.0], dtype=np.float32)
    bits = synth.f32_to_bf16_bits(x)
    assert M.bf16_to_f64(bits)[0] == 1.0
    assert M.bf16_to_f64(bits)[1] == -2.5
    assert M.bf16_to_f64(bits)[2] == 3.140625


@pytest.mark.parametrize("v,want", [
    (1.0 + 2.0**-8, 1.0),                 # tie, even neighbour below
    (1.0 + 3 * 2.0**-8, 1.0 + 2.0**-6),   # tie, even neighbour above
    (1.0 + 2.0**-8 + 2.0**-20, 1.0 + 2.0**-7),
    (-3.0, -3.0),
    (0.0, 0.0),
])
def test_round_to_bf16_known_values(v, want):
    assert M.round_to_bf16(np.array([v]))[0] == want


def test_round_to_bf16_matches_input_generator():
    # the generator's float32 -> bf16 rounding and the oracle's float64 rounding
    # agree on float32 inputs (independent implementations)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(10000).astype(np.float32)
    a = M.bf16_to_f64(synth.f32_to_bf16_bits(x))
    b = M.round_to_bf16(x.astype(np.float64))
    assert np.array_equal(a, b)


def test_normwise_error():
    assert M.normwise_error([1.0, 2.0], [1.0, 4.0]) == 0.5
