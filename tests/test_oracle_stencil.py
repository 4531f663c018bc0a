"""Pins for the stencil oracle: exact special cases, loops vs arrays, and the
point evaluator vs the full grid."""
import numpy as np
import pytest

from oracle import stencil as S


def test_zero_coefficient_is_identity():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((7, 6, 9))
    assert np.array_equal(S.jacobi7(u, np.zeros_like(u), 5), u)


def test_constant_field_stays_constant():
    u = np.full((6, 6, 6), 2.5)
    c = np.random.default_rng(1).uniform(0.1, 1.0, u.shape)
    assert np.array_equal(S.jacobi7(u, c, 4), u)


def test_linear_field_is_fixed_point_with_unit_coefficient():
    z, y, x = np.meshgrid(np.arange(8), np.arange(9), np.arange(10), indexing="ij")
    u = 3.0 * x - 2.0 * y + 5.0 * z + 1.0        # integers: every sum exact
    assert np.array_equal(S.jacobi7(u, np.ones_like(u), 6), u)


def test_single_interior_cell_by_hand():
    u = np.zeros((3, 3, 3))
    u[0, 1, 1] = 6.0                              # one neighbour of the centre
    c = np.full(u.shape, 0.5)
    out = S.jacobi7(u, c, 1)
    assert out[1, 1, 1] == 0.0 + 0.5 * (6.0 / 6.0 - 0.0)
    assert out[0, 1, 1] == 6.0                    # boundary unchanged


@pytest.mark.parametrize("shape,sweeps", [((6, 6, 6), 2), ((5, 7, 8), 3), ((8, 8, 8), 1)])
def test_loops_equal_arrays(shape, sweeps):
    rng = np.random.default_rng(sum(shape))
    u = rng.standard_normal(shape)
    c = rng.uniform(0.1, 1.0, shape)
    np.testing.assert_allclose(S.jacobi7_loops(u, c, sweeps), S.jacobi7(u, c, sweeps), rtol=0, atol=1e-14)


def test_points_equal_full_grid():
    rng = np.random.default_rng(5)
    shape = (24, 20, 22)
    u = rng.standard_normal(shape)
    c = rng.uniform(0.1, 1.0, shape)
    sweeps = 6
    full = S.jacobi7(u, c, sweeps)
    pts = [(0, 0, 0), (12, 10, 11), (1, 19, 5), (23, 3, 21), (7, 7, 7), (6, 14, 16)]
    got = S.jacobi7_points(u, c, sweeps, pts)
    want = np.array([full[p] for p in pts])
    assert np.array_equal(got, want)
