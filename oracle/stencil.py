"""Oracle: the 7-point stencil function body (test infrastructure only).

The paper's scientific-computing functions (Table 1: lbm, mrif, tpacf from
Parboil) are not available.  The stand-in is a variable-coefficient Jacobi
relaxation whose coefficient grid is the read-only blob shared by
invocations (read-only sharing is not limited to DNN weights: Sharing-based
Memory Management, "Read-only Memory Sharing").  Readings fixed here:

* grid u[z][y][x], x fastest;
* boundary cells (any index 0 or n-1) keep their initial value;
* interior update, all cells from the previous sweep (Jacobi):
      u'_p = u_p + c_p * ((sum of the 6 face neighbours of p) / 6 - u_p);
* float64 evaluation; error metric max|u - u_ref| / max|u_ref|.

Pins (tests/test_oracle_stencil.py): c = 0 leaves the field unchanged; a
constant field stays constant; a linear field with c = 1 is a fixed point
(the 6-neighbour average of a linear function is its centre value); a scalar
loop agrees with the array form; the point evaluator agrees with the full
grid.
"""
from __future__ import annotations

import numpy as np


def jacobi7(u0, c, sweeps: int) -> np.ndarray:
    u = np.array(u0, dtype=np.float64, copy=True)
    c = np.asarray(c, dtype=np.float64)
    ci = c[1:-1, 1:-1, 1:-1]
    for _ in range(sweeps):
        nb = (u[:-2, 1:-1, 1:-1] + u[2:, 1:-1, 1:-1] + u[1:-1, :-2, 1:-1] +
              u[1:-1, 2:, 1:-1] + u[1:-1, 1:-1, :-2] + u[1:-1, 1:-1, 2:])
        centre = u[1:-1, 1:-1, 1:-1]
        new = centre + ci * (nb / 6.0 - centre)
        u = u.copy()
        u[1:-1, 1:-1, 1:-1] = new
    return u


def jacobi7_loops(u0, c, sweeps: int) -> np.ndarray:
    u = np.array(u0, dtype=np.float64, copy=True)
    nz, ny, nx = u.shape
    for _ in range(sweeps):
        v = u.copy()
        for z in range(1, nz - 1):
            for y in range(1, ny - 1):
                for x in range(1, nx - 1):
                    s = (u[z - 1, y, x] + u[z + 1, y, x] + u[z, y - 1, x] +
                         u[z, y + 1, x] + u[z, y, x - 1] + u[z, y, x + 1])
                    v[z, y, x] = u[z, y, x] + float(c[z, y, x]) * (s / 6.0 - u[z, y, x])
        u = v
    return u


def jacobi7_points(u0, c, sweeps: int, points) -> np.ndarray:
    """Values after ``sweeps`` at the given (z, y, x) points, each computed on
    the sub-grid of half-width ``sweeps`` around it (its whole dependency
    region); ``u0`` and ``c`` may be any array-likes indexable by slices."""
    shape = u0.shape
    out = []
    for p in points:
        lo = [max(0, q - sweeps) for q in p]
        hi = [min(n, q + sweeps + 1) for q, n in zip(p, shape)]
        sl = tuple(slice(a, b) for a, b in zip(lo, hi))
        sub_u = np.asarray(u0[sl], dtype=np.float64)
        sub_c = np.asarray(c[sl], dtype=np.float64).copy()
        # jacobi7 holds the sub-grid's outer layer fixed.  Where that layer is
        # the true boundary this is exact; elsewhere it is stale after the
        # first sweep, and after s sweeps the stale values have reached s
        # layers inwards, so p (``sweeps`` layers in) is still exact.
        r = jacobi7(sub_u, sub_c, sweeps)
        out.append(r[tuple(q - a for q, a in zip(p, lo))])
    return np.array(out, dtype=np.float64)


def normwise_error(u, u_ref) -> float:
    u = np.asarray(u, dtype=np.float64)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    denom = np.max(np.abs(u_ref))
    err = np.max(np.abs(u - u_ref))
    return float(err / denom) if denom > 0 else float(err)
