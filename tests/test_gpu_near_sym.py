"""Symmetric near field of the log-kernel leaf pass against the dense oracle.

The leaf pass takes each pair of neighbouring leaves once (a leaf with its E
neighbour and the three leaves of the row above) and hands the source sums to
the other leaf through per-node partial-sum slots.  This point set fixes the
leaf occupancies on an 8 x 8 grid so that every branch of that scheme runs:
empty leaves next to occupied ones and on every border (slots cleared by their
receiver), single points, lane-group passes of 8/16/32 lanes, leaves of exactly
64 and 65 nodes, and leaves of several passes (source sums added across
passes).  Matvec parity with the dense sum (eq. phs_interp's kernel block) at
the FP64 tolerance.
"""
import numpy as np
import pytest

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

G = 8
# occupancy of cell (row, col) = _COUNTS[(row * G + col) % len], a pattern
# whose rows shift against each other so that every count meets empty and
# full neighbours in all directions
_COUNTS = [0, 1, 65, 7, 0, 0, 64, 9, 33, 129, 0, 16, 17, 200, 31, 32, 8, 63, 0, 96, 2, 128,
           15, 0, 40, 3]


def _points(seed: int):
    rng = W.rng_for(seed)
    pts = []
    counts = np.zeros((G, G), dtype=np.int64)
    for r in range(G):
        for c in range(G):
            m = _COUNTS[(r * G + c) % len(_COUNTS)]
            counts[r, c] = m
            if m:
                u = rng.uniform(0.1, 0.9, size=(m, 2))
                pts.append(np.stack([(c + u[:, 0]) / G, (r + u[:, 1]) / G], axis=1))
    # the bounding box is exactly the unit square, so the cells are the
    # leaves of a depth-3 tree (the two corner nodes fall in cells (0, 0) and
    # (7, 7), clamped)
    pts.append(np.array([[0.0, 0.0], [1.0, 1.0]]))
    xy = np.concatenate(pts)
    return xy, counts


@pytest.mark.parametrize("k", [2, 4])
def test_symmetric_near_field_occupancies(k):
    xy, _ = _points(700 + k)
    n = len(xy)
    print(f"[case] symmetric near field k={k} n={n}", flush=True)
    # leaf size n/64: depth 3, the cells above
    pl = N.Plan(dev(xy), k, -1, leaf_size=max(1, n // 64))
    assert pl.leaf_level == 3
    c, rho, xi = D.normalize(xy, k)
    _, keys = D.leaf_order(xi, pl.tree_half_width, 3)
    occ = np.bincount(keys, minlength=G * G).reshape(G, G)
    # the scheme's cases are present
    assert (occ == 0).any() and (occ == 1).any()
    assert ((occ > 1) & (occ <= 8)).any() and ((occ > 8) & (occ <= 16)).any()
    assert ((occ > 16) & (occ <= 32)).any() and ((occ > 32) & (occ < 64)).any()
    assert (occ == 64).any() and (occ == 65).any() and (occ > 128).any()
    for edge in (occ[0], occ[-1], occ[:, 0], occ[:, -1]):
        assert (edge == 0).any() and (edge > 0).any()
    rng = W.rng_for(710 + k)
    for trial in range(2):
        v = rng.standard_normal(n)
        if trial == 1:  # a projected vector, as PCG applies the matvec
            B = D.poly_block(xi, D.d_min(k))
            Q, _ = np.linalg.qr(B)
            v = v - Q @ (Q.T @ v)
        y_ref = D.matvec_dense(k, xi, v)
        y = host(pl.matvec(dev(v)))
        e = rel(y, y_ref)
        print(f"k={k} trial={trial} fp64 matvec rel err {e:.3e}")
        assert e <= 1e-10
        # again: the partial-sum slots are rewritten, not accumulated, per matvec
        y2 = host(pl.matvec(dev(v)))
        np.testing.assert_array_equal(y2, y)
    pl.close()
