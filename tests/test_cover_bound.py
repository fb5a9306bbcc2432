"""Lower bound on the pair rows of the 256^3 workload's product-Gram.

A closed triplet (a <= b <= c) is the entry G[(x, y), z] for any of its three
pairs (a, b), (a, c), (b, c), so the rows of the product-Gram must cover
every triplet with at least one of its pairs.  The fused tail also keeps the
24 rows (b, b) for P and the p = 4 tile.  An exact set cover by integer
programming shows that 127 rows in all are needed for the 1522 closed
triplets of 24 linear bins at 256^3, i.e. four 32-row tiles: no cheaper
cover exists for the library's greedy one to miss.  The triplet list is the
stored oracle output for that workload.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_256_bubbles.fftref.npz")


def _pairs(t):
    a, b, c = t
    return ((a, b), (a, c), (b, c))


def test_minimum_cover_of_the_256cube_triplets_needs_four_tiles():
    optimize = pytest.importorskip("scipy.optimize")
    tri = np.sort(np.load(GOLDEN)["triplets"], axis=1)
    assert len(tri) == 1522
    nb = 24
    fixed = {(b, b) for b in range(nb)}
    open_t = [tuple(t) for t in tri if not any(p in fixed for p in _pairs(t))]
    cand = sorted({p for t in open_t for p in _pairs(t)})
    col = {p: i for i, p in enumerate(cand)}
    a = np.zeros((len(open_t), len(cand)))
    for r, t in enumerate(open_t):
        for p in _pairs(t):
            a[r, col[p]] = 1.0
    res = optimize.milp(c=np.ones(len(cand)), constraints=optimize.LinearConstraint(a, lb=1.0, ub=np.inf),
                        integrality=np.ones(len(cand)), bounds=optimize.Bounds(0, 1),
                        options={"time_limit": 120})
    assert res.status == 0                     # proven optimal
    rows = len(fixed) + int(round(res.fun))
    assert rows == 127
    assert (rows + 31) // 32 == 4
    # the chosen rows do cover every triplet
    chosen = fixed | {cand[i] for i in np.flatnonzero(res.x > 0.5)}
    assert all(any(p in chosen for p in _pairs(tuple(t))) for t in tri)
