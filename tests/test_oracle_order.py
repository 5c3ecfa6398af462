"""Pins of the oracle's Gauss-Seidel sweep order on levels swept in block order.

The block colours are recomputed here with NumPy from their definition (the
two coordinate axes of largest extent, square cells of side slightly more
than the largest coupling distance along them, the parity pair of the cell),
and the property the block sweep relies on is checked directly on A_l: two
coupled rows lie in the same or in neighbouring cells, so coupled rows of
equal block colour share a cell.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import problem

MARGIN = 1.0 + 2.0 ** -20


def grid_cells(lv):
    X = lv["X"]
    ext = X.max(0) - X.min(0)
    drop = int(np.argmin(ext))                   # first minimum
    keep = [a for a in range(3) if a != drop]
    rows = np.repeat(np.arange(lv["n"]), np.diff(lv["arp"]))
    off = rows != lv["acol"]
    d = np.abs(X[lv["acol"][off]][:, keep] - X[rows[off]][:, keep])
    side = d.max() * MARGIN
    cells = np.floor((X[:, keep] - X[:, keep].min(0)) / side).astype(np.int64)
    return cells, rows[off], lv["acol"][off]


@pytest.mark.parametrize("name,minc,bmin", [("torus96", 200, 1000), ("pc20k", 500, 1000), ("ico5", 100, 500),
                                            ("hubs", 100, 500)])
def test_block_colours_from_the_grid(name, minc, bmin):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc, block_min_rows=bmin))
    seen = 0
    for l in range(h.num_levels):
        lv = h.level(l)
        bc = lv["block_colors"]
        if l == 0 or l == h.num_levels - 1 or lv["n"] <= bmin:
            assert len(bc) == 0, (l, lv["n"])
            continue
        seen += 1
        cells, i, j = grid_cells(lv)
        assert np.array_equal(bc, (cells[:, 0] & 1) + 2 * (cells[:, 1] & 1))
        assert np.abs(cells[i] - cells[j]).max() <= 1
        same = bc[i] == bc[j]
        assert np.array_equal(cells[i][same], cells[j][same])
    assert seen >= 1


def test_block_order_on_the_default_levels():
    """Default threshold: the first Galerkin level of a 256 x 256 torus (more than
    4096 points) sweeps in block order; level 0 and the small levels do not."""
    import synth
    p = synth.config_torus(256, 256)
    h = oracle.Hierarchy.from_problem(p)
    flags = [h.sizes(l)["blocks"] for l in range(h.num_levels)]
    sizes = [h.sizes(l)["n"] for l in range(h.num_levels)]
    assert flags[0] == 0 and flags[-1] == 0
    for l in range(1, h.num_levels - 1):
        assert flags[l] == (1 if sizes[l] > 4096 else 0), (sizes, flags)
    assert flags[1] == 1
