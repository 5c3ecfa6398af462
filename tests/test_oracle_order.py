"""Pins of the oracle's Gauss-Seidel sweep order on levels swept in block order.

The block colours are recomputed here with NumPy from their definition (the
two coordinate axes of largest extent, square cells of side slightly more
than the largest coupling distance along them, bricks of two cells side by
side shifted by one cell on odd rows with three brick colours, or single cells
with their parity pair where a brick would hold more than 256 rows), and the
property the block sweep relies on is checked directly on A_l: two coupled
rows lie in the same or in neighbouring cells, so coupled rows of equal block
colour share a block.
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


def bricks(cells):
    """Brick key and brick colour of every cell (x, y): brick bx = (x + y mod 2) div 2
    of row y, colour (bx - (y + 1) div 2 - y) mod 3."""
    x, y = cells[:, 0], cells[:, 1]
    bx = (x + (y & 1)) // 2
    return y * ((x.max() + 1) // 2 + 1) + bx, (bx - (y + 1) // 2 - y) % 3


def test_brick_colours_differ_between_touching_bricks():
    """Brute force over a 13 x 11 grid of cells: two cells that share a side or a
    corner lie in one brick or in bricks of different colours; every brick holds
    at most two cells, side by side, and touches exactly six others away from
    the grid's edge."""
    gx, gy = 13, 11
    cells = np.array([(x, y) for y in range(gy) for x in range(gx)], np.int64)
    key, col = bricks(cells)
    at = {(int(x), int(y)): t for t, (x, y) in enumerate(cells)}
    touch = {}
    for t, (x, y) in enumerate(cells):
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                u = at.get((int(x) + dx, int(y) + dy))
                if u is None or key[u] == key[t]:
                    continue
                assert col[u] != col[t]
                touch.setdefault(int(key[t]), set()).add(int(key[u]))
    for k in np.unique(key):
        mem = cells[key == k]
        assert len(mem) <= 2 and (len(mem) == 1 or (mem[1, 0] - mem[0, 0] == 1 and mem[1, 1] == mem[0, 1]))
        x0, y0 = mem[0]
        if 2 <= x0 <= gx - 4 and 1 <= y0 <= gy - 2:
            assert len(touch[int(k)]) == 6


def blocks(cells):
    """Block key and block colour of every cell: bricks when no brick holds more
    than 256 rows, else single cells coloured by their parity pair."""
    key, col = bricks(cells)
    if np.bincount(key).max() <= 256:
        return key, col
    x, y = cells[:, 0], cells[:, 1]
    return y * (x.max() + 1) + x, (x & 1) + 2 * (y & 1)


def cell_colouring_fits(lv, cells):
    """Whether every block has at most 512 rows and its couplings can be coloured
    by DSATUR with fewer than 64 colours."""
    key, _ = blocks(cells)
    rp, ci = lv["arp"], lv["acol"]
    for k in np.unique(key):
        rows = np.flatnonzero(key == k)
        if len(rows) > 512:
            return False
        loc = {int(r): t for t, r in enumerate(rows)}
        adj = [[loc[int(j)] for j in ci[rp[r]:rp[r + 1]] if j != r and int(j) in loc] for r in rows]
        crp = np.concatenate([[0], np.cumsum([len(a) for a in adj])]).astype(np.int32)
        ccl = np.array([v for a in adj for v in a], np.int32)
        if oracle.dsatur(crp, ccl)[1] < 0:
            return False
    return True


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
        cells, i, j = grid_cells(lv)
        if len(bc) == 0:
            # the level went back to the colour order: a cell is too large or needs 64 colours
            assert not cell_colouring_fits(lv, cells), (name, l)
            continue
        seen += 1
        key, col = blocks(cells)
        assert np.array_equal(bc, col)
        assert np.abs(cells[i] - cells[j]).max() <= 1
        same = bc[i] == bc[j]
        assert np.array_equal(key[i][same], key[j][same])
    assert seen >= 1 or name == "hubs"


def test_bricks_or_cells_on_the_torus():
    """1024 x 1024 torus, default options: level 1 has bricks of more than 256
    rows, so its blocks are single cells with the four parity colours; level 2's
    bricks all fit, so it takes bricks and three colours."""
    import synth
    h = oracle.Hierarchy.from_problem(synth.config_torus(1024, 1024))
    forms = []
    for l in (1, 2):
        lv = h.level(l)
        cells, i, j = grid_cells(lv)
        bkey, bcol = bricks(cells)
        x, y = cells[:, 0], cells[:, 1]
        if np.bincount(bkey).max() > 256:
            assert np.array_equal(lv["block_colors"], (x & 1) + 2 * (y & 1))
            forms.append("cells")
        else:
            assert np.array_equal(lv["block_colors"], bcol)
            forms.append("bricks")
        same = lv["block_colors"][i] == lv["block_colors"][j]
        key, _ = blocks(cells)
        assert np.array_equal(key[i][same], key[j][same])
    assert forms == ["cells", "bricks"]


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


def csr(m, edges):
    adj = [[] for _ in range(m)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    rp = np.zeros(m + 1, np.int32)
    rp[1:] = np.cumsum([len(x) for x in adj])
    col = np.array([v for x in adj for v in sorted(x)], np.int32)
    return rp, col


def test_dsatur_hand_worked_path():
    """Path 0-1-2-3: all saturations 0, vertices 1 and 2 have degree 2, the
    smaller number goes first (colour 0); then 2 (saturation 1, degree 2)
    takes colour 1; 0 and 3 have saturation 1 and degree 1: 0 goes first and
    takes colour 1, then 3 takes colour 0."""
    col, nc = oracle.dsatur(*csr(4, [(0, 1), (1, 2), (2, 3)]))
    assert nc == 2 and col.tolist() == [1, 0, 1, 0]


@pytest.mark.parametrize("graph,chi", [
    ("even_cycle", 2), ("odd_cycle", 3), ("complete6", 6), ("k34", 2), ("wheel6", 3), ("wheel5", 4),
    ("grid", 2), ("crown4", 2)])
def test_dsatur_exact_on_classic_graphs(graph, chi):
    """DSATUR is exact on bipartite graphs, cycles, wheels and complete graphs:
    it reaches the chromatic number, which is known for each."""
    if graph == "even_cycle":
        m, e = 10, [(i, (i + 1) % 10) for i in range(10)]
    elif graph == "odd_cycle":
        m, e = 9, [(i, (i + 1) % 9) for i in range(9)]
    elif graph == "complete6":
        m, e = 6, [(i, j) for i in range(6) for j in range(i + 1, 6)]
    elif graph == "k34":
        m, e = 7, [(i, j) for i in range(3) for j in range(3, 7)]
    elif graph.startswith("wheel"):
        k = int(graph[5:])
        m, e = k + 1, [(i, (i + 1) % k) for i in range(k)] + [(k, i) for i in range(k)]
    elif graph == "grid":
        m, e = 20, [(r * 5 + c, r * 5 + c + 1) for r in range(4) for c in range(4)] + \
            [(r * 5 + c, (r + 1) * 5 + c) for r in range(3) for c in range(5)]
    else:                                         # crown graph S_4^0: bipartite, greedy-hard
        m, e = 8, [(i, 4 + j) for i in range(4) for j in range(4) if i != j]
    rp, cl = csr(m, e)
    col, nc = oracle.dsatur(rp, cl)
    assert nc == chi
    for a, b in e:
        assert col[a] != col[b]


def test_dsatur_colour_limit():
    """A clique of 64 needs colour 63; one of 65 would need colour 64: refused."""
    rp, cl = csr(64, [(i, j) for i in range(64) for j in range(i + 1, 64)])
    assert oracle.dsatur(rp, cl)[1] == 64
    rp, cl = csr(65, [(i, j) for i in range(65) for j in range(i + 1, 65)])
    assert oracle.dsatur(rp, cl)[1] == -1


@pytest.mark.parametrize("name,minc,bmin", [("torus96", 200, 1000), ("pc20k", 500, 1000), ("ico5", 100, 500)])
def test_cell_colouring_of_block_levels(name, minc, bmin):
    """On every level swept in block order, the colours are a proper colouring
    of each brick's couplings, and every row of colour c has a neighbour in its
    brick of every colour below c (the property of any greedy colouring, which
    DSATUR is); rows of different bricks may share colours freely."""
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc, block_min_rows=bmin))
    seen = 0
    for l in range(1, h.num_levels - 1):
        lv = h.level(l)
        if len(lv["block_colors"]) == 0:
            continue
        seen += 1
        cells, _, _ = grid_cells(lv)
        key, _ = blocks(cells)
        col = lv["colors"]
        rp, ci = lv["arp"], lv["acol"]
        for i in range(lv["n"]):
            nb = [j for j in ci[rp[i]:rp[i + 1]] if j != i and key[j] == key[i]]
            ncols = {col[j] for j in nb}
            assert col[i] not in ncols
            assert set(range(col[i])) <= ncols
        assert h.sizes(l)["colors"] == col.max() + 1
    assert seen >= 1
