"""Pins of the ordering oracle (oracle/orderings.py) against closed forms and the defining
properties of each ordering (Section 5), independent of the oracle's own code."""
import numpy as np
import pytest

from oracle import orderings as O
from paper_1912_00539_amd import workloads as W


def pattern(mesh):
    c = W.assemble(mesh, W.natural_order(mesh), 0, "const", s=1.0)
    return c


def grid(nx, ny):
    return pattern(W.quad_mesh(nx, ny))


def block_1norm(vals):
    return np.abs(vals).sum(axis=1).max(axis=1)


def bfs_levels(adj, root):
    lev = {root: 0}
    q = [root]
    for v in q:
        for u in adj[v]:
            if u not in lev:
                lev[u] = lev[v] + 1
                q.append(u)
    return lev


# ------------------------------------------------------------------ pseudo-peripheral node, RCM
def test_pseudo_peripheral_path_and_grid():
    c = pattern(W.chain_mesh(9))
    adj = O.adjacency(c.n, c.rowptr, c.colidx)
    for start in (0, 4, 8):
        assert O.pseudo_peripheral(adj, start, [True] * c.n) in (0, 8)
    g = grid(7, 4)
    adj = O.adjacency(g.n, g.rowptr, g.colidx)
    corners = {0, 6, 21, 27}
    for start in (0, 9, 17, 13):
        assert O.pseudo_peripheral(adj, start, [True] * g.n) in corners


def test_rcm_path_is_the_reversed_path():
    c = pattern(W.chain_mesh(11))
    new = O.rcm(c.n, c.rowptr, c.colidx)
    np.testing.assert_array_equal(new, np.arange(c.n)[::-1])
    assert O.bandwidth(c.n, c.rowptr, c.colidx, new) == 1


@pytest.mark.parametrize("nx,ny", [(7, 4), (12, 12), (30, 5)])
def test_rcm_grid_bandwidth(nx, ny):
    """From a corner the level sets of an nx x ny grid are anti-diagonals of at most min(nx, ny)
    cells, so Cuthill-McKee's bandwidth is at most 2 min(nx, ny) - 1, against nx for the natural
    row-by-row order when ny > nx."""
    g = grid(nx, ny)
    new = O.rcm(g.n, g.rowptr, g.colidx)
    assert O.bandwidth(g.n, g.rowptr, g.colidx, new) <= 2 * min(nx, ny) - 1


@pytest.mark.parametrize("mesh", ["tri", "random", "nine"])
def test_cuthill_mckee_is_a_degree_sorted_breadth_first_order(mesh):
    """Definition: reversed, the order is breadth first from its first vertex (levels never
    decrease), every vertex after the first is appended by its earliest-placed neighbour, and the
    vertices one vertex appends come in increasing (degree, index)."""
    m = {"tri": W.split_tri_mesh(9, 7, 2), "random": W.random_graph_mesh(60, 3.0, 5),
         "nine": W.nine_point_mesh(8, 6)}[mesh]
    c = pattern(m)
    adj = O.adjacency(c.n, c.rowptr, c.colidx)
    comps = O._components(adj, list(range(c.n)), [True] * c.n)
    new = O.rcm(c.n, c.rowptr, c.colidx)
    order = np.argsort(new)
    pos = 0
    for comp in comps:
        cm = list(order[pos:pos + len(comp)][::-1])
        pos += len(comp)
        assert sorted(cm) == comp
        lev = bfs_levels(adj, cm[0])
        assert all(lev[cm[k]] <= lev[cm[k + 1]] for k in range(len(cm) - 1))
        place = {v: k for k, v in enumerate(cm)}
        parent = {v: min((u for u in adj[v]), key=lambda u: place[u]) for v in cm[1:]}
        for p in cm:
            kids = [v for v in cm[1:] if parent[v] == p]
            assert kids == sorted(kids, key=lambda v: (len(adj[v]), v))
            assert all(place[a] < place[b] for a, b in zip(kids, kids[1:]))


# ------------------------------------------------------------------ one-way dissection
def test_one_way_dissection_grid_closed_form():
    """10 x 100 grid: the root is a corner, L = 109 levels (anti-diagonals), w = 1000/109,
    delta = sqrt((3w + 13)/2) = 4.50..., separator levels floor(k delta + 1/2) <= 107: 24 of
    them (5, 9, 14, ..., 104, 108 is excluded). Separators come last; removing them leaves pieces
    that no edge joins; each piece is numbered contiguously."""
    g = grid(10, 100)
    adj = O.adjacency(g.n, g.rowptr, g.colidx)
    new = O.one_way_dissection(g.n, g.rowptr, g.colidx)
    order = np.argsort(new)
    w = 1000 / 109
    delta = ((3 * w + 13) / 2) ** 0.5
    seps = sorted({int(np.floor(k * delta + 0.5)) for k in range(1, 200) if np.floor(k * delta + 0.5) <= 107})
    r = O.pseudo_peripheral(adj, 0, [True] * g.n)
    assert r in (0, 9, 990, 999)
    lev = bfs_levels(adj, r)
    sep = {v for v in range(g.n) if lev[v] in seps and any(lev[u] == lev[v] + 1 for u in adj[v])}
    nsep = len(sep)
    assert set(order[g.n - nsep:]) == sep
    # pieces: components of the rest; contiguous and not adjacent to each other
    rest = [v for v in range(g.n) if v not in sep]
    inside = [False] * g.n
    for v in rest:
        inside[v] = True
    pieces = O._components(adj, rest, inside)
    assert len(pieces) == len(seps) + 1
    piece_of = {v: k for k, p in enumerate(pieces) for v in p}
    for p in pieces:
        ids = np.sort(new[p])
        assert ids[-1] - ids[0] == len(p) - 1
    for v in rest:
        assert all(u in sep or piece_of[u] == piece_of[v] for u in adj[v])


@pytest.mark.parametrize("mesh", ["tri", "random", "quad"])
def test_one_way_dissection_properties(mesh):
    m = {"tri": W.split_tri_mesh(20, 15, 1), "random": W.random_graph_mesh(300, 3.0, 9),
         "quad": W.quad_mesh(40, 9)}[mesh]
    c = pattern(m)
    new = O.one_way_dissection(c.n, c.rowptr, c.colidx)
    assert sorted(new) == list(range(c.n))


# ------------------------------------------------------------------ lines (Section 5.1)
def aniso_case(nt, nn, seed=3):
    m = W.aniso_quad_mesh(nt, nn)
    return m, W.assemble(m, W.natural_order(m), seed, "cfl", cfl=100.0)


def geo(m, c):
    return W.block_face_weights(m, W.natural_order(m), c.rowptr, c.colidx)


def test_lines_follow_wall_normal_columns():
    """On the boundary-layer mesh the strong couplings are wall normal, so every line is a run of
    one column (same tangential index) from the wall (layer 0) outward, layers consecutive and
    head at the wall; the lines stop before the outer, nearly isotropic layers."""
    nt, nn = 30, 40
    m, c = aniso_case(nt, nn)
    lo, lp, nl = O.find_lines(c.n, c.rowptr, c.colidx, geo(m, c), 10.0, 4.0)
    assert nl == nt
    for li in range(nl):
        cells = np.nonzero(lo == li)[0]
        cells = cells[np.argsort(lp[cells])]
        t = cells % nt
        k = cells // nt
        assert (t == t[0]).all()
        np.testing.assert_array_equal(k, np.arange(len(k)))
        assert 5 < len(k) < nn
    assert (lo[(np.arange(c.n) // nt) == nn - 1] == -1).all()


def test_no_lines_on_isotropic_mesh():
    m = W.quad_mesh(20, 20)
    c = pattern(m)
    lo, lp, nl = O.find_lines(c.n, c.rowptr, c.colidx, geo(m, c), 10.0, 4.0)
    assert nl == 0 and (lo == -1).all() and (lp == -1).all()
    # the matrix itself (random face weights in [0.5, 1.5]) is not anisotropic either
    c2 = W.assemble(m, W.natural_order(m), 4, "cfl", cfl=100.0)
    lo, lp, nl = O.find_lines(c2.n, c2.rowptr, c2.colidx, block_1norm(c2.vals), 10.0, 4.0)
    assert nl == 0


def test_line_orderings_keep_lines_contiguous_and_hybrid_of_full_columns():
    """Line ordering and hybrid line-X orderings place every line's cells consecutively, head to
    tail. With lines of full columns the graph of lines is a path along the wall, so line-RCM
    orders the columns along the wall (one direction or the other)."""
    nt, nn = 25, 12
    m, c = aniso_case(nt, nn)
    lo, lp, nl = O.find_lines(c.n, c.rowptr, c.colidx, geo(m, c), 1.0, 1.5)
    for new in (O.line_order(c.n, lo, lp), O.hybrid_line_order(c.n, c.rowptr, c.colidx, lo, lp, "rcm"),
                O.hybrid_line_order(c.n, c.rowptr, c.colidx, lo, lp, "1wd")):
        assert sorted(new) == list(range(c.n))
        for li in range(nl):
            cells = np.nonzero(lo == li)[0]
            cells = cells[np.argsort(lp[cells])]
            np.testing.assert_array_equal(np.diff(new[cells]), np.ones(len(cells) - 1))
    full = all((lo[(np.arange(c.n) % nt) == t] >= 0).all() for t in range(nt)) and nl == nt
    if full:
        new = O.hybrid_line_order(c.n, c.rowptr, c.colidx, lo, lp, "rcm")
        first = [new[t] for t in range(nt)]      # wall cell of column t opens its line
        d = np.diff(first)
        assert (d == nn).all() or (d == -nn).all()
