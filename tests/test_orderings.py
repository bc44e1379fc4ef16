"""The library's orderings (host C++, include/abilu.h) against the ordering oracle: integers,
bit-exact. No GPU needed: the orderings run on the host."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import orderings as O
from paper_1912_00539_amd import abilu as L
from paper_1912_00539_amd import workloads as W


def meshes():
    return {
        "chain9": W.chain_mesh(9),
        "quad7x4": W.quad_mesh(7, 4),
        "quad10x100": W.quad_mesh(10, 100),
        "tri20x15": W.split_tri_mesh(20, 15, 1),
        "nine12x9": W.nine_point_mesh(12, 9),
        "random300": W.random_graph_mesh(300, 3.0, 9),
        "random_sparse": W.random_graph_mesh(200, 1.2, 4),     # several components
        "aniso40x30": W.aniso_quad_mesh(40, 30),
        "single": W.chain_mesh(1),
    }


def case_of(m, order="natural", seed=0):
    o = W.natural_order(m) if order == "natural" else W.rcm_order(m, seed)
    return W.assemble(m, o, seed, "const", s=1.0), o


@pytest.mark.parametrize("name", list(meshes()))
@pytest.mark.parametrize("order", ["natural", "rcm"])
def test_rcm_and_1wd_bit_exact(name, order):
    m = meshes()[name]
    c, _ = case_of(m, order)
    np.testing.assert_array_equal(L.abilu_order(c.n, c.rowptr, c.colidx, "rcm"), O.rcm(c.n, c.rowptr, c.colidx))
    np.testing.assert_array_equal(L.abilu_order(c.n, c.rowptr, c.colidx, "1wd"),
                                  O.one_way_dissection(c.n, c.rowptr, c.colidx))


@pytest.mark.parametrize("name,theta,rho", [("aniso40x30", 10.0, 4.0), ("aniso40x30", 3.0, 2.0),
                                           ("aniso40x30", 1.0, 1.5), ("tri20x15", 1.0, 1.2),
                                           ("random300", 1.0, 1.1), ("quad7x4", 1.0, 2.0)])
@pytest.mark.parametrize("order", ["natural", "rcm"])
def test_lines_and_line_orderings_bit_exact(name, theta, rho, order):
    m = meshes()[name]
    c, o = case_of(m, order, seed=2)
    if m.kind == "aniso_quad":
        w = W.block_face_weights(m, o, c.rowptr, c.colidx)
    else:   # matrix-derived weights: irregular couplings, many short lines
        w = np.abs(c.vals).sum(axis=1).max(axis=1)
    lo, lp, nl = L.abilu_find_lines(c.n, c.rowptr, c.colidx, w, theta, rho)
    olo, olp, onl = O.find_lines(c.n, c.rowptr, c.colidx, w, theta, rho)
    assert nl == onl
    np.testing.assert_array_equal(lo, olo)
    np.testing.assert_array_equal(lp, olp)
    np.testing.assert_array_equal(L.abilu_order(c.n, c.rowptr, c.colidx, "line", lo, lp), O.line_order(c.n, olo, olp))
    for x in ("rcm", "1wd"):
        np.testing.assert_array_equal(L.abilu_order(c.n, c.rowptr, c.colidx, f"line_{x}", lo, lp),
                                      O.hybrid_line_order(c.n, c.rowptr, c.colidx, olo, olp, x))


def test_full_size_orderings_are_permutations_with_lines_contiguous():
    """500,000-cell boundary-layer mesh (the size the measurements use): every ordering is a
    permutation, lines stay contiguous head to tail, and the lines are wall-normal runs from the
    wall (checked on every line). The oracle runs on the smaller cases above."""
    m = W.aniso_quad_mesh(1000, 500)
    c, o = case_of(m)
    w = W.block_face_weights(m, o, c.rowptr, c.colidx)
    lo, lp, nl = L.abilu_find_lines(c.n, c.rowptr, c.colidx, w, 10.0, 4.0)
    assert nl == 1000
    cells = np.nonzero(lo >= 0)[0]
    key = np.lexsort((lp[cells], lo[cells]))
    srt = cells[key]
    same_line = lo[srt][1:] == lo[srt][:-1]
    assert (srt[1:][same_line] - srt[:-1][same_line] == 1000).all()     # next layer, same column
    assert (srt[np.r_[True, ~same_line]] < 1000).all()                  # every line starts at the wall
    for name in ("rcm", "1wd", "line", "line_rcm", "line_1wd"):
        new = L.abilu_order(c.n, c.rowptr, c.colidx, name, lo, lp)
        assert np.array_equal(np.sort(new), np.arange(c.n)), name
        if name.startswith("line"):
            nsrt = new[srt]
            assert (nsrt[1:][same_line] - nsrt[:-1][same_line] == 1).all(), name


def test_order_argument_checks():
    c, _ = case_of(W.quad_mesh(4, 3))
    with pytest.raises(L.AbiluError):
        L.abilu_order(c.n, c.rowptr, c.colidx, "line")               # lines required
    bad = c.colidx.copy(); bad[3] = c.n + 5
    with pytest.raises(L.AbiluError) as ei:
        L.abilu_order(c.n, c.rowptr, bad, "rcm")
    assert ei.value.status == L.ABILU_EPATTERN
    lo = np.full(c.n, -1, np.int32); lp = np.full(c.n, -1, np.int32)
    lo[[0, 1]] = 0; lp[[0, 1]] = 0                                     # two cells at one position
    with pytest.raises(L.AbiluError):
        L.abilu_order(c.n, c.rowptr, c.colidx, "line", lo, lp)
    with pytest.raises(L.AbiluError):
        L.abilu_find_lines(c.n, c.rowptr, c.colidx, np.ones(c.nnzb), 0.5, 4.0)


# ------------------------------------------------------------------ randomized: any pattern, any weights


def random_pattern(n, edges, unsym):
    """A CSR block pattern with the diagonal, the given undirected edges (i != j), and optionally
    only one direction of some edges (the library and the oracle both symmetrise)."""
    rows = [set([i]) for i in range(n)]
    for k, (a, b) in enumerate(edges):
        if a == b:
            continue
        rows[a].add(b)
        if not (unsym and k % 3 == 0):
            rows[b].add(a)
    rp = np.zeros(n + 1, np.int32)
    for i in range(n):
        rp[i + 1] = rp[i] + len(rows[i])
    ci = np.concatenate([np.array(sorted(r), np.int32) for r in rows]) if n else np.zeros(0, np.int32)
    return rp, ci


@settings(max_examples=60, deadline=None)
@given(n=st.integers(1, 60), data=st.data(), unsym=st.booleans())
def test_orderings_random_graphs_bit_exact(n, data, unsym):
    m = data.draw(st.integers(0, 3 * n))
    edges = data.draw(st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), min_size=m, max_size=m))
    rp, ci = random_pattern(n, edges, unsym)
    np.testing.assert_array_equal(L.abilu_order(n, rp, ci, "rcm"), O.rcm(n, rp, ci))
    np.testing.assert_array_equal(L.abilu_order(n, rp, ci, "1wd"), O.one_way_dissection(n, rp, ci))
    w = np.asarray(data.draw(st.lists(st.sampled_from([0.5, 1.0, 2.0, 7.0, 40.0, 300.0]), min_size=len(ci),
                                      max_size=len(ci))), np.float64)
    theta = data.draw(st.sampled_from([1.0, 2.0, 10.0]))
    rho = data.draw(st.sampled_from([1.5, 4.0]))
    lo, lp, nl = L.abilu_find_lines(n, rp, ci, w, theta, rho)
    olo, olp, onl = O.find_lines(n, rp, ci, w, theta, rho)
    assert nl == onl
    np.testing.assert_array_equal(lo, olo)
    np.testing.assert_array_equal(lp, olp)
    for x in ("rcm", "1wd"):
        np.testing.assert_array_equal(L.abilu_order(n, rp, ci, f"line_{x}", lo, lp),
                                      O.hybrid_line_order(n, rp, ci, olo, olp, x))
    np.testing.assert_array_equal(L.abilu_order(n, rp, ci, "line", lo, lp), O.line_order(n, olo, olp))
