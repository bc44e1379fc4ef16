"""Orderings of mesh cells (Section 5): plain Python reference implementations.

TEST INFRASTRUCTURE ONLY: only tests/ and the benchmark may import this module. It shares no code
with the library (paper_1912_00539_amd), whose C++ implementations must give the same integers.

Graphs are undirected and come from a block pattern: the neighbours of cell i are the columns j != i
of row i together with the rows that hold column i (the pattern is symmetrised). Everything below is
deterministic; every tie is broken by the lower index.

  * rooted level structure: breadth-first levels from a root inside a vertex subset;
  * pseudo-peripheral node (George and Liu): start from the subset's lowest vertex r; take the
    level structure from r; among its last level pick the vertex x of least degree; if the level
    structure from x is deeper, set r = x and repeat, otherwise r is the result;
  * Cuthill-McKee from a root: breadth first, the unvisited neighbours of each vertex appended in
    increasing (degree, index); reverse Cuthill-McKee (RCM) reverses it. Degrees count neighbours
    inside the subset. Components are taken in increasing order of their lowest vertex, each
    reversed on its own;
  * one-way dissection (George): per component, the level structure from a pseudo-peripheral node
    (L levels, |C| vertices); with width w = |C|/L and delta = sqrt((3w + 13)/2), levels
    j_k = floor(k delta + 1/2), k = 1, 2, ..., j_k <= L - 2, are separator levels, and the vertices
    of a separator level with a neighbour in the next level form the separator. The components
    left after removing the separators are numbered first, each by RCM, in increasing (lowest
    level, lowest vertex); the separator vertices follow, by level then index. Components with
    fewer than 3 levels, or whose delta leaves no separator level, are numbered by RCM;
  * lines of anisotropic cells (Section 5.1): coupling c_ij = w_ij + w_ji from per-block weights;
    a cell is anisotropic when max_j c_ij / min_j c_ij >= theta; (i, j) is a strong link when c_ij
    is at least 1/rho of both cells' largest coupling. Seeds are the anisotropic cells in
    decreasing anisotropy; a line grows from its seed at its tail, then at its head, each step to
    the unassigned anisotropic neighbour with the strongest strong link; lines of one cell are
    dropped (the cell stays isotropic);
  * line ordering: cells in their order, each line placed whole (head to tail) where its first
    cell comes; hybrid line-X (Section 5.2): the graph whose vertices are the lines and the
    isotropic cells, joined when any of their cells are neighbours, ordered by X, then expanded.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def adjacency(n, rowptr, colidx):
    """Sorted neighbour lists of the symmetrised pattern (self loops removed)."""
    nb = [set() for _ in range(n)]
    for i in range(n):
        for e in range(int(rowptr[i]), int(rowptr[i + 1])):
            j = int(colidx[e])
            if j != i:
                nb[i].add(j)
                nb[j].add(i)
    return [sorted(s) for s in nb]


def level_structure(adj, root, inside):
    """Levels (lists) of the breadth-first search from root over vertices with inside[v]."""
    seen = {root}
    levels = [[root]]
    while True:
        nxt = []
        for v in levels[-1]:
            for u in adj[v]:
                if inside[u] and u not in seen:
                    seen.add(u)
                    nxt.append(u)
        if not nxt:
            return levels
        levels.append(nxt)


def _deg(adj, v, inside):
    return sum(1 for u in adj[v] if inside[u])


def pseudo_peripheral(adj, start, inside):
    r = start
    lv = level_structure(adj, r, inside)
    while True:
        x = min(lv[-1], key=lambda v: (_deg(adj, v, inside), v))
        lx = level_structure(adj, x, inside)
        if len(lx) > len(lv):
            r, lv = x, lx
        else:
            return r


def _components(adj, verts, inside):
    """Components of the subgraph on `verts` (sorted), in increasing order of their lowest vertex."""
    seen = set()
    out = []
    for v in verts:
        if v in seen:
            continue
        comp = [v]
        seen.add(v)
        q = deque([v])
        while q:
            a = q.popleft()
            for u in adj[a]:
                if inside[u] and u not in seen:
                    seen.add(u)
                    comp.append(u)
                    q.append(u)
        out.append(sorted(comp))
    return out


def _cm(adj, root, inside):
    order = [root]
    seen = {root}
    h = 0
    while h < len(order):
        v = order[h]
        h += 1
        new = [u for u in adj[v] if inside[u] and u not in seen]
        new.sort(key=lambda u: (_deg(adj, u, inside), u))
        for u in new:
            seen.add(u)
            order.append(u)
    return order


def rcm_subset(adj, verts, inside):
    out = []
    for comp in _components(adj, verts, inside):
        r = pseudo_peripheral(adj, comp[0], inside)
        out.extend(reversed(_cm(adj, r, inside)))
    return out


def one_way_dissection_subset(adj, verts, inside):
    out = []
    for comp in _components(adj, verts, inside):
        r = pseudo_peripheral(adj, comp[0], inside)
        lv = level_structure(adj, r, inside)
        L = len(lv)
        if L < 3:
            out.extend(rcm_subset(adj, comp, inside))
            continue
        w = len(comp) / L
        delta = ((3.0 * w + 13.0) / 2.0) ** 0.5
        seps = []
        k = 1
        while True:
            j = int(np.floor(k * delta + 0.5))
            if j > L - 2:
                break
            if not seps or seps[-1] != j:
                seps.append(j)
            k += 1
        if not seps:
            out.extend(rcm_subset(adj, comp, inside))
            continue
        level_of = {}
        for li, lvl in enumerate(lv):
            for v in lvl:
                level_of[v] = li
        sep_nodes = []
        is_sep = set()
        for j in seps:
            nxt = set(lv[j + 1])
            for v in sorted(lv[j]):
                if any(inside[u] and u in nxt for u in adj[v]):
                    sep_nodes.append(v)
                    is_sep.add(v)
        inner = [False] * len(inside)
        rest = [v for v in comp if v not in is_sep]
        for v in rest:
            inner[v] = True
        blocks = _components(adj, rest, inner)
        blocks.sort(key=lambda b: (min(level_of[v] for v in b), b[0]))
        for b in blocks:
            binside = [False] * len(inside)
            for v in b:
                binside[v] = True
            out.extend(rcm_subset(adj, b, binside))
        out.extend(sep_nodes)
    return out


def rcm(n, rowptr, colidx):
    """new_of_old of RCM on the cell graph."""
    adj = adjacency(n, rowptr, colidx)
    return _new_of_old(rcm_subset(adj, list(range(n)), [True] * n), n)


def one_way_dissection(n, rowptr, colidx):
    adj = adjacency(n, rowptr, colidx)
    return _new_of_old(one_way_dissection_subset(adj, list(range(n)), [True] * n), n)


def _new_of_old(order, n):
    assert sorted(order) == list(range(n))
    new = np.empty(n, np.int64)
    new[np.asarray(order, np.int64)] = np.arange(n)
    return new


def find_lines(n, rowptr, colidx, weight, theta, rho):
    """(line_of[n], line_pos[n], nlines): line id and position in it, -1 for isotropic cells."""
    adj = adjacency(n, rowptr, colidx)
    wd = {}
    for i in range(n):
        for e in range(int(rowptr[i]), int(rowptr[i + 1])):
            j = int(colidx[e])
            if j != i:
                wd[(i, j)] = float(weight[e])
    c = {}
    for i in range(n):
        for j in adj[i]:
            c[(i, j)] = wd.get((i, j), 0.0) + wd.get((j, i), 0.0)
    cmax = [max((c[(i, j)] for j in adj[i]), default=0.0) for i in range(n)]
    cmin = [min((c[(i, j)] for j in adj[i]), default=0.0) for i in range(n)]
    alpha = []
    for i in range(n):
        if not adj[i]:
            alpha.append(1.0)
        elif cmin[i] > 0:
            alpha.append(cmax[i] / cmin[i])
        else:
            alpha.append(float("inf"))
    aniso = [a >= theta for a in alpha]

    def strong(i, j):
        return c[(i, j)] >= cmax[i] / rho and c[(i, j)] >= cmax[j] / rho

    line_of = [-1] * n
    assigned = [False] * n
    lines = []

    def step(e):
        best, bc = -1, -1.0
        for j in adj[e]:
            if not assigned[j] and aniso[j] and strong(e, j) and c[(e, j)] > bc:
                best, bc = j, c[(e, j)]
        return best

    for s in sorted((i for i in range(n) if aniso[i]), key=lambda i: (-alpha[i], i)):
        if assigned[s]:
            continue
        line = deque([s])
        assigned[s] = True
        while True:
            j = step(line[-1])
            if j < 0:
                break
            assigned[j] = True
            line.append(j)
        while True:
            j = step(line[0])
            if j < 0:
                break
            assigned[j] = True
            line.appendleft(j)
        if len(line) < 2:
            assigned[s] = False
            continue
        for v in line:
            line_of[v] = len(lines)
        lines.append(list(line))
    line_pos = [-1] * n
    for li in lines:
        for p, v in enumerate(li):
            line_pos[v] = p
    return np.asarray(line_of, np.int32), np.asarray(line_pos, np.int32), len(lines)


def _units(n, line_of, line_pos):
    """Lines and isotropic cells in order of their first cell: list of cell lists."""
    members = {}
    for v in range(n):
        if line_of[v] >= 0:
            members.setdefault(int(line_of[v]), []).append(v)
    for k in members:
        members[k].sort(key=lambda v: line_pos[v])
    units, unit_of, done = [], [0] * n, set()
    for v in range(n):
        if line_of[v] < 0:
            unit_of[v] = len(units)
            units.append([v])
        elif int(line_of[v]) not in done:
            done.add(int(line_of[v]))
            for u in members[int(line_of[v])]:
                unit_of[u] = len(units)
            units.append(members[int(line_of[v])])
    return units, unit_of


def line_order(n, line_of, line_pos):
    units, _ = _units(n, line_of, line_pos)
    return _new_of_old([v for u in units for v in u], n)


def hybrid_line_order(n, rowptr, colidx, line_of, line_pos, x="rcm"):
    """Hybrid line-X ordering: X = 'rcm' or '1wd' on the graph of lines and isotropic cells."""
    units, unit_of = _units(n, line_of, line_pos)
    adj = adjacency(n, rowptr, colidx)
    m = len(units)
    uadj = [set() for _ in range(m)]
    for v in range(n):
        for u in adj[v]:
            a, b = unit_of[v], unit_of[u]
            if a != b:
                uadj[a].add(b)
    uadj = [sorted(s) for s in uadj]
    fn = rcm_subset if x == "rcm" else one_way_dissection_subset
    uorder = fn(uadj, list(range(m)), [True] * m)
    return _new_of_old([v for k in uorder for v in units[k]], n)


def bandwidth(n, rowptr, colidx, new_of_old):
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    return int(np.max(np.abs(new_of_old[rows] - new_of_old[np.asarray(colidx)]))) if len(colidx) else 0
