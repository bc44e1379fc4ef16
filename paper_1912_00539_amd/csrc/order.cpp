// Orderings of mesh cells (Section 5): reverse Cuthill-McKee, one-way dissection, lines of
// anisotropic cells (Section 5.1), and the line and hybrid line-X orderings (Section 5.2). Host
// code: orderings are computed once per mesh, before any factorisation, as the paper does.
//
// Every routine is deterministic; every tie goes to the lower index. The graph is the symmetrised
// block pattern without its diagonal.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "abilu.h"

namespace {

using Vec = std::vector<int32_t>;

// Symmetrised adjacency in CSR form, neighbour lists ascending and unique.
struct Graph {
    int32_t n = 0;
    std::vector<int64_t> ptr;
    Vec nb;
    int32_t deg(int32_t v) const { return (int32_t)(ptr[v + 1] - ptr[v]); }
};

Graph sym_graph(int32_t n, const int32_t *rowptr, const int32_t *colidx) {
    Graph g;
    g.n = n;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = colidx[e];
            if (j != i) {
                ++cnt[i];
                ++cnt[j];
            }
        }
    std::vector<int64_t> p(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) p[i + 1] = p[i] + cnt[i];
    Vec tmp(p[n]);
    std::vector<int64_t> fill(p.begin(), p.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = colidx[e];
            if (j != i) {
                tmp[fill[i]++] = j;
                tmp[fill[j]++] = i;
            }
        }
    g.ptr.assign(n + 1, 0);
    g.nb.reserve(tmp.size() / 2 + 1);
    for (int32_t i = 0; i < n; ++i) {
        auto b = tmp.begin() + p[i], e = tmp.begin() + p[i + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        g.nb.insert(g.nb.end(), b, u);
        g.ptr[i + 1] = (int64_t)g.nb.size();
    }
    return g;
}

// Work arrays shared by the routines below. `in` marks the current vertex subset; `mark` and
// `level` are stamped per search so they never need clearing.
struct Work {
    const Graph &g;
    std::vector<char> in;
    std::vector<int32_t> mark;
    int32_t stamp = 0;
    Vec level;
    Vec sdeg;   // degree inside the subset
    explicit Work(const Graph &gr) : g(gr), in(gr.n, 0), mark(gr.n, 0), level(gr.n, 0), sdeg(gr.n, 0) {}
    int32_t fresh() { return ++stamp; }
};

void subset_degrees(Work &w, const Vec &verts) {
    for (int32_t v : verts) {
        int32_t d = 0;
        for (int64_t e = w.g.ptr[v]; e < w.g.ptr[v + 1]; ++e) d += w.in[w.g.nb[e]] ? 1 : 0;
        w.sdeg[v] = d;
    }
}

// Breadth-first levels from root inside the subset: flat vertex list, level k being
// flat[off[k] .. off[k+1]); w.level holds each reached vertex's level.
void levels(Work &w, int32_t root, Vec &flat, Vec &off) {
    const int32_t s = w.fresh();
    flat.assign(1, root);
    off.assign(1, 0);
    w.mark[root] = s;
    w.level[root] = 0;
    size_t b = 0;
    for (int32_t lv = 0; b < flat.size(); ++lv) {
        const size_t e = flat.size();
        for (size_t q = b; q < e; ++q) {
            const int32_t v = flat[q];
            for (int64_t k = w.g.ptr[v]; k < w.g.ptr[v + 1]; ++k) {
                const int32_t u = w.g.nb[k];
                if (w.in[u] && w.mark[u] != s) {
                    w.mark[u] = s;
                    w.level[u] = lv + 1;
                    flat.push_back(u);
                }
            }
        }
        off.push_back((int32_t)e);
        b = e;
    }
}

int32_t nlevels(const Vec &off) { return (int32_t)off.size() - 1; }

// George and Liu's pseudo-peripheral node finder from `start` (degrees inside the subset).
int32_t pseudo_peripheral(Work &w, int32_t start, Vec &flat, Vec &off) {
    int32_t r = start;
    levels(w, r, flat, off);
    int32_t L = nlevels(off);
    Vec f2, o2;
    while (true) {
        int32_t x = -1;
        for (int32_t q = off[L - 1]; q < off[L]; ++q) {
            const int32_t v = flat[q];
            if (x < 0 || w.sdeg[v] < w.sdeg[x] || (w.sdeg[v] == w.sdeg[x] && v < x)) x = v;
        }
        levels(w, x, f2, o2);
        if (nlevels(o2) > L) {
            r = x;
            flat.swap(f2);
            off.swap(o2);
            L = nlevels(off);
        } else {
            levels(w, r, flat, off);   // leave the level structure of the result in flat/off
            return r;
        }
    }
}

// Components of the subset listed in `verts` (ascending), in increasing order of lowest vertex.
std::vector<Vec> components(Work &w, const Vec &verts) {
    std::vector<Vec> out;
    const int32_t s = w.fresh();
    for (int32_t v0 : verts) {
        if (w.mark[v0] == s) continue;
        Vec comp{v0};
        w.mark[v0] = s;
        for (size_t h = 0; h < comp.size(); ++h) {
            const int32_t a = comp[h];
            for (int64_t k = w.g.ptr[a]; k < w.g.ptr[a + 1]; ++k) {
                const int32_t u = w.g.nb[k];
                if (w.in[u] && w.mark[u] != s) {
                    w.mark[u] = s;
                    comp.push_back(u);
                }
            }
        }
        std::sort(comp.begin(), comp.end());
        out.push_back(std::move(comp));
    }
    return out;
}

// Cuthill-McKee from root over the subset: each vertex's unvisited neighbours in increasing
// (degree inside the subset, index).
void cuthill_mckee(Work &w, int32_t root, Vec &order) {
    const int32_t s = w.fresh();
    const size_t base = order.size();
    order.push_back(root);
    w.mark[root] = s;
    Vec kids;
    for (size_t h = base; h < order.size(); ++h) {
        const int32_t v = order[h];
        kids.clear();
        for (int64_t k = w.g.ptr[v]; k < w.g.ptr[v + 1]; ++k) {
            const int32_t u = w.g.nb[k];
            if (w.in[u] && w.mark[u] != s) {
                w.mark[u] = s;
                kids.push_back(u);
            }
        }
        std::sort(kids.begin(), kids.end(), [&](int32_t a, int32_t b) {
            return w.sdeg[a] != w.sdeg[b] ? w.sdeg[a] < w.sdeg[b] : a < b;
        });
        order.insert(order.end(), kids.begin(), kids.end());
    }
}

// RCM of the subset given by `verts` (and w.in), appended to `out`.
void rcm_subset(Work &w, const Vec &verts, Vec &out) {
    subset_degrees(w, verts);
    const std::vector<Vec> comps = components(w, verts);
    Vec flat, off;
    for (const Vec &c : comps) {
        const int32_t r = pseudo_peripheral(w, c[0], flat, off);
        const size_t b = out.size();
        cuthill_mckee(w, r, out);
        std::reverse(out.begin() + b, out.end());
    }
}

void set_in(Work &w, const Vec &verts, char v) {
    for (int32_t x : verts) w.in[x] = v;
}

// George's one-way dissection of the subset `verts` (w.in set on it), appended to `out`.
// Components are never adjacent, so each one's searches stay inside it.
void one_way_subset(Work &w, const Vec &verts, Vec &out) {
    subset_degrees(w, verts);
    const std::vector<Vec> comps = components(w, verts);
    Vec flat, off;
    for (const Vec &c : comps) {
        pseudo_peripheral(w, c[0], flat, off);   // leaves the levels from the result in flat/off
        const int32_t L = nlevels(off);
        std::vector<int32_t> seps;
        if (L >= 3) {
            const double width = (double)c.size() / (double)L;
            const double delta = std::sqrt((3.0 * width + 13.0) / 2.0);
            for (int k = 1;; ++k) {
                const int32_t j = (int32_t)std::floor(k * delta + 0.5);
                if (j > L - 2) break;
                if (seps.empty() || seps.back() != j) seps.push_back(j);
            }
        }
        if (seps.empty()) {
            rcm_subset(w, c, out);
            continue;
        }
        // separator: the vertices of a separator level with a neighbour in the next level
        Vec sep_nodes;
        for (int32_t j : seps) {
            Vec lvl(flat.begin() + off[j], flat.begin() + off[j + 1]);
            std::sort(lvl.begin(), lvl.end());
            for (int32_t v : lvl) {
                bool adj_next = false;
                for (int64_t k = w.g.ptr[v]; k < w.g.ptr[v + 1] && !adj_next; ++k) {
                    const int32_t u = w.g.nb[k];
                    adj_next = w.in[u] && w.level[u] == j + 1;
                }
                if (adj_next) sep_nodes.push_back(v);
            }
        }
        Vec lev_of_c(c.size());   // c is ascending
        for (size_t q = 0; q < c.size(); ++q) lev_of_c[q] = w.level[c[q]];
        for (int32_t v : sep_nodes) w.in[v] = 0;
        Vec rest;
        rest.reserve(c.size());
        for (int32_t v : c)
            if (w.in[v]) rest.push_back(v);
        const std::vector<Vec> blocks = components(w, rest);
        // blocks in increasing (lowest level, lowest vertex)
        std::vector<std::pair<std::pair<int32_t, int32_t>, size_t>> key(blocks.size());
        for (size_t b = 0; b < blocks.size(); ++b) {
            int32_t ml = std::numeric_limits<int32_t>::max();
            for (int32_t v : blocks[b]) {
                const size_t q = (size_t)(std::lower_bound(c.begin(), c.end(), v) - c.begin());
                ml = std::min(ml, lev_of_c[q]);
            }
            key[b] = {{ml, blocks[b][0]}, b};
        }
        std::sort(key.begin(), key.end());
        set_in(w, rest, 0);
        for (const auto &kb : key) {   // each block by RCM, degrees inside the block
            const Vec &blk = blocks[kb.second];
            set_in(w, blk, 1);
            rcm_subset(w, blk, out);
            set_in(w, blk, 0);
        }
        out.insert(out.end(), sep_nodes.begin(), sep_nodes.end());
        set_in(w, c, 1);
    }
}

bool pattern_ok(int32_t n, const int32_t *rowptr, const int32_t *colidx) {
    if (rowptr[0] != 0) return false;
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return false;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colidx[e] < 0 || colidx[e] >= n) return false;
    }
    return true;
}

void to_new_of_old(const Vec &order, int32_t *new_of_old) {
    for (size_t k = 0; k < order.size(); ++k) new_of_old[order[k]] = (int32_t)k;
}

// Lines and isotropic cells in order of their first cell: flat cell list with unit offsets.
bool units(int32_t n, const int32_t *line_of, const int32_t *line_pos, Vec &cells, Vec &uoff, Vec &unit_of) {
    int32_t nl = 0;
    for (int32_t v = 0; v < n; ++v) nl = std::max(nl, line_of[v] + 1);
    std::vector<int32_t> len(nl, 0);
    for (int32_t v = 0; v < n; ++v)
        if (line_of[v] >= 0) ++len[line_of[v]];
    std::vector<int64_t> lstart(nl + 1, 0);
    for (int32_t l = 0; l < nl; ++l) lstart[l + 1] = lstart[l] + len[l];
    Vec members(lstart[nl], -1);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t l = line_of[v];
        if (l < 0) continue;
        const int32_t p = line_pos[v];
        if (p < 0 || p >= len[l] || members[lstart[l] + p] != -1) return false;
        members[lstart[l] + p] = v;
    }
    cells.clear();
    uoff.assign(1, 0);
    unit_of.assign(n, -1);
    std::vector<char> placed(nl, 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t l = line_of[v];
        if (l < 0) {
            unit_of[v] = (int32_t)uoff.size() - 1;
            cells.push_back(v);
            uoff.push_back((int32_t)cells.size());
        } else if (!placed[l]) {
            placed[l] = 1;
            for (int64_t q = lstart[l]; q < lstart[l + 1]; ++q) {
                unit_of[members[q]] = (int32_t)uoff.size() - 1;
                cells.push_back(members[q]);
            }
            uoff.push_back((int32_t)cells.size());
        }
    }
    return true;
}

}  // namespace

extern "C" abilu_status abilu_find_lines(int32_t n, const int32_t *h_rowptr, const int32_t *h_colidx,
                                         const double *h_weight, double threshold, double strong_ratio,
                                         int32_t *h_line_of, int32_t *h_line_pos, int32_t *nlines) {
    if (n < 0 || !h_rowptr || !h_line_of || !h_line_pos || !nlines) return ABILU_EINVAL;
    if (!(threshold >= 1.0) || !(strong_ratio >= 1.0)) return ABILU_EINVAL;
    const int32_t Z = n > 0 ? h_rowptr[n] : 0;
    if (Z > 0 && (!h_colidx || !h_weight)) return ABILU_EINVAL;
    if (n > 0 && !pattern_ok(n, h_rowptr, h_colidx)) return ABILU_EPATTERN;
    const Graph g = sym_graph(n, h_rowptr, h_colidx);
    // c_ij = w_ij + w_ji on the symmetrised neighbour lists
    std::vector<double> c(g.nb.size(), 0.0);
    auto slot = [&](int32_t i, int32_t j) -> int64_t {
        auto b = g.nb.begin() + g.ptr[i], e = g.nb.begin() + g.ptr[i + 1];
        return (int64_t)(std::lower_bound(b, e, j) - g.nb.begin());
    };
    std::vector<double> wd(g.nb.size(), 0.0);   // w_ij at the (i, j) slot
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = h_rowptr[i]; e < h_rowptr[i + 1]; ++e) {
            const int32_t j = h_colidx[e];
            if (j != i) wd[slot(i, j)] = h_weight[e];
        }
    for (int32_t i = 0; i < n; ++i)
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) c[k] = wd[k] + wd[slot(g.nb[k], i)];
    std::vector<double> cmax(n, 0.0), alpha(n, 1.0);
    for (int32_t i = 0; i < n; ++i) {
        if (g.deg(i) == 0) continue;
        double mx = c[g.ptr[i]], mn = c[g.ptr[i]];
        for (int64_t k = g.ptr[i] + 1; k < g.ptr[i + 1]; ++k) {
            mx = std::max(mx, c[k]);
            mn = std::min(mn, c[k]);
        }
        cmax[i] = mx;
        alpha[i] = mn > 0 ? mx / mn : std::numeric_limits<double>::infinity();
    }
    std::vector<char> aniso(n), assigned(n, 0);
    Vec seeds;
    for (int32_t i = 0; i < n; ++i) {
        aniso[i] = alpha[i] >= threshold;
        if (aniso[i]) seeds.push_back(i);
    }
    std::stable_sort(seeds.begin(), seeds.end(), [&](int32_t a, int32_t b) { return alpha[a] > alpha[b]; });
    auto step = [&](int32_t e) -> int32_t {
        int32_t best = -1;
        double bc = -1.0;
        for (int64_t k = g.ptr[e]; k < g.ptr[e + 1]; ++k) {
            const int32_t j = g.nb[k];
            if (assigned[j] || !aniso[j]) continue;
            const double cij = c[k];
            if (cij >= cmax[e] / strong_ratio && cij >= cmax[j] / strong_ratio && cij > bc) {
                best = j;
                bc = cij;
            }
        }
        return best;
    };
    for (int32_t v = 0; v < n; ++v) {
        h_line_of[v] = -1;
        h_line_pos[v] = -1;
    }
    int32_t nl = 0;
    Vec tail, head;
    for (int32_t s : seeds) {
        if (assigned[s]) continue;
        assigned[s] = 1;
        tail.assign(1, s);
        for (int32_t j; (j = step(tail.back())) >= 0;) {
            assigned[j] = 1;
            tail.push_back(j);
        }
        head.clear();
        for (int32_t j; (j = step(head.empty() ? s : head.back())) >= 0;) {
            assigned[j] = 1;
            head.push_back(j);
        }
        if (tail.size() + head.size() < 2) {
            assigned[s] = 0;
            continue;
        }
        int32_t p = 0;
        for (auto it = head.rbegin(); it != head.rend(); ++it, ++p) {
            h_line_of[*it] = nl;
            h_line_pos[*it] = p;
        }
        for (int32_t v : tail) {
            h_line_of[v] = nl;
            h_line_pos[v] = p++;
        }
        ++nl;
    }
    *nlines = nl;
    return ABILU_OK;
}

extern "C" abilu_status abilu_order(int32_t n, const int32_t *h_rowptr, const int32_t *h_colidx,
                                    const int32_t *h_line_of, const int32_t *h_line_pos, int32_t ordering,
                                    int32_t *h_new_of_old) {
    if (n < 0 || !h_rowptr || !h_new_of_old) return ABILU_EINVAL;
    if (ordering < ABILU_ORDER_RCM || ordering > ABILU_ORDER_LINE_1WD) return ABILU_EINVAL;
    const bool lines = ordering >= ABILU_ORDER_LINE;
    if (lines && (!h_line_of || !h_line_pos)) return ABILU_EINVAL;
    const int32_t Z = n > 0 ? h_rowptr[n] : 0;
    if (Z > 0 && !h_colidx) return ABILU_EINVAL;
    if (n == 0) return ABILU_OK;
    if (!pattern_ok(n, h_rowptr, h_colidx)) return ABILU_EPATTERN;
    if (lines)
        for (int32_t v = 0; v < n; ++v)
            if (h_line_of[v] < -1 || h_line_of[v] >= n) return ABILU_EINVAL;
    Vec order;
    order.reserve(n);
    if (!lines) {
        const Graph g = sym_graph(n, h_rowptr, h_colidx);
        Work w(g);
        Vec all(n);
        for (int32_t v = 0; v < n; ++v) all[v] = v;
        set_in(w, all, 1);
        if (ordering == ABILU_ORDER_RCM) rcm_subset(w, all, order);
        else one_way_subset(w, all, order);
    } else {
        Vec cells, uoff, unit_of;
        if (!units(n, h_line_of, h_line_pos, cells, uoff, unit_of)) return ABILU_EINVAL;
        const int32_t m = (int32_t)uoff.size() - 1;
        if (ordering == ABILU_ORDER_LINE) {
            order = cells;
        } else {
            // graph of lines and isotropic cells: joined when any of their cells are neighbours
            const Graph g = sym_graph(n, h_rowptr, h_colidx);
            Vec urow(m + 1, 0), ucol;
            {
                std::vector<Vec> tmp(m);
                for (int32_t v = 0; v < n; ++v)
                    for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
                        const int32_t a = unit_of[v], b = unit_of[g.nb[k]];
                        if (a != b) tmp[a].push_back(b);
                    }
                for (int32_t a = 0; a < m; ++a) {
                    std::sort(tmp[a].begin(), tmp[a].end());
                    tmp[a].erase(std::unique(tmp[a].begin(), tmp[a].end()), tmp[a].end());
                    ucol.insert(ucol.end(), tmp[a].begin(), tmp[a].end());
                    urow[a + 1] = (int32_t)ucol.size();
                }
            }
            const Graph ug = sym_graph(m, urow.data(), ucol.data());
            Work w(ug);
            Vec all(m);
            for (int32_t a = 0; a < m; ++a) all[a] = a;
            set_in(w, all, 1);
            Vec uorder;
            uorder.reserve(m);
            if (ordering == ABILU_ORDER_LINE_RCM) rcm_subset(w, all, uorder);
            else one_way_subset(w, all, uorder);
            for (int32_t a : uorder) order.insert(order.end(), cells.begin() + uoff[a], cells.begin() + uoff[a + 1]);
        }
    }
    if ((int32_t)order.size() != n) return ABILU_EINVAL;
    to_new_of_old(order, h_new_of_old);
    return ABILU_OK;
}
