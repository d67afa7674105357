// Host integer phases (compiled without floating-point contraction so the
// quantisation rounds exactly as written).
//
// Octree (Sec. 2): root cube from the bounding box, 21-bit quantisation,
// Morton keys, stable sort, adaptive 8-way split while a box holds more
// than leaf_max points. Partition (Eq. 8, Fig. 1) with adjacency
// admissibility by symmetric dual traversal. Ordering (Algorithm 1):
// Cuthill-McKee from a George-Liu pseudo-peripheral node, reversed for
// RCM; Sloan's and King's profile-reducing orderings from the same start.
// Symbolic fill (Sec. 3.3): row patterns of the eliminated leaf graph
// via the elimination tree.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <stdexcept>

namespace hs {

namespace {

constexpr int64_t kQMax = (int64_t(1) << kLevels) - 1;

// Bit i of a 21-bit value moved to bit 3 i, by the usual shift-and-mask
// steps (each halves the width of the bit groups: 16, 8, 4, 2, 1).
uint64_t spread3(uint64_t v) {
    static_assert(kLevels == 21, "the masks below are for 21-bit coordinates");
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// bit i of qx, qy, qz at bits 3 i, 3 i + 1, 3 i + 2
int64_t morton3(int64_t qx, int64_t qy, int64_t qz) {
    return (int64_t)(spread3((uint64_t)qx) | spread3((uint64_t)qy) << 1 | spread3((uint64_t)qz) << 2);
}

}  // namespace

Tree build_tree(const double* pts, int64_t n, int leaf_max) {
    if (n < 1) throw std::invalid_argument("n must be >= 1");
    if (leaf_max < 1) throw std::invalid_argument("leaf_max must be >= 1");
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = pts[a]; hi[a] = pts[a]; }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = pts[3 * i + a];
            if (!std::isfinite(v)) throw std::invalid_argument("non-finite point coordinate");
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    if (!(ext > 0.0)) throw std::invalid_argument("points span no volume");
    double o[3];
    for (int a = 0; a < 3; ++a) {
        double c = (lo[a] + hi[a]) / 2.0;
        o[a] = c - ext / 2.0;
    }
    const double scale = double(int64_t(1) << kLevels) / ext;
    std::vector<int64_t> q(3 * n), key(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double t = (pts[3 * i + a] - o[a]) * scale;
            double f = std::floor(t);
            int64_t v = f < 0.0 ? 0 : (f > double(kQMax) ? kQMax : (int64_t)f);
            q[3 * i + a] = v;
        }
        key[i] = morton3(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
    }
    Tree t;
    t.n = n;
    // points by key, equal keys in input order: an LSD radix sort, 16 bits
    // a pass (the same order as a stable comparison sort, in a fraction of
    // its time at tens of thousands of points)
    t.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
    {
        int64_t mx = 0;
        for (int64_t i = 0; i < n; ++i) mx = std::max(mx, key[i]);
        std::vector<int64_t> tmp(n);
        std::vector<int64_t> cnt(int64_t(1) << 16);
        for (int shift = 0; shift < 64 && (mx >> shift) != 0; shift += 16) {
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t i = 0; i < n; ++i) ++cnt[(key[i] >> shift) & 0xffff];
            int64_t sum = 0;
            for (auto& c : cnt) {
                const int64_t v = c;
                c = sum;
                sum += v;
            }
            for (int64_t i = 0; i < n; ++i) {
                const int64_t v = t.perm[i];
                tmp[cnt[(key[v] >> shift) & 0xffff]++] = v;
            }
            t.perm.swap(tmp);
        }
    }
    t.keys.resize(n);
    std::vector<int64_t> qs(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        t.keys[i] = key[t.perm[i]];
        for (int a = 0; a < 3; ++a) qs[3 * i + a] = q[3 * t.perm[i] + a];
    }
    std::vector<std::vector<int64_t>> children;
    std::function<int64_t(int64_t, int64_t, int64_t, int64_t)> visit =
        [&](int64_t lvl, int64_t s, int64_t c, int64_t par) -> int64_t {
        int64_t bid = t.nbox();
        t.level.push_back(lvl);
        t.start.push_back(s);
        t.count.push_back(c);
        for (int a = 0; a < 3; ++a) t.anchor.push_back(qs[3 * s + a] >> (kLevels - lvl));
        t.parent.push_back(par);
        t.leaf_id.push_back(-1);
        children.emplace_back();
        if (c > leaf_max && lvl < kLevels) {
            const int shift = 3 * (kLevels - (int)lvl - 1);
            int64_t p = s;
            const int64_t e = s + c;
            while (p < e) {
                int64_t oct = (t.keys[p] >> shift) & 7;
                int64_t r = p;
                while (r < e && ((t.keys[r] >> shift) & 7) == oct) ++r;
                int64_t cid = visit(lvl + 1, p, r - p, bid);
                children[bid].push_back(cid);
                p = r;
            }
        } else {
            t.leaf_id[bid] = t.nb();
            t.leaf_box.push_back(bid);
        }
        return bid;
    };
    visit(0, 0, n, -1);
    t.child_ptr.assign(1, 0);
    for (auto& ch : children) {
        for (int64_t c : ch) t.child_idx.push_back(c);
        t.child_ptr.push_back((int64_t)t.child_idx.size());
    }
    return t;
}

namespace {

bool adjacent(const Tree& t, int64_t a, int64_t b) {
    const int64_t sa = int64_t(1) << (kLevels - t.level[a]);
    const int64_t sb = int64_t(1) << (kLevels - t.level[b]);
    for (int x = 0; x < 3; ++x) {
        int64_t la = t.anchor[3 * a + x] * sa, lb = t.anchor[3 * b + x] * sb;
        if (!(la <= lb + sb && lb <= la + sa)) return false;
    }
    return true;
}

void sort_pairs(std::vector<int64_t>& v) {
    size_t m = v.size() / 2;
    std::vector<std::pair<int64_t, int64_t>> p(m);
    for (size_t i = 0; i < m; ++i) p[i] = {v[2 * i], v[2 * i + 1]};
    std::sort(p.begin(), p.end());
    for (size_t i = 0; i < m; ++i) { v[2 * i] = p[i].first; v[2 * i + 1] = p[i].second; }
}

}  // namespace

Partition build_partition(const Tree& t) {
    Partition p;
    auto is_leaf = [&](int64_t b) { return t.leaf_id[b] >= 0; };
    std::function<void(int64_t, int64_t)> T = [&](int64_t a, int64_t b) {
        if (a == b) {
            if (is_leaf(a)) {
                p.near.push_back(t.leaf_id[a]);
                p.near.push_back(t.leaf_id[a]);
                return;
            }
            for (int64_t x = t.child_ptr[a]; x < t.child_ptr[a + 1]; ++x)
                for (int64_t y = x; y < t.child_ptr[a + 1]; ++y) T(t.child_idx[x], t.child_idx[y]);
            return;
        }
        if (!adjacent(t, a, b)) {
            p.far.push_back(a);
            p.far.push_back(b);
            return;
        }
        bool la = is_leaf(a), lb = is_leaf(b);
        if (la && lb) {
            p.near.push_back(t.leaf_id[a]);
            p.near.push_back(t.leaf_id[b]);
        } else if (!la && !lb) {
            for (int64_t x = t.child_ptr[a]; x < t.child_ptr[a + 1]; ++x)
                for (int64_t y = t.child_ptr[b]; y < t.child_ptr[b + 1]; ++y) T(t.child_idx[x], t.child_idx[y]);
        } else if (!la) {
            for (int64_t x = t.child_ptr[a]; x < t.child_ptr[a + 1]; ++x) T(t.child_idx[x], b);
        } else {
            for (int64_t y = t.child_ptr[b]; y < t.child_ptr[b + 1]; ++y) T(a, t.child_idx[y]);
        }
    };
    T(0, 0);
    sort_pairs(p.near);
    sort_pairs(p.far);
    return p;
}

namespace {

struct Graph {
    std::vector<std::vector<int64_t>> adj;
    std::vector<int64_t> deg;
};

Graph leaf_graph(int64_t nb, const Partition& p) {
    Graph g;
    g.adj.resize(nb);
    for (int64_t e = 0; e < p.n_near(); ++e) {
        int64_t i = p.near[2 * e], j = p.near[2 * e + 1];
        if (i == j) continue;
        g.adj[i].push_back(j);
        g.adj[j].push_back(i);
    }
    g.deg.resize(nb);
    for (int64_t v = 0; v < nb; ++v) {
        auto& a = g.adj[v];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        g.deg[v] = (int64_t)a.size();
    }
    return g;
}

// Rooted level structure: returns the number of levels, the last level and the component size.
int64_t levels(const Graph& g, int64_t root, std::vector<int64_t>& mark, int64_t stamp,
               std::vector<int64_t>& last, int64_t& size) {
    std::vector<int64_t> cur{root}, nxt;
    mark[root] = stamp;
    int64_t nlev = 1;
    size = 1;
    for (;;) {
        nxt.clear();
        for (int64_t v : cur)
            for (int64_t w : g.adj[v])
                if (mark[w] != stamp) { mark[w] = stamp; nxt.push_back(w); }
        if (nxt.empty()) { last = cur; return nlev; }
        size += (int64_t)nxt.size();
        ++nlev;
        cur.swap(nxt);
    }
}

bool deg_less(const Graph& g, int64_t a, int64_t b) {
    return g.deg[a] != g.deg[b] ? g.deg[a] < g.deg[b] : a < b;
}

}  // namespace

namespace {

// George-Liu pseudo-peripheral node of r's component (size: its node count)
int64_t pseudo_peripheral(const Graph& g, int64_t r, std::vector<int64_t>& mark, int64_t& stamp, int64_t& size) {
    std::vector<int64_t> last;
    size = 0;
    int64_t nlev = levels(g, r, mark, stamp++, last, size);
    int64_t start = r;
    if (!(nlev == 1 || nlev == size)) {
        for (;;) {
            int64_t x = last[0];
            for (int64_t v : last) if (deg_less(g, v, x)) x = v;
            int64_t sz2 = 0;
            std::vector<int64_t> last2;
            int64_t nlev2 = levels(g, x, mark, stamp++, last2, sz2);
            if (nlev2 <= nlev) { start = x; break; }
            r = x; nlev = nlev2; last.swap(last2);
            start = r;
            if (nlev >= size) break;
        }
    }
    return start;
}

// Sloan's ordering of one component from start s (statuses, priorities
// P = w1 dist(e) - w2 (deg + 1), largest priority first, ties to the lowest id)
void sloan_component(const Graph& g, int64_t s, std::vector<int64_t>& mark, int64_t& stamp,
                     std::vector<int>& status, std::vector<int64_t>& prio, std::vector<int64_t>& order) {
    constexpr int64_t W1 = 1, W2 = 2;
    enum { INACT = 0, PRE = 1, ACT = 2, POST = 3 };
    std::vector<int64_t> last;
    int64_t size = 0;
    levels(g, s, mark, stamp++, last, size);
    int64_t e = last[0];
    for (int64_t v : last) if (deg_less(g, v, e)) e = v;
    // distances from e (breadth-first levels of e's component)
    std::vector<int64_t> cur{e}, nxt;
    const int64_t st = stamp++;
    mark[e] = st;
    for (int64_t d = 0; !cur.empty(); ++d) {
        nxt.clear();
        for (int64_t v : cur) {
            prio[v] = W1 * d - W2 * (g.deg[v] + 1);
            for (int64_t w : g.adj[v])
                if (mark[w] != st) { mark[w] = st; nxt.push_back(w); }
        }
        cur.swap(nxt);
    }
    // queue of preactive and active nodes: a max-heap on (priority, -id)
    // with one entry per priority change; stale entries are skipped
    typedef std::pair<int64_t, int64_t> Ent;   // (priority, -id)
    std::vector<Ent> heap;
    auto push = [&](int64_t v) {
        heap.push_back({prio[v], -v});
        std::push_heap(heap.begin(), heap.end());
    };
    status[s] = PRE;
    push(s);
    while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end());
        const Ent top = heap.back();
        heap.pop_back();
        const int64_t i = -top.second;
        if (status[i] == POST || status[i] == INACT || prio[i] != top.first) continue;
        if (status[i] == PRE) {
            for (int64_t j : g.adj[i]) {
                prio[j] += W2;
                if (status[j] == INACT) status[j] = PRE;
                if (status[j] == PRE || status[j] == ACT) push(j);
            }
        }
        order.push_back(i);
        status[i] = POST;
        for (int64_t j : g.adj[i]) {
            if (status[j] != PRE) continue;
            status[j] = ACT;
            prio[j] += W2;
            push(j);
            for (int64_t k : g.adj[j]) {
                if (status[k] == POST) continue;
                prio[k] += W2;
                if (status[k] == INACT) status[k] = PRE;
                push(k);
            }
        }
    }
}

// King's ordering of one component from start s: number, from the front,
// the node adding the fewest new front nodes, ties to the lowest id
void king_component(const Graph& g, int64_t s, std::vector<char>& numbered, std::vector<char>& infront,
                    std::vector<int64_t>& order) {
    std::vector<int64_t> front;
    int64_t nxt = s;
    while (nxt >= 0) {
        numbered[nxt] = 1;
        if (infront[nxt]) {
            infront[nxt] = 0;
            front.erase(std::find(front.begin(), front.end(), nxt));
        }
        order.push_back(nxt);
        for (int64_t w : g.adj[nxt])
            if (!numbered[w] && !infront[w]) { infront[w] = 1; front.push_back(w); }
        nxt = -1;
        int64_t best = 0;
        for (int64_t v : front) {
            int64_t add = 0;
            for (int64_t w : g.adj[v]) add += (!numbered[w] && !infront[w]) ? 1 : 0;
            if (nxt < 0 || add < best || (add == best && v < nxt)) { nxt = v; best = add; }
        }
    }
}

}  // namespace

std::vector<int64_t> make_order(int kind, int64_t nb, const Partition& p) {
    std::vector<int64_t> order;
    order.reserve(nb);
    if (kind == 0) {
        for (int64_t i = 0; i < nb; ++i) order.push_back(i);
        return order;
    }
    if (kind < 1 || kind > 4) throw std::invalid_argument("unknown ordering");
    Graph g = leaf_graph(nb, p);
    std::vector<char> visited(nb, 0), infront(nb, 0);
    std::vector<int64_t> mark(nb, -1), prio(nb, 0);
    std::vector<int> status(nb, 0);
    int64_t stamp = 0;
    // candidates in (degree, id) order for picking each component's first node
    std::vector<int64_t> cand(nb);
    for (int64_t i = 0; i < nb; ++i) cand[i] = i;
    std::sort(cand.begin(), cand.end(), [&](int64_t a, int64_t b) { return deg_less(g, a, b); });
    size_t cpos = 0;
    while ((int64_t)order.size() < nb) {
        while (visited[cand[cpos]]) ++cpos;
        int64_t size = 0;
        const int64_t start = pseudo_peripheral(g, cand[cpos], mark, stamp, size);
        const size_t head0 = order.size();
        if (kind == 3) {
            sloan_component(g, start, mark, stamp, status, prio, order);
        } else if (kind == 4) {
            king_component(g, start, visited, infront, order);
        } else {
            // breadth-first search, neighbours in (degree, id) order
            size_t head = order.size();
            visited[start] = 1;
            order.push_back(start);
            std::vector<int64_t> nbrs;
            while (head < order.size()) {
                int64_t v = order[head++];
                nbrs.clear();
                for (int64_t w : g.adj[v]) if (!visited[w]) nbrs.push_back(w);
                std::sort(nbrs.begin(), nbrs.end(), [&](int64_t a, int64_t b) { return deg_less(g, a, b); });
                for (int64_t w : nbrs) { visited[w] = 1; order.push_back(w); }
            }
        }
        for (size_t q = head0; q < order.size(); ++q) visited[order[q]] = 1;
    }
    if (kind == 1) std::reverse(order.begin(), order.end());
    return order;
}

Symbolic symbolic(int64_t nb, const Partition& p, const std::vector<int64_t>& order) {
    Symbolic s;
    s.order = order;
    s.rank.assign(nb, -1);
    for (int64_t k = 0; k < nb; ++k) {
        if (order[k] < 0 || order[k] >= nb || s.rank[order[k]] != -1)
            throw std::invalid_argument("order is not a permutation");
        s.rank[order[k]] = k;
    }
    Graph g = leaf_graph(nb, p);
    std::vector<std::vector<int64_t>> kids(nb);
    std::vector<int64_t> mark(nb, -1), row;
    s.rowptr.assign(1, 0);
    s.parent.assign(nb, -1);
    std::vector<std::vector<int64_t>> rows(nb);
    for (int64_t k = 0; k < nb; ++k) {
        row.clear();
        for (int64_t w : g.adj[order[k]]) {
            int64_t j = s.rank[w];
            if (j > k && mark[j] != k) { mark[j] = k; row.push_back(j); }
        }
        for (int64_t c : kids[k])
            for (int64_t j : rows[c])
                if (j > k && mark[j] != k) { mark[j] = k; row.push_back(j); }
        std::sort(row.begin(), row.end());
        rows[k] = row;
        if (!row.empty()) {
            s.parent[k] = row[0];
            kids[row[0]].push_back(k);
        }
    }
    for (int64_t k = 0; k < nb; ++k) {
        const auto& ak = g.adj[order[k]];
        for (int64_t j : rows[k]) {
            s.cols.push_back(j);
            s.orig.push_back(std::binary_search(ak.begin(), ak.end(), order[j]) ? 1 : 0);
        }
        s.rowptr.push_back((int64_t)s.cols.size());
        std::vector<int64_t>().swap(rows[k]);   // release as we go; children already merged
    }
    return s;
}

}  // namespace hs
