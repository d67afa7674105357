// Host-side integer phases (octree, partition, the five orderings, symbolic
// fill) on awkward inputs under AddressSanitizer and UBSan: tiny and
// single-point clouds, collinear and coincident points, a thin plate, leaf
// sizes 1-96. Checks the invariants the GPU path relies on (permutations,
// sorted near pairs, filled rows above the diagonal, elimination-tree parent
// = first entry of S_k) and that bad input is rejected by an exception.
// Built and run by tests/test_host_sanitizers.py with g++ only.
#include "plan.h"
#include <cmath>
#include <cstdio>
#include <random>
#include <algorithm>
#include <stdexcept>

static void check(bool c, const char* what) { if (!c) { std::fprintf(stderr, "FAIL %s\n", what); std::exit(1); } }

static std::vector<double> cloud(int kind, int n, std::mt19937_64& g) {
    std::vector<double> p(3 * (size_t)n);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int i = 0; i < n; ++i) {
        double x = u(g), y = u(g), z = u(g);
        if (kind == 1) { double r = std::sqrt(x*x + y*y + z*z) + 1e-12; x /= r; y /= r; z /= r; }   // sphere
        if (kind == 2) z = 0.025 * z;                     // thin plate
        if (kind == 3) { y = 0; z = 0; }                  // collinear
        if (kind == 4) { x = std::floor(x * 3) / 3; y = std::floor(y * 3) / 3; z = std::floor(z * 3) / 3; }  // coincident clusters
        p[3*i] = x; p[3*i+1] = y; p[3*i+2] = z;
    }
    return p;
}

int main() {
    std::mt19937_64 g(7);
    const int ns[] = {1, 2, 3, 17, 200, 1500, 6000};
    const int leaves[] = {1, 2, 3, 5, 24, 64, 96};
    long cases = 0, rejected = 0;
    for (int kind = 0; kind < 5; ++kind)
        for (int n : ns)
            for (int leaf : leaves) {
                if (n > 1500 && leaf < 5) continue;
                auto pts = cloud(kind, n, g);
                hs::Tree t;
                try {
                    t = hs::build_tree(pts.data(), n, leaf);
                } catch (const std::invalid_argument& e) {
                    ++rejected;   // e.g. a cloud with no extent
                    continue;
                }
                std::vector<int64_t> seen(n, 0);
                for (auto v : t.perm) { check(v >= 0 && v < n, "perm range"); seen[v]++; }
                for (auto s : seen) check(s == 1, "perm");
                int64_t tot = 0;
                for (int64_t l = 0; l < t.nb(); ++l) { tot += t.count[t.leaf_box[l]]; }
                check(tot == n, "leaves cover");
                hs::Partition p = hs::build_partition(t);
                for (int64_t e = 0; e < p.n_near(); ++e) check(p.near[2*e] <= p.near[2*e+1] && p.near[2*e+1] < t.nb(), "near pair");
                for (int ord = 0; ord <= 4; ++ord) {
                    auto o = hs::make_order(ord, t.nb(), p);
                    std::vector<int64_t> s2(t.nb(), 0);
                    for (auto v : o) { check(v >= 0 && v < t.nb(), "order range"); s2[v]++; }
                    for (auto s : s2) check(s == 1, "order perm");
                    hs::Symbolic sy = hs::symbolic(t.nb(), p, o);
                    check((int64_t)sy.rowptr.size() == t.nb() + 1, "rowptr");
                    for (int64_t k = 0; k < t.nb(); ++k) {
                        for (int64_t e = sy.rowptr[k]; e < sy.rowptr[k+1]; ++e) {
                            check(sy.cols[e] > k && sy.cols[e] < t.nb(), "cols");
                            if (e > sy.rowptr[k]) check(sy.cols[e] > sy.cols[e-1], "sorted");
                        }
                        const int64_t par = sy.rowptr[k+1] > sy.rowptr[k] ? sy.cols[sy.rowptr[k]] : -1;
                        check(sy.parent[k] == par, "parent");
                    }
                    ++cases;
                }
            }
    // bad input is rejected, not read out of bounds
    bool threw = false;
    try { std::vector<double> q(3, 0.0); hs::build_tree(q.data(), 1, 0); } catch (const std::invalid_argument&) { threw = true; }
    check(threw, "leaf_max 0 rejected");
    std::printf("ok: %ld plan cases under the sanitizers, %ld inputs rejected\n", cases, rejected);
    return 0;
}
