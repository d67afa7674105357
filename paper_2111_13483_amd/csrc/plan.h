// Host-side integer phases: octree, near/far partition, near-field block
// ordering and the symbolic fill of the scaling coefficients.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hs {

constexpr int kLevels = 21;

struct Tree {
    int64_t n = 0;
    std::vector<int64_t> perm;      // tree position -> caller index
    std::vector<int64_t> keys;      // Morton keys in tree order
    std::vector<int64_t> level, start, count, parent, leaf_id;   // per box, preorder
    std::vector<int64_t> anchor;    // nbox * 3
    std::vector<int64_t> child_ptr, child_idx;                   // CSR of children
    std::vector<int64_t> leaf_box;  // box of each leaf
    int64_t nbox() const { return (int64_t)level.size(); }
    int64_t nb() const { return (int64_t)leaf_box.size(); }
};

struct Partition {
    std::vector<int64_t> near;      // pairs (i, j), i <= j, sorted
    std::vector<int64_t> far;       // pairs (t, s), t < s, sorted
    int64_t n_near() const { return (int64_t)near.size() / 2; }
    int64_t n_far() const { return (int64_t)far.size() / 2; }
};

struct Symbolic {
    std::vector<int64_t> order, rank;       // new -> old, old -> new
    std::vector<int64_t> rowptr, cols;      // filled pattern S_k (new numbering, cols > k, sorted)
    std::vector<int64_t> orig;              // 1 if near-field pair, else fill-in
    std::vector<int64_t> parent;            // elimination tree
    int64_t nnz() const { return (int64_t)cols.size(); }
};

// Throws std::invalid_argument on bad input.
Tree build_tree(const double* pts, int64_t n, int leaf_max);
Partition build_partition(const Tree& t);
std::vector<int64_t> make_order(int kind, int64_t nb, const Partition& p);
Symbolic symbolic(int64_t nb, const Partition& p, const std::vector<int64_t>& order);

}  // namespace hs
