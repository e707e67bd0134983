// Cluster tree and block partition of Sec. II-A, built on the host.
//
// The tree is a KD bisection: tight axis-aligned boxes, split on the widest
// extent (lowest axis on ties), points ordered by (coordinate, original index),
// left child gets floor(n/2).  All leaves sit at depth D, the smallest d with
// ceil(n / 2^d) <= leaf_size.  Nodes use heap numbering (children of i are
// 2i+1, 2i+2); a node owns the contiguous slice [begin, end) of `perm`.
//
// The block partition comes from the dual-tree traversal of same-depth
// cluster pairs starting at (root, root): an admissible pair is a far block
// (F_tau), an inadmissible pair at the leaf depth a dense block (N_tau),
// otherwise the four child pairs are visited.  It is run breadth first, one
// depth at a time and one cluster row at a time, on up to 16 host threads.
// Lists are stored per depth as CSR over local node indices, each row
// ascending.
#pragma once

#include <cstdint>
#include <vector>

namespace h2 {

struct Plan {
  int64_t n = 0;
  int dim = 0;
  int leaf_size = 0;
  double eta = 0;
  int depth = 0;                       // D
  std::vector<int32_t> perm;           // tree position -> original index
  std::vector<int32_t> begin, end;     // per heap node
  std::vector<double> lo, hi;          // per heap node, dim entries each (tight box)
  std::vector<int32_t> near_ptr, near_idx;              // leaf depth
  std::vector<std::vector<int32_t>> far_ptr, far_idx;   // per depth 0..D

  int num_nodes() const { return (2 << depth) - 1; }
  int level_begin(int t) const { return (1 << t) - 1; }
};

// Depth D for n points and the given leaf size.
int tree_depth(int64_t n, int leaf_size);

// General admissibility condition (Sec. II-A) without square roots:
// adm <=> gap^2 > 0 and q >= 0 and 4 a_s a_t <= q^2, q = 4 eta^2 gap^2 - a_s - a_t,
// where a_* are the squared box diagonals.  Every operation is rounded on its own.
bool admissible(const double* lo_s, const double* hi_s, const double* lo_t, const double* hi_t, int dim,
                double eta);

// Builds tree and lists.  points: host (dim x n) SoA.  Throws std::invalid_argument.
Plan make_plan(int64_t n, int dim, const double* points, int leaf_size, double eta);

}  // namespace h2
