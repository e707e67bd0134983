// Host cluster tree and block partition (Sec. II-A).  Compiled with
// floating-point contraction disabled so that the box and admissibility
// arithmetic is reproducible operation by operation.
#include "h2_plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <utility>

#pragma clang fp contract(off)

namespace h2 {

int tree_depth(int64_t n, int leaf_size) {
  int d = 0;
  // ceil(n / 2^d) > leaf_size  <=>  n > leaf_size * 2^d
  while (d < 30 && n > static_cast<int64_t>(leaf_size) * (int64_t{1} << d)) ++d;
  return d;
}

bool admissible(const double* lo_s, const double* hi_s, const double* lo_t, const double* hi_t, int dim,
                double eta) {
  double as = 0.0, at = 0.0, gap2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double es = hi_s[a] - lo_s[a];
    as = as + es * es;
    const double et = hi_t[a] - lo_t[a];
    at = at + et * et;
    const double g = std::max(std::max(0.0, lo_t[a] - hi_s[a]), lo_s[a] - hi_t[a]);
    gap2 = gap2 + g * g;
  }
  if (!(gap2 > 0.0)) return false;
  const double four_eta2 = 4.0 * (eta * eta);
  const double q = (four_eta2 * gap2 - as) - at;
  if (!(q >= 0.0)) return false;
  return (4.0 * as) * at <= q * q;
}

namespace {

struct Traversal {
  const Plan& p;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> far;  // per depth (s_local, t_local)
  std::vector<std::pair<int32_t, int32_t>> near;

  explicit Traversal(const Plan& plan) : p(plan), far(plan.depth + 1) {}

  void visit(int s, int t, int depth) {
    const int dim = p.dim;
    const int base = p.level_begin(depth);
    if (admissible(&p.lo[s * dim], &p.hi[s * dim], &p.lo[t * dim], &p.hi[t * dim], dim, p.eta)) {
      far[depth].emplace_back(s - base, t - base);
    } else if (depth == p.depth) {
      near.emplace_back(s - base, t - base);
    } else {
      for (int i = 2 * s + 1; i <= 2 * s + 2; ++i)
        for (int j = 2 * t + 1; j <= 2 * t + 2; ++j) visit(i, j, depth + 1);
    }
  }
};

void to_csr(std::vector<std::pair<int32_t, int32_t>>& pairs, int rows, std::vector<int32_t>& ptr,
            std::vector<int32_t>& idx) {
  std::sort(pairs.begin(), pairs.end());
  ptr.assign(rows + 1, 0);
  idx.resize(pairs.size());
  for (size_t k = 0; k < pairs.size(); ++k) {
    ptr[pairs[k].first + 1]++;
    idx[k] = pairs[k].second;
  }
  for (int r = 0; r < rows; ++r) ptr[r + 1] += ptr[r];
}

}  // namespace

Plan make_plan(int64_t n, int dim, const double* points, int leaf_size, double eta) {
  if (n < 1 || n > (int64_t{1} << 30)) throw std::invalid_argument("n must be in [1, 2^30]");
  if (dim < 1 || dim > 3) throw std::invalid_argument("dim must be 1, 2 or 3");
  if (leaf_size < 2 || leaf_size > 256) throw std::invalid_argument("leaf_size must be in [2, 256]");
  if (!(eta > 0.0) || !std::isfinite(eta)) throw std::invalid_argument("eta must be finite and > 0");
  if (!points) throw std::invalid_argument("points is NULL");
  for (int64_t k = 0; k < n * dim; ++k)
    if (!std::isfinite(points[k])) throw std::invalid_argument("points must be finite");

  Plan p;
  p.n = n;
  p.dim = dim;
  p.leaf_size = leaf_size;
  p.eta = eta;
  p.depth = tree_depth(n, leaf_size);
  const int nn = p.num_nodes();
  p.perm.resize(n);
  std::iota(p.perm.begin(), p.perm.end(), 0);
  p.begin.assign(nn, 0);
  p.end.assign(nn, 0);
  p.lo.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.hi.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.begin[0] = 0;
  p.end[0] = static_cast<int32_t>(n);

  for (int node = 0; node < nn; ++node) {
    const int b = p.begin[node], e = p.end[node];
    double* lo = &p.lo[static_cast<size_t>(node) * dim];
    double* hi = &p.hi[static_cast<size_t>(node) * dim];
    for (int a = 0; a < dim; ++a) {
      const double* x = points + static_cast<size_t>(a) * n;
      double mn = x[p.perm[b]], mx = mn;
      for (int q = b + 1; q < e; ++q) {
        const double v = x[p.perm[q]];
        if (v < mn) mn = v;
        if (v > mx) mx = v;
      }
      lo[a] = mn;
      hi[a] = mx;
    }
    if (2 * node + 2 < nn) {
      int axis = 0;
      double widest = hi[0] - lo[0];
      for (int a = 1; a < dim; ++a) {
        const double ext = hi[a] - lo[a];
        if (ext > widest) {
          widest = ext;
          axis = a;
        }
      }
      const double* x = points + static_cast<size_t>(axis) * n;
      std::sort(p.perm.begin() + b, p.perm.begin() + e, [x](int32_t i, int32_t j) {
        return x[i] < x[j] || (x[i] == x[j] && i < j);
      });
      const int mid = b + (e - b) / 2;
      p.begin[2 * node + 1] = b;
      p.end[2 * node + 1] = mid;
      p.begin[2 * node + 2] = mid;
      p.end[2 * node + 2] = e;
    }
  }

  Traversal tr(p);
  tr.visit(0, 0, 0);
  p.far_ptr.resize(p.depth + 1);
  p.far_idx.resize(p.depth + 1);
  for (int t = 0; t <= p.depth; ++t) to_csr(tr.far[t], 1 << t, p.far_ptr[t], p.far_idx[t]);
  to_csr(tr.near, 1 << p.depth, p.near_ptr, p.near_idx);
  return p;
}

}  // namespace h2
