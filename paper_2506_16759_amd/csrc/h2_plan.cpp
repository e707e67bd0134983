// Host cluster tree and block partition (Sec. II-A).  Compiled with
// floating-point contraction disabled so that the box and admissibility
// arithmetic is reproducible operation by operation.
#include "h2_plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <atomic>
#include <thread>
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

// Runs f(i) for i in [0, n) on up to 16 host threads (the GPU machine's CPU share).
template <typename F>
void parallel_for(int n, F&& f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = static_cast<int>(std::min<unsigned>(std::min(hw, 16u), static_cast<unsigned>((n + 63) / 64)));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  std::atomic<int> next{0};
  for (int w = 0; w < nt; ++w)
    pool.emplace_back([&] {
      for (;;) {
        const int i0 = next.fetch_add(32);
        if (i0 >= n) break;
        for (int i = i0; i < std::min(n, i0 + 32); ++i) f(i);
      }
    });
  for (auto& t : pool) t.join();
}

void tight_box(const Plan& p, const double* points, int node, double* lo, double* hi) {
  const int b = p.begin[node], e = p.end[node];
  for (int a = 0; a < p.dim; ++a) {
    const double* x = points + static_cast<size_t>(a) * p.n;
    double mn = x[p.perm[b]], mx = mn;
    for (int q = b + 1; q < e; ++q) {
      const double v = x[p.perm[q]];
      if (v < mn) mn = v;
      if (v > mx) mx = v;
    }
    lo[a] = mn;
    hi[a] = mx;
  }
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
  const int D = p.depth;
  const int nn = p.num_nodes();
  p.perm.resize(n);
  std::iota(p.perm.begin(), p.perm.end(), 0);
  p.begin.assign(nn, 0);
  p.end.assign(nn, 0);
  p.lo.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.hi.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.end[0] = static_cast<int32_t>(n);

  // Tree, one depth at a time.  Above the last split only the membership of
  // each half matters (the children reorder their own points), so a partial
  // partition suffices; the last split sorts fully, which fixes the order of
  // the points inside every leaf.
  for (int t = 0; t <= D; ++t) {
    const int base = p.level_begin(t);
    parallel_for(1 << t, [&](int i) {
      const int node = base + i;
      double* lo = &p.lo[static_cast<size_t>(node) * dim];
      double* hi = &p.hi[static_cast<size_t>(node) * dim];
      tight_box(p, points, node, lo, hi);
      if (t == D) return;
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
      auto less = [x](int32_t a, int32_t b) { return x[a] < x[b] || (x[a] == x[b] && a < b); };
      const int b = p.begin[node], e = p.end[node];
      const int mid = b + (e - b) / 2;
      if (t == D - 1) {
        std::sort(p.perm.begin() + b, p.perm.begin() + e, less);
      } else if (mid > b && mid < e) {
        std::nth_element(p.perm.begin() + b, p.perm.begin() + mid, p.perm.begin() + e, less);
      }
      p.begin[2 * node + 1] = b;
      p.end[2 * node + 1] = mid;
      p.begin[2 * node + 2] = mid;
      p.end[2 * node + 2] = e;
    });
  }

  // Dual-tree traversal, breadth first: the candidate partners of s at depth
  // t are the children of the clusters that were inadmissible with s's
  // parent at depth t-1.  Those lists are ascending, so every list below
  // comes out ascending without a sort.
  std::vector<std::vector<int32_t>> inadm(1);
  p.far_ptr.assign(D + 1, {});
  p.far_idx.assign(D + 1, {});
  auto flatten = [](const std::vector<std::vector<int32_t>>& rows, std::vector<int32_t>& ptr,
                    std::vector<int32_t>& idx) {
    ptr.assign(rows.size() + 1, 0);
    for (size_t r = 0; r < rows.size(); ++r) ptr[r + 1] = ptr[r] + static_cast<int32_t>(rows[r].size());
    idx.resize(ptr.back());
    for (size_t r = 0; r < rows.size(); ++r) std::copy(rows[r].begin(), rows[r].end(), idx.begin() + ptr[r]);
  };
  for (int t = 0; t <= D; ++t) {
    const int cnt = 1 << t, base = p.level_begin(t);
    std::vector<std::vector<int32_t>> far(cnt), keep(cnt);
    parallel_for(cnt, [&](int i) {
      const int s = base + i;
      auto test = [&](int c) {  // c: local index at depth t
        const int tn = base + c;
        if (admissible(&p.lo[size_t(s) * dim], &p.hi[size_t(s) * dim], &p.lo[size_t(tn) * dim],
                       &p.hi[size_t(tn) * dim], dim, eta))
          far[i].push_back(c);
        else
          keep[i].push_back(c);
      };
      if (t == 0) {
        test(0);
      } else {
        for (int32_t q : inadm[i >> 1]) {
          test(2 * q);
          test(2 * q + 1);
        }
      }
    });
    flatten(far, p.far_ptr[t], p.far_idx[t]);
    if (t == D) {
      flatten(keep, p.near_ptr, p.near_idx);
    } else {
      inadm.swap(keep);
    }
  }
  return p;
}

}  // namespace h2
