// Host cluster tree and block partition (Sec. II-A).  Compiled with
// floating-point contraction disabled so that the box and admissibility
// arithmetic is reproducible operation by operation.
#include "h2_plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <utility>

#include "h2_pool.hpp"

#pragma clang fp contract(off)

namespace h2 {

int tree_depth(int64_t n, int leaf_size) {
  int d = 0;
  // ceil(n / 2^d) > leaf_size  <=>  n > leaf_size * 2^d
  while (d < 30 && n > static_cast<int64_t>(leaf_size) * (int64_t{1} << d)) ++d;
  return d;
}

namespace {

// Squared diagonal of a box, summed over the axes in order.
inline double sq_diag(const double* lo, const double* hi, int dim) {
  double d2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double e = hi[a] - lo[a];
    d2 = d2 + e * e;
  }
  return d2;
}

// The admissibility test given both squared diagonals.  All three conditions
// are evaluated without branches: along a candidate list the outcome is
// close to random.
template <int DIM>
inline int adm_pair(const double* lo_s, const double* hi_s, double as, const double* lo_t, const double* hi_t,
                    double at, double four_eta2) {
  double gap2 = 0.0;
  for (int a = 0; a < DIM; ++a) {
    const double g = std::max(std::max(0.0, lo_t[a] - hi_s[a]), lo_s[a] - hi_t[a]);
    gap2 = gap2 + g * g;
  }
  const double q = (four_eta2 * gap2 - as) - at;
  return (gap2 > 0.0) & (q >= 0.0) & ((4.0 * as) * at <= q * q);
}

}  // namespace

bool admissible(const double* lo_s, const double* hi_s, const double* lo_t, const double* hi_t, int dim,
                double eta) {
  const double as = sq_diag(lo_s, hi_s, dim), at = sq_diag(lo_t, hi_t, dim);
  const double four_eta2 = 4.0 * (eta * eta);
  switch (dim) {
    case 1: return adm_pair<1>(lo_s, hi_s, as, lo_t, hi_t, at, four_eta2);
    case 2: return adm_pair<2>(lo_s, hi_s, as, lo_t, hi_t, at, four_eta2);
    default: return adm_pair<3>(lo_s, hi_s, as, lo_t, hi_t, at, four_eta2);
  }
}

namespace {

// A point with its original index: the tree sorts these records, so every
// comparison and box scan reads contiguous memory.
struct TreePoint {
  double c[3];
  int32_t id;
};

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
  p.begin.assign(nn, 0);
  p.end.assign(nn, 0);
  p.lo.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.hi.assign(static_cast<size_t>(nn) * dim, 0.0);
  p.end[0] = static_cast<int32_t>(n);
  std::vector<TreePoint> pt(static_cast<size_t>(n));
  parallel_for(static_cast<int>((n + 4095) / 4096), 1, [&](int c) {
    const int64_t r1 = std::min<int64_t>(n, int64_t(c + 1) * 4096);
    for (int64_t r = int64_t(c) * 4096; r < r1; ++r) {
      for (int a = 0; a < 3; ++a) pt[r].c[a] = a < dim ? points[static_cast<size_t>(a) * n + r] : 0.0;
      pt[r].id = static_cast<int32_t>(r);
    }
  });

  // Tree, one depth at a time, nodes of a depth in parallel.  Points are
  // ordered by (coordinate on the split axis, original index), a strict total
  // order, so the membership of each half is unique whatever the selection
  // algorithm.  Above the last split only that membership matters (the
  // children reorder their own points), so a partial partition suffices; the
  // last split sorts fully, which fixes the order of the points inside every
  // leaf.
  for (int t = 0; t <= D; ++t) {
    const int base = p.level_begin(t);
    parallel_for(1 << t, 1, [&](int i) {
      const int node = base + i;
      double* lo = &p.lo[static_cast<size_t>(node) * dim];
      double* hi = &p.hi[static_cast<size_t>(node) * dim];
      const int b = p.begin[node], e = p.end[node];
      for (int a = 0; a < dim; ++a) lo[a] = hi[a] = pt[b].c[a];
      for (int q = b + 1; q < e; ++q)
        for (int a = 0; a < dim; ++a) {
          const double v = pt[q].c[a];
          if (v < lo[a]) lo[a] = v;
          if (v > hi[a]) hi[a] = v;
        }
      // a signed zero becomes +0 (-0 and +0 compare equal; which one is the
      // first extreme depends on the point order inside the node)
      for (int a = 0; a < dim; ++a) {
        lo[a] = lo[a] + 0.0;
        hi[a] = hi[a] + 0.0;
      }
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
      auto less = [axis](const TreePoint& u, const TreePoint& v) {
        return u.c[axis] < v.c[axis] || (u.c[axis] == v.c[axis] && u.id < v.id);
      };
      const int mid = b + (e - b) / 2;
      if (t == D - 1) {
        std::sort(pt.begin() + b, pt.begin() + e, less);
      } else if (mid > b && mid < e) {
        std::nth_element(pt.begin() + b, pt.begin() + mid, pt.begin() + e, less);
      }
      p.begin[2 * node + 1] = b;
      p.end[2 * node + 1] = mid;
      p.begin[2 * node + 2] = mid;
      p.end[2 * node + 2] = e;
    });
  }
  p.perm.resize(n);
  for (int64_t r = 0; r < n; ++r) p.perm[r] = pt[r].id;

  // Dual-tree traversal, breadth first: the candidate partners of s at depth
  // t are the children of the clusters that were inadmissible with s's
  // parent at depth t-1.  Those lists are ascending, so every list below
  // comes out ascending without a sort.  Each row writes its results into a
  // preallocated slice as long as its candidate list, and the slices are then
  // compacted into CSR, so the parallel part allocates nothing.
  std::vector<int32_t> iptr{0, 0}, iidx;  // inadmissible partners at depth t-1 (CSR)
  p.far_ptr.assign(D + 1, {});
  p.far_idx.assign(D + 1, {});
  std::vector<int32_t> cptr, cfar, cnear, nfar, nnear;
  const double four_eta2 = 4.0 * (eta * eta);
  std::vector<double> diag2(nn);
  parallel_for(nn, 256, [&](int v) { diag2[v] = sq_diag(&p.lo[size_t(v) * dim], &p.hi[size_t(v) * dim], dim); });
  auto compact = [](const std::vector<int32_t>& cptr, const std::vector<int32_t>& buf,
                    const std::vector<int32_t>& cnt, std::vector<int32_t>& ptr, std::vector<int32_t>& idx) {
    const int rows = static_cast<int>(cnt.size());
    ptr.assign(rows + 1, 0);
    for (int r = 0; r < rows; ++r) ptr[r + 1] = ptr[r] + cnt[r];
    idx.resize(ptr.back());
    parallel_for(rows, 64, [&](int r) {
      std::copy(buf.begin() + cptr[r], buf.begin() + cptr[r] + cnt[r], idx.begin() + ptr[r]);
    });
  };
  for (int t = 0; t <= D; ++t) {
    const int cnt = 1 << t, base = p.level_begin(t);
    cptr.assign(cnt + 1, 0);
    for (int i = 0; i < cnt; ++i) cptr[i + 1] = cptr[i] + (t == 0 ? 1 : 2 * (iptr[(i >> 1) + 1] - iptr[i >> 1]));
    cfar.resize(cptr[cnt]);
    cnear.resize(cptr[cnt]);
    nfar.assign(cnt, 0);
    nnear.assign(cnt, 0);
    auto rows = [&](auto dimc) {
      constexpr int DIM = decltype(dimc)::value;
      parallel_for(cnt, 16, [&](int i) {
        const int s = base + i;
        const double* lo_s = &p.lo[size_t(s) * DIM];
        const double* hi_s = &p.hi[size_t(s) * DIM];
        int32_t* fo = cfar.data() + cptr[i];
        int32_t* ko = cnear.data() + cptr[i];
        int nf = 0, nk = 0;
        auto test = [&](int c) {  // c: local index at depth t
          const int tn = base + c;
          const int adm = adm_pair<DIM>(lo_s, hi_s, diag2[s], &p.lo[size_t(tn) * DIM], &p.hi[size_t(tn) * DIM],
                                        diag2[tn], four_eta2);
          fo[nf] = c;
          ko[nk] = c;
          nf += adm;
          nk += 1 - adm;
        };
        if (t == 0) {
          test(0);
        } else {
          for (int j = iptr[i >> 1]; j < iptr[(i >> 1) + 1]; ++j) {
            test(2 * iidx[j]);
            test(2 * iidx[j] + 1);
          }
        }
        nfar[i] = nf;
        nnear[i] = nk;
      });
    };
    if (dim == 1) rows(std::integral_constant<int, 1>{});
    else if (dim == 2) rows(std::integral_constant<int, 2>{});
    else rows(std::integral_constant<int, 3>{});
    compact(cptr, cfar, nfar, p.far_ptr[t], p.far_idx[t]);
    if (t == D) {
      compact(cptr, cnear, nnear, p.near_ptr, p.near_idx);
    } else {
      compact(cptr, cnear, nnear, iptr, iidx);
    }
  }
  return p;
}

}  // namespace h2
