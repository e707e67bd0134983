// Cluster tree and block partition of Sec. II-A built on the device.
//
// Same definitions as the host planner (h2_plan.cpp), so the result is the
// same plan bit for bit: tight boxes (first occurrence of the extreme value in
// the node's point order, signed zeros made +0), the widest axis with the
// lowest axis on ties, points ordered by (coordinate on that axis, original
// index) and floor(m/2) of them to the left child; then the breadth-first
// dual-tree traversal with the square-root-free admissibility test evaluated
// operation by operation (contraction off).
//
// Tree: one kernel per depth, one workgroup per node.  Above the last split
// only the membership of each half matters (the children reorder their own
// points), so the node finds its left half's size-th element by radix
// selection on (order key of the coordinate, original index) and partitions
// around it, keeping the order inside each half; the last split (nodes of at
// most 2 x leaf_size <= 512 points) sorts its node in LDS, which fixes the
// order inside every leaf.  Traversal: per depth, the candidate partners of a
// cluster are the children of the clusters that were inadmissible with its
// parent, ascending; one workgroup per cluster tests them and compacts the
// admissible and the inadmissible ones in candidate order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <vector>

#include "h2_device.hpp"
#include "h2_internal.hpp"
#include "h2_plan.hpp"

#pragma clang fp contract(off)

namespace h2 {
namespace {

using h2i::DevArray;

constexpr int kPlanThreads = 256;
constexpr int kSortSlots = 512;  // 2 x the largest leaf size

// Unsigned key in the order of the coordinate values; -0.0 and +0.0 share a
// key (the tree compares coordinates with <, ties broken by original index).
__device__ __forceinline__ uint64_t order_key(double x) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x + 0.0));
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ bool key_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Inclusive prefix sum over the 256 threads of the workgroup (in thread order).
__device__ int block_inclusive_scan(int v, int* sh /* kPlanThreads / 64 ints */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wave; ++w) add += sh[w];
  __syncthreads();
  return v + add;
}

// Wave-0 search of the histogram bin holding rank k: writes the bin, the
// count below it and its count.
__device__ void find_bin(const uint32_t* hist, uint32_t k, uint32_t* out /* 3 */) {
  if ((threadIdx.x >> 6) != 0) return;
  const int lane = threadIdx.x & 63;
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c[j] = hist[lane * 4 + j];
    sum += c[j];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  const uint32_t excl = incl - sum;
  if (k >= excl && k < incl) {
    uint32_t acc = excl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (k < acc + c[j]) {
        out[0] = lane * 4 + j;
        out[1] = acc;
        out[2] = c[j];
        break;
      }
      acc += c[j];
    }
  }
}

// One depth of the tree.  Xc/idc: points of every node in the current order
// (SoA with leading dimension n); the node's points go to Xn/idn in the
// children's order.  Writes the node's box and squared diagonal.
template <int DIM>
__global__ __launch_bounds__(kPlanThreads) void tree_level_kernel(
    int t, int D, int base, const int32_t* __restrict__ begin, const int32_t* __restrict__ end, int64_t n,
    const double* __restrict__ Xc, const int32_t* __restrict__ idc, double* __restrict__ Xn,
    int32_t* __restrict__ idn, double* __restrict__ lo, double* __restrict__ hi, double* __restrict__ diag2,
    int32_t* __restrict__ err) {
  __shared__ double s_lo[4][DIM], s_hi[4][DIM];
  __shared__ int s_axis;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_bin[3];
  __shared__ uint64_t s_pkey;
  __shared__ int32_t s_pid;
  __shared__ int s_scan[kPlanThreads / 64];
  __shared__ uint64_t skey[kSortSlots];
  __shared__ int32_t sid[kSortSlots];
  __shared__ int32_t spos[kSortSlots];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int node = base + blockIdx.x;
  const int b = begin[node], e = end[node], m = e - b;
  const int chunk = (m + kPlanThreads - 1) / kPlanThreads;
  const int q0 = min(e, b + tid * chunk), q1 = min(e, q0 + chunk);

  // tight box: the first occurrence of each extreme value, in point order
  double l[DIM], h[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    l[a] = __builtin_huge_val();
    h[a] = -__builtin_huge_val();
  }
  for (int q = q0; q < q1; ++q)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double v = Xc[a * n + q];
      if (v < l[a]) l[a] = v;
      if (v > h[a]) h[a] = v;
    }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double ol = __shfl_down(l[a], off), oh = __shfl_down(h[a], off);
      if (lane + off < 64) {
        if (ol < l[a]) l[a] = ol;
        if (oh > h[a]) h[a] = oh;
      }
    }
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      s_lo[wave][a] = l[a];
      s_hi[wave][a] = h[a];
    }
  __syncthreads();
  if (tid == 0) {
    double L[DIM], H[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      L[a] = s_lo[0][a];
      H[a] = s_hi[0][a];
      for (int w = 1; w < kPlanThreads / 64; ++w) {
        if (s_lo[w][a] < L[a]) L[a] = s_lo[w][a];
        if (s_hi[w][a] > H[a]) H[a] = s_hi[w][a];
      }
      L[a] = L[a] + 0.0;
      H[a] = H[a] + 0.0;
      lo[int64_t(node) * DIM + a] = L[a];
      hi[int64_t(node) * DIM + a] = H[a];
    }
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double ext = H[a] - L[a];
      d2 = d2 + ext * ext;
    }
    diag2[node] = d2;
    int axis = 0;
    double widest = H[0] - L[0];
#pragma unroll
    for (int a = 1; a < DIM; ++a) {
      const double ext = H[a] - L[a];
      if (ext > widest) {
        widest = ext;
        axis = a;
      }
    }
    s_axis = axis;
  }
  __syncthreads();
  if (t == D) return;
  const int axis = s_axis;
  const double* xa = Xc + axis * n;
  const int k = m / 2;  // the left child gets floor(m / 2) points
  const int mid = b + k;

  if (t == D - 1) {
    // last split: sort the node (m <= 2 x leaf_size) by (key, index) in LDS
    int P = 1;
    while (P < m) P <<= 1;
    for (int j = tid; j < P; j += kPlanThreads) {
      if (j < m) {
        skey[j] = order_key(xa[b + j]);
        sid[j] = idc[b + j];
        spos[j] = b + j;
      } else {
        skey[j] = ~0ull;  // larger than every finite coordinate's key
        sid[j] = 0x7fffffff;
        spos[j] = -1;
      }
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int j = tid; j < P; j += kPlanThreads) {
          const int pj = j ^ stride;
          if (pj > j) {
            const bool up = (j & size) == 0;
            const bool gt = key_less(skey[pj], sid[pj], skey[j], sid[j]);
            if (gt == up) {
              const uint64_t tk = skey[j];
              skey[j] = skey[pj];
              skey[pj] = tk;
              const int32_t ti = sid[j];
              sid[j] = sid[pj];
              sid[pj] = ti;
              const int32_t tp = spos[j];
              spos[j] = spos[pj];
              spos[pj] = tp;
            }
          }
        }
        __syncthreads();
      }
    for (int j = tid; j < m; j += kPlanThreads) {
      const int src = spos[j];
#pragma unroll
      for (int a = 0; a < DIM; ++a) Xn[a * n + b + j] = Xc[a * n + src];
      idn[b + j] = idc[src];
    }
    return;
  }

  if (m < 2) {  // nothing to split (not reached for tree depths from tree_depth)
    for (int q = b + tid; q < e; q += kPlanThreads) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) Xn[a * n + q] = Xc[a * n + q];
      idn[q] = idc[q];
    }
    return;
  }

  // radix selection of the element of rank k by (key, index), 8 bits at a time
  uint64_t prefix = 0, mask = 0;
  uint32_t kr = static_cast<uint32_t>(k), cnt = static_cast<uint32_t>(m);
  for (int shift = 56; shift >= 0 && cnt > 1; shift -= 8) {
    for (int j = tid; j < 256; j += kPlanThreads) hist[j] = 0;
    __syncthreads();
    int run_d = -1;
    uint32_t run_c = 0;
    for (int q = q0; q < q1; ++q) {
      const uint64_t K = order_key(xa[q]);
      if ((K & mask) != prefix) continue;
      const int d = static_cast<int>((K >> shift) & 0xff);
      if (d == run_d) {
        ++run_c;
      } else {
        if (run_c) atomicAdd(&hist[run_d], run_c);
        run_d = d;
        run_c = 1;
      }
    }
    if (run_c) atomicAdd(&hist[run_d], run_c);
    __syncthreads();
    find_bin(hist, kr, s_bin);
    __syncthreads();
    prefix |= uint64_t(s_bin[0]) << shift;
    mask |= uint64_t(0xff) << shift;
    kr -= s_bin[1];
    cnt = s_bin[2];
    __syncthreads();
  }
  if (cnt == 1) {
    // one element carries the selected key bits: it is the pivot
    for (int q = q0; q < q1; ++q) {
      const uint64_t K = order_key(xa[q]);
      if ((K & mask) == prefix) {
        s_pkey = K;
        s_pid = idc[q];
      }
    }
  } else {
    // equal coordinates: select among them by original index
    uint32_t iprefix = 0, imask = 0;
    for (int shift = 24; shift >= 0 && cnt > 1; shift -= 8) {
      for (int j = tid; j < 256; j += kPlanThreads) hist[j] = 0;
      __syncthreads();
      for (int q = q0; q < q1; ++q) {
        if (order_key(xa[q]) != prefix) continue;
        const uint32_t id = static_cast<uint32_t>(idc[q]);
        if ((id & imask) == iprefix) atomicAdd(&hist[(id >> shift) & 0xff], 1u);
      }
      __syncthreads();
      find_bin(hist, kr, s_bin);
      __syncthreads();
      iprefix |= s_bin[0] << shift;
      imask |= 0xffu << shift;
      kr -= s_bin[1];
      cnt = s_bin[2];
      __syncthreads();
    }
    for (int q = q0; q < q1; ++q) {
      const uint32_t id = static_cast<uint32_t>(idc[q]);
      if (order_key(xa[q]) == prefix && (id & imask) == iprefix) {
        s_pkey = prefix;
        s_pid = static_cast<int32_t>(id);
      }
    }
  }
  __syncthreads();
  const uint64_t pkey = s_pkey;
  const int32_t pid = s_pid;

  // partition around the pivot, keeping the order inside each half
  int nl = 0;
  for (int q = q0; q < q1; ++q) nl += key_less(order_key(xa[q]), idc[q], pkey, pid) ? 1 : 0;
  const int incl = block_inclusive_scan(nl, s_scan);
  int total_left = 0;
  for (int w = 0; w < kPlanThreads / 64; ++w) total_left += s_scan[w];
  if (total_left != k) {  // the selection must leave exactly k points below the pivot
    if (tid == 0) atomicOr(err, 1);
    return;
  }
  int wl = b + (incl - nl);
  int wr = mid + ((q0 - b) - (incl - nl));
  for (int q = q0; q < q1; ++q) {
    const int32_t id = idc[q];
    const int dst = key_less(order_key(xa[q]), id, pkey, pid) ? wl++ : wr++;
#pragma unroll
    for (int a = 0; a < DIM; ++a) Xn[a * n + dst] = Xc[a * n + q];
    idn[dst] = id;
  }
}

// counts[i] = candidate partners of cluster i at depth t >= 1: both children
// of every cluster inadmissible with its parent.
__global__ __launch_bounds__(256) void candidate_count_kernel(int rows, const int32_t* __restrict__ iptr,
                                                              int32_t* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) counts[i] = 2 * (iptr[(i >> 1) + 1] - iptr[i >> 1]);
}

// The admissibility test of the host planner, operation by operation.
template <int DIM>
__device__ __forceinline__ int adm_pair(const double* ls, const double* hs, double as, const double* lt,
                                        const double* ht, double at, double four_eta2) {
  double gap2 = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double u = lt[a] - hs[a], v = ls[a] - ht[a];
    const double g0 = 0.0 < u ? u : 0.0;  // std::max(0.0, u)
    const double g = g0 < v ? v : g0;      // std::max(g0, v)
    gap2 = gap2 + g * g;
  }
  const double q = (four_eta2 * gap2 - as) - at;
  return (gap2 > 0.0) & (q >= 0.0) & ((4.0 * as) * at <= q * q);
}

// One workgroup per cluster s of depth t: tests its candidates in order and
// writes the admissible ones to cfar and the others to cnear (both at
// cptr[i]), with their counts.
template <int DIM>
__global__ __launch_bounds__(kPlanThreads) void traverse_level_kernel(
    int t, int base, const int32_t* __restrict__ iptr, const int32_t* __restrict__ iidx,
    const int32_t* __restrict__ cptr, const double* __restrict__ lo, const double* __restrict__ hi,
    const double* __restrict__ diag2, double four_eta2, int32_t* __restrict__ cfar, int32_t* __restrict__ cnear,
    int32_t* __restrict__ nfar, int32_t* __restrict__ nnear) {
  __shared__ int wf[kPlanThreads / 64], wn[kPlanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = blockIdx.x, s = base + i;
  const int c_begin = cptr[i], cnt = cptr[i + 1] - c_begin;
  const int j0 = t == 0 ? 0 : iptr[i >> 1];
  double ls[DIM], hs[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    ls[a] = lo[int64_t(s) * DIM + a];
    hs[a] = hi[int64_t(s) * DIM + a];
  }
  const double as = diag2[s];
  const uint64_t below = (uint64_t(1) << lane) - 1;
  int of = 0, on = 0;
  for (int c0 = 0; c0 < cnt; c0 += kPlanThreads) {
    const int j = c0 + tid;
    int adm = 0, inadm = 0, c = 0;
    if (j < cnt) {
      c = t == 0 ? 0 : 2 * iidx[j0 + (j >> 1)] + (j & 1);
      const int tn = base + c;
      double lt[DIM], ht[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        lt[a] = lo[int64_t(tn) * DIM + a];
        ht[a] = hi[int64_t(tn) * DIM + a];
      }
      adm = adm_pair<DIM>(ls, hs, as, lt, ht, diag2[tn], four_eta2);
      inadm = 1 - adm;
    }
    const uint64_t bf = __ballot(adm), bn = __ballot(inadm);
    if (lane == 0) {
      wf[wave] = __popcll(bf);
      wn[wave] = __popcll(bn);
    }
    __syncthreads();
    int bfw = of, bnw = on, tf = 0, tn_ = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) {
      if (w < wave) {
        bfw += wf[w];
        bnw += wn[w];
      }
      tf += wf[w];
      tn_ += wn[w];
    }
    if (adm) cfar[c_begin + bfw + __popcll(bf & below)] = c;
    if (inadm) cnear[c_begin + bnw + __popcll(bn & below)] = c;
    of += tf;
    on += tn_;
    __syncthreads();
  }
  if (tid == 0) {
    nfar[i] = of;
    nnear[i] = on;
  }
}

// dst[ptr[i] + r] = src[cptr[i] + r] for r < ptr[i + 1] - ptr[i]; one workgroup per row.
__global__ __launch_bounds__(256) void compact_rows_kernel(const int32_t* __restrict__ cptr,
                                                           const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ src,
                                                           int32_t* __restrict__ dst) {
  const int i = blockIdx.x;
  const int c = cptr[i], p = ptr[i], len = ptr[i + 1] - p;
  for (int r = threadIdx.x; r < len; r += blockDim.x) dst[p + r] = src[c + r];
}

// Copies the caller's (dim x n) points into the first buffer with zero for the
// unused coordinates, numbers them, and flags any non-finite coordinate.
__global__ __launch_bounds__(256) void load_points_kernel(int64_t n, int dim, const double* __restrict__ P,
                                                          double* __restrict__ X, int32_t* __restrict__ id,
                                                          int32_t* __restrict__ bad) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  int nonfinite = 0;
  for (int a = 0; a < dim; ++a) {
    const double v = P[a * n + q];
    nonfinite |= !isfinite(v);
    X[a * n + q] = v;
  }
  id[q] = static_cast<int32_t>(q);
  if (nonfinite) atomicOr(bad, 1);
}

template <typename T>
std::vector<T> fetch(const T* d, size_t count, hipStream_t s) {
  std::vector<T> h(count);
  if (count) {
    H2_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
  }
  return h;
}

}  // namespace

Plan make_plan_device(hipStream_t s, int64_t n, int dim, const double* points, int leaf_size, double eta) {
  if (n < 1 || n > (int64_t{1} << 30)) throw std::invalid_argument("n must be in [1, 2^30]");
  if (dim < 1 || dim > 3) throw std::invalid_argument("dim must be 1, 2 or 3");
  if (leaf_size < 2 || leaf_size > 256) throw std::invalid_argument("leaf_size must be in [2, 256]");
  if (!(eta > 0.0) || !std::isfinite(eta)) throw std::invalid_argument("eta must be finite and > 0");
  if (!points) throw std::invalid_argument("points is NULL");

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
  p.end[0] = static_cast<int32_t>(n);
  for (int t = 0; t < D; ++t)
    for (int v = p.level_begin(t); v < p.level_begin(t + 1); ++v) {
      const int b = p.begin[v], e = p.end[v], mid = b + (e - b) / 2;
      p.begin[2 * v + 1] = b;
      p.end[2 * v + 1] = mid;
      p.begin[2 * v + 2] = mid;
      p.end[2 * v + 2] = e;
    }

  DevArray<double> X[2], lo, hi, diag2;
  DevArray<int32_t> id[2], d_begin, d_end, bad;
  for (int k = 0; k < 2; ++k) {
    X[k].alloc(size_t(dim) * n, s);
    id[k].alloc(size_t(n), s);
  }
  lo.alloc(size_t(nn) * dim, s);
  hi.alloc(size_t(nn) * dim, s);
  diag2.alloc(size_t(nn), s);
  d_begin.upload(p.begin, s);
  d_end.upload(p.end, s);
  bad.upload(std::vector<int32_t>{0}, s);
  load_points_kernel<<<unsigned((n + 255) / 256), 256, 0, s>>>(n, dim, points, X[0].get(), id[0].get(), bad.get());
  H2_HIP(hipGetLastError());
  if (fetch(bad.get(), 1, s)[0]) throw std::invalid_argument("points must be finite");

  // the last split sorts a node of at most ceil(n / 2^(D-1)) <= 2 x leaf_size points in LDS
  if (D >= 1 && ((n + (int64_t{1} << (D - 1)) - 1) >> (D - 1)) > kSortSlots)
    throw std::invalid_argument("node of the last split exceeds the sort capacity");
  int cur = 0;
  for (int t = 0; t <= D; ++t) {
    const int nodes = 1 << t, base = p.level_begin(t);
#define H2_TREE(DD)                                                                                                \
  tree_level_kernel<DD><<<nodes, kPlanThreads, 0, s>>>(t, D, base, d_begin.get(), d_end.get(), n, X[cur].get(), \
                                                       id[cur].get(), X[1 - cur].get(), id[1 - cur].get(),    \
                                                       lo.get(), hi.get(), diag2.get(), bad.get())
    if (dim == 1) H2_TREE(1);
    else if (dim == 2) H2_TREE(2);
    else H2_TREE(3);
#undef H2_TREE
    H2_HIP(hipGetLastError());
    if (t < D) cur = 1 - cur;
  }

  if (fetch(bad.get(), 1, s)[0]) throw h2i::Error(H2_ERR_STATE, "device tree: a split did not select its median");

  // traversal, one depth at a time
  const double four_eta2 = 4.0 * (eta * eta);
  p.far_ptr.assign(D + 1, {});
  p.far_idx.assign(D + 1, {});
  std::vector<DevArray<int32_t>> fptr(D + 1), fidx(D + 1);
  DevArray<int32_t> iptr, iidx, nptr, nidx;
  for (int t = 0; t <= D; ++t) {
    const int rows = 1 << t, base = p.level_begin(t);
    DevArray<int32_t> cptr, counts;
    cptr.alloc(size_t(rows) + 1, s);
    if (t == 0) {
      cptr.upload(std::vector<int32_t>{0, 1}, s);
    } else {
      counts.alloc(size_t(rows), s);
      candidate_count_kernel<<<(rows + 255) / 256, 256, 0, s>>>(rows, iptr.get(), counts.get());
      H2_HIP(hipGetLastError());
      H2_HIP(h2dev::scan_i32(s, rows, counts.get(), cptr.get()));
    }
    const int32_t total = fetch(cptr.get() + rows, 1, s)[0];
    DevArray<int32_t> cfar, cnear, nfar, nnear;
    cfar.alloc(size_t(std::max(total, 1)), s);
    cnear.alloc(size_t(std::max(total, 1)), s);
    nfar.alloc(size_t(rows), s);
    nnear.alloc(size_t(rows), s);
#define H2_TRAV(DD)                                                                                                 \
  traverse_level_kernel<DD><<<rows, kPlanThreads, 0, s>>>(t, base, iptr.get(), iidx.get(), cptr.get(), lo.get(),  \
                                                          hi.get(), diag2.get(), four_eta2, cfar.get(),         \
                                                          cnear.get(), nfar.get(), nnear.get())
    if (dim == 1) H2_TRAV(1);
    else if (dim == 2) H2_TRAV(2);
    else H2_TRAV(3);
#undef H2_TRAV
    H2_HIP(hipGetLastError());
    fptr[t].alloc(size_t(rows) + 1, s);
    fidx[t].alloc(size_t(std::max(total, 1)), s);
    H2_HIP(h2dev::scan_i32(s, rows, nfar.get(), fptr[t].get()));
    compact_rows_kernel<<<rows, 256, 0, s>>>(cptr.get(), fptr[t].get(), cfar.get(), fidx[t].get());
    H2_HIP(hipGetLastError());
    nptr.alloc(size_t(rows) + 1, s);
    nidx.alloc(size_t(std::max(total, 1)), s);
    H2_HIP(h2dev::scan_i32(s, rows, nnear.get(), nptr.get()));
    compact_rows_kernel<<<rows, 256, 0, s>>>(cptr.get(), nptr.get(), cnear.get(), nidx.get());
    H2_HIP(hipGetLastError());
    iptr = std::move(nptr);
    iidx = std::move(nidx);
  }

  // results to the host plan
  p.perm = fetch(id[cur].get(), size_t(n), s);
  p.lo = fetch(lo.get(), size_t(nn) * dim, s);
  p.hi = fetch(hi.get(), size_t(nn) * dim, s);
  for (int t = 0; t <= D; ++t) {
    p.far_ptr[t] = fetch(fptr[t].get(), (size_t(1) << t) + 1, s);
    p.far_idx[t] = fetch(fidx[t].get(), size_t(p.far_ptr[t].back()), s);
  }
  p.near_ptr = fetch(iptr.get(), (size_t(1) << D) + 1, s);
  p.near_idx = fetch(iidx.get(), size_t(p.near_ptr.back()), s);
  return p;
}

}  // namespace h2
