// Entries of a built H^2 matrix (h2_entries): A_H(i, j) from the definition
// of the format (Sec. II-A, Table I, nested basis).  Entry (i, j) lies in
// exactly one block of the partition: the dense leaf block D_{s,b} when b is
// in N_s, else the admissible pair (s, b) of the ancestors of i's and j's
// leaves at the one depth where b is in F_s, where it equals
//   row_i(U_s) B_{s,b} row_j(V_b)^T,
// row_i(U_s) being the row of the nested basis U_s = diag(U_nu1, U_nu2)
// [E_nu1; E_nu2], expanded from the leaf basis through the transfer matrices.
//
// The first call expands those rows for every point and every processed
// depth (one pass per depth, leaves first); they stay with the matrix.  A
// block batch is then evaluated with one workgroup per block, one entry per
// thread: locate the block of the partition by binary searches in the
// ascending near/far lists, then one dot product of length k_s * k_b.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "h2_internal.hpp"

using namespace h2i;

namespace {

// Per processed depth: the far lists with their blocks, the rank offsets of
// both sides and the expanded basis rows (column-major, n rows).
struct EntryLevel {
  const int32_t* fptr;
  const int32_t* fidx;
  const int64_t* boff;
  const double* B;
  const int32_t* koff_r;
  const int32_t* koff_c;
  const double* R;  // R[a * n + p] = row p of the row-side nested basis at depth t, a < kmax
  const double* C;  // the same for the column side (== R for a symmetric matrix)
};

struct EntryCache {
  DevArray<int32_t> inv, leaf_of;
  std::vector<DevArray<double>> R, C;  // per depth
  DevArray<EntryLevel> levels;         // depth top..D, index t - top
  int top = 0;
};

__global__ __launch_bounds__(256) void inverse_perm_kernel(int64_t n, const int32_t* __restrict__ perm,
                                                           int32_t* __restrict__ inv) {
  const int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (p < n) inv[perm[p]] = static_cast<int32_t>(p);
}

__global__ __launch_bounds__(256) void leaf_of_kernel(const int32_t* __restrict__ leafoff,
                                                      int32_t* __restrict__ leaf_of) {
  const int l = blockIdx.x;
  for (int p = leafoff[l] + threadIdx.x; p < leafoff[l + 1]; p += blockDim.x) leaf_of[p] = l;
}

// Leaf depth: R[a * n + p] = U_leaf(p - leafoff[l], a) for a < k_l, 0 up to kmax.
__global__ __launch_bounds__(256) void basis_rows_leaf_kernel(int64_t n, int kmax, const int32_t* __restrict__ leaf_of,
                                                              const int32_t* __restrict__ leafoff,
                                                              const int32_t* __restrict__ koff,
                                                              const double* __restrict__ U,
                                                              const int64_t* __restrict__ uoff,
                                                              double* __restrict__ R) {
  const int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (p >= n) return;
  const int l = leaf_of[p];
  const int m = leafoff[l + 1] - leafoff[l];
  const int k = koff[l + 1] - koff[l];
  const double* u = U + uoff[l] + (p - leafoff[l]);
  for (int a = 0; a < kmax; ++a) R[a * n + p] = a < k ? u[int64_t(a) * m] : 0.0;
}

// Inner depth t: point p's ancestor c at depth t+1 is a row block of its
// parent's ID matrix [E_nu1; E_nu2] (rows rowbase.., rowbase + k_c), so
//   R_t(p, a) = sum_q R_{t+1}(p, q) U_par(rowbase + q, a).
__global__ __launch_bounds__(256) void basis_rows_inner_kernel(
    int64_t n, int shift, int kmax, const int32_t* __restrict__ leaf_of,
    const int32_t* __restrict__ rowoff, const int32_t* __restrict__ koff, const int32_t* __restrict__ koff_child,
    const double* __restrict__ U, const int64_t* __restrict__ uoff, const double* __restrict__ Rc,
    double* __restrict__ R) {
  const int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (p >= n) return;
  const int c = leaf_of[p] >> shift;  // ancestor at depth t+1
  const int par = c >> 1;
  const int m = rowoff[par + 1] - rowoff[par];
  const int k = koff[par + 1] - koff[par];
  const int kc = koff_child[c + 1] - koff_child[c];
  const int rowbase = koff_child[c] - rowoff[par];
  const double* u = U + uoff[par] + rowbase;
  for (int a = 0; a < kmax; ++a) {
    double acc = 0.0;
    if (a < k) {
      const double* ua = u + int64_t(a) * m;
      for (int q = 0; q < kc; ++q) acc = __builtin_fma(Rc[q * n + p], ua[q], acc);
    }
    R[a * n + p] = acc;
  }
}

// Index j in [lo, hi) with a[j] == key (a ascending, no duplicates), or -1.
__device__ __forceinline__ int find_sorted(const int32_t* __restrict__ a, int lo, int hi, int key) {
  int l = lo, h = hi;
  while (l < h) {
    const int mid = (l + h) >> 1;
    if (a[mid] < key)
      l = mid + 1;
    else
      h = mid;
  }
  return (l < hi && a[l] == key) ? l : -1;
}

struct EntryArgs {
  int64_t n;
  int depth, top, lr_rank;
  const int32_t* inv;
  const int32_t* leaf_of;
  const int32_t* leafoff;
  const int32_t* nptr;
  const int32_t* nidx;
  const int64_t* doff;
  const double* D;
  const double* lrU;  // n x lr_rank, tree order
  const double* lrV;
  const EntryLevel* levels;
};

__global__ __launch_bounds__(256) void entries_kernel(EntryArgs A, int nblocks, const int32_t* __restrict__ idx,
                                                      const int64_t* __restrict__ rbeg,
                                                      const int32_t* __restrict__ rcnt,
                                                      const int64_t* __restrict__ cbeg,
                                                      const int32_t* __restrict__ ccnt,
                                                      const int64_t* __restrict__ off, double* __restrict__ out) {
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int m = rcnt[b], nc = ccnt[b];
    const int64_t total = int64_t(m) * nc;
    const int32_t* ri = idx + rbeg[b];
    const int32_t* ci = idx + cbeg[b];
    double* o = out + off[b];
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      const int r = static_cast<int>(e % m), c = static_cast<int>(e / m);
      const int pi = A.inv[ri[r]], pj = A.inv[ci[c]];
      const int ls = A.leaf_of[pi], lb = A.leaf_of[pj];
      double v = __builtin_nan("");
      const int jn = find_sorted(A.nidx, A.nptr[ls], A.nptr[ls + 1], lb);
      if (jn >= 0) {
        const int ms = A.leafoff[ls + 1] - A.leafoff[ls];
        v = A.D[A.doff[jn] + (pi - A.leafoff[ls]) + int64_t(pj - A.leafoff[lb]) * ms];
        for (int q = 0; q < A.lr_rank; ++q) v = __builtin_fma(A.lrU[q * A.n + pi], A.lrV[q * A.n + pj], v);
      } else {
        for (int t = A.depth; t >= A.top; --t) {
          const EntryLevel L = A.levels[t - A.top];
          const int s = ls >> (A.depth - t), u = lb >> (A.depth - t);
          const int jf = find_sorted(L.fidx, L.fptr[s], L.fptr[s + 1], u);
          if (jf < 0) continue;
          const int ks = L.koff_r[s + 1] - L.koff_r[s];
          const int kb = L.koff_c[u + 1] - L.koff_c[u];
          const double* Bj = L.B + L.boff[jf];
          double acc = 0.0;
          for (int cc = 0; cc < kb; ++cc) {
            double w = 0.0;
            const double* col = Bj + int64_t(cc) * ks;
            for (int a = 0; a < ks; ++a) w = __builtin_fma(L.R[a * A.n + pi], col[a], w);
            acc = __builtin_fma(w, L.C[cc * A.n + pj], acc);
          }
          v = acc;
          break;
        }
      }
      o[r + int64_t(c) * m] = v;
    }
  }
}

__global__ __launch_bounds__(256) void gather_idx_kernel(int64_t n, const int32_t* __restrict__ map,
                                                         const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>(std::max<int64_t>((n + 255) / 256, 1)); }

// Expands the nested-basis rows of one side of h for every point.
void expand_side(const h2_matrix& h, const std::vector<Level>& lv, const EntryCache& ec,
                 std::vector<DevArray<double>>& out, hipStream_t s) {
  const int64_t n = h.plan.n;
  const int D = h.plan.depth;
  out.clear();
  out.resize(D + 1);
  for (int t = D; t >= h.top; --t) {
    const Level& L = lv[t];
    const int kmax = std::max(L.max_k, 1);
    out[t].alloc(size_t(n) * kmax, s);
    if (t == D) {
      basis_rows_leaf_kernel<<<blocks_for(n), 256, 0, s>>>(n, kmax, ec.leaf_of.get(), h.leafoff.get(), L.koff.get(),
                                                             L.U.get(), L.uoff.get(), out[t].get());
    } else {
      const Level& Cl = lv[t + 1];
      basis_rows_inner_kernel<<<blocks_for(n), 256, 0, s>>>(n, D - t - 1, kmax, ec.leaf_of.get(), L.rowoff.get(), L.koff.get(),
                                                              Cl.koff.get(), L.U.get(), L.uoff.get(),
                                                              out[t + 1].get(), out[t].get());
    }
    H2_HIP(hipGetLastError());
  }
}

const EntryCache& entry_cache(const h2_matrix& h, hipStream_t s) {
  if (h.entry_cache) return *static_cast<const EntryCache*>(h.entry_cache.get());
  auto ec = std::make_shared<EntryCache>();
  const int64_t n = h.plan.n;
  const int D = h.plan.depth;
  ec->inv.alloc(size_t(n), s);
  ec->leaf_of.alloc(size_t(n), s);
  inverse_perm_kernel<<<blocks_for(n), 256, 0, s>>>(n, h.perm.get(), ec->inv.get());
  H2_HIP(hipGetLastError());
  leaf_of_kernel<<<1 << D, 256, 0, s>>>(h.leafoff.get(), ec->leaf_of.get());
  H2_HIP(hipGetLastError());
  ec->top = h.top;
  if (h.top <= D) {
    expand_side(h, h.lv, *ec, ec->R, s);
    if (h.two_sided()) expand_side(h, h.lvc, *ec, ec->C, s);
    std::vector<EntryLevel> lv;
    for (int t = h.top; t <= D; ++t) {
      const Level& L = h.lv[t];
      const Level& Lc = h.col_levels()[t];
      EntryLevel e{};
      e.fptr = L.fptr.get();
      e.fidx = L.fidx.get();
      e.boff = L.boff.get();
      e.B = L.B.get();
      e.koff_r = L.koff.get();
      e.koff_c = Lc.koff.get();
      e.R = ec->R[t].get();
      e.C = h.two_sided() ? ec->C[t].get() : ec->R[t].get();
      lv.push_back(e);
    }
    ec->levels.alloc(lv.size(), s);
    H2_HIP(hipMemcpyAsync(ec->levels.get(), lv.data(), lv.size() * sizeof(EntryLevel), hipMemcpyHostToDevice, s));
    H2_HIP(hipStreamSynchronize(s));  // the host vector above is released on return
  }
  h.entry_cache = ec;
  return *ec;
}

}  // namespace

namespace h2dev {
hipError_t gather_idx(hipStream_t s, int64_t n, const int32_t* map, const int32_t* src, int32_t* dst) {
  if (n <= 0) return hipSuccess;
  gather_idx_kernel<<<blocks_for(n), 256, 0, s>>>(n, map, src, dst);
  return hipGetLastError();
}
}  // namespace h2dev

extern "C" h2_status h2_entries(h2_ctx* ctx, const h2_matrix* hm, int32_t nblocks, const int32_t* idx,
                                const int64_t* rbeg, const int32_t* rcnt, const int64_t* cbeg, const int32_t* ccnt,
                                const int64_t* off, double* out, int32_t max_rows, int32_t max_cols) {
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && hm != nullptr, "NULL argument");
    H2_REQUIRE(nblocks >= 0, "nblocks < 0");
    if (nblocks == 0) return;
    H2_REQUIRE(idx && rbeg && rcnt && cbeg && ccnt && off && out, "NULL array");
    H2_REQUIRE(max_rows >= 0 && max_cols >= 0, "negative block bound");
    const h2_matrix& h = *hm;
    H2_HIP(hipSetDevice(ctx->device));
    ArenaScope none(nullptr);  // the cache lives with the matrix, not with a build in progress
    hipStream_t s = ctx->stream;
    const EntryCache& ec = entry_cache(h, s);
    EntryArgs A{};
    A.n = h.plan.n;
    A.depth = h.plan.depth;
    A.top = h.top;
    A.lr_rank = h.lr_rank;
    A.inv = ec.inv.get();
    A.leaf_of = ec.leaf_of.get();
    A.leafoff = h.leafoff.get();
    A.nptr = h.nptr.get();
    A.nidx = h.nidx.get();
    A.doff = h.doff.get();
    A.D = h.Dblk.get();
    A.lrU = h.lrU.get();
    A.lrV = h.lrV.get();
    A.levels = ec.levels.get();
    const unsigned grid = static_cast<unsigned>(std::min(nblocks, 65535 * 8));
    entries_kernel<<<grid, 256, 0, s>>>(A, nblocks, idx, rbeg, rcnt, cbeg, ccnt, off, out);
    H2_HIP(hipGetLastError());
  });
}
