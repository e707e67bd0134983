// C ABI of the H^2 construction library: argument checking, device memory,
// and the host-driven level loop of Algorithm 1 with adaptive sampling
// (Sec. III-A, III-B).  All arithmetic runs in the kernels of h2_kernels.hip;
// the host only plans (cluster tree, interaction lists, offsets) and decides
// when to draw more samples.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "h2.h"
#include "h2_device.hpp"
#include "h2_internal.hpp"
#include "h2_plan.hpp"

namespace h2i {
thread_local std::string g_last_error;
}  // namespace h2i

using namespace h2i;

namespace h2i {

h2dev::KernelFn kernel_fn(const h2_kernel& k) {
  h2dev::KernelFn f;
  f.kind = k.kind;
  if (k.kind == H2_K_EXP)
    f.scale = 1.0 / k.length;
  else if (k.kind == H2_K_GAUSS)
    f.scale = 1.0 / (2.0 * k.length * k.length);
  else
    f.scale = k.wavenumber;
  return f;
}

void check_kernel(const h2_kernel* k) {
  H2_REQUIRE(k != nullptr, "kernel is NULL");
  H2_REQUIRE(k->kind == H2_K_EXP || k->kind == H2_K_GAUSS || k->kind == H2_K_HELMHOLTZ, "unknown kernel kind");
  if (k->kind == H2_K_HELMHOLTZ)
    H2_REQUIRE(k->wavenumber > 0.0 && std::isfinite(k->wavenumber), "wavenumber must be finite and > 0");
  else
    H2_REQUIRE(k->length > 0.0 && std::isfinite(k->length), "kernel length must be finite and > 0");
}

void call_sketch(h2_sketch_fn fn, void* user, int64_t n, int d, const double* om, int64_t ldo, double* y,
                 int64_t ldy, hipStream_t s) {
  ArenaScope none(nullptr);  // the callback's own library calls must not draw from the build's arena
  const int rc = fn(user, n, d, om, ldo, y, ldy, s);
  if (rc != 0) throw Error(H2_ERR_CALLBACK, "sketch callback returned " + std::to_string(rc));
}

void call_entries(h2_entry_fn fn, void* user, int nblocks, const int32_t* idx, const int64_t* rbeg,
                  const int32_t* rcnt, const int64_t* cbeg, const int32_t* ccnt, const int64_t* off, double* out,
                  int max_rows, int max_cols, hipStream_t s) {
  if (nblocks <= 0) return;
  ArenaScope none(nullptr);
  const int rc = fn(user, nblocks, idx, rbeg, rcnt, cbeg, ccnt, off, out, max_rows, max_cols, s);
  if (rc != 0) throw Error(H2_ERR_CALLBACK, "entry callback returned " + std::to_string(rc));
}

namespace {
struct HugeBlock {
  void* p;
  size_t bytes;
  hipStream_t s;
  int dev;
};
std::mutex g_huge_mu;
std::vector<HugeBlock> g_huge_free;         // released, kept for reuse
std::map<void*, HugeBlock> g_huge_live;     // handed out (bytes = the block's own size)
std::map<int, int64_t> g_huge_taken;        // bytes handed out from the cache since the last peak reset
}  // namespace

int64_t huge_taken(int device) {
  std::lock_guard<std::mutex> lock(g_huge_mu);
  return g_huge_taken[device];
}

void pool_peak_reset(int device) {
  {
    std::lock_guard<std::mutex> lock(g_huge_mu);
    g_huge_taken[device] = 0;
  }
  uint64_t zero = 0;
  hipMemPool_t def = nullptr;
  if (hipDeviceGetDefaultMemPool(&def, device) == hipSuccess)
    (void)hipMemPoolSetAttribute(def, hipMemPoolAttrUsedMemHigh, &zero);
  (void)hipMemPoolSetAttribute(large_pool(), hipMemPoolAttrUsedMemHigh, &zero);
}

// Bytes in use (high = false) or the high-water mark since the last reset
// (high = true) of the two stream-ordered pools the library allocates from.
int64_t pool_bytes(int device, bool high) {
  const hipMemPoolAttr attr = high ? hipMemPoolAttrUsedMemHigh : hipMemPoolAttrUsedMemCurrent;
  uint64_t a = 0, b = 0;
  hipMemPool_t def = nullptr;
  if (hipDeviceGetDefaultMemPool(&def, device) == hipSuccess) (void)hipMemPoolGetAttribute(def, attr, &a);
  (void)hipMemPoolGetAttribute(large_pool(), attr, &b);
  return static_cast<int64_t>(a + b);
}

hipMemPool_t large_pool() {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  H2_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  H2_HIP(hipMemPoolCreate(&pool, &props));
  uint64_t thr = UINT64_MAX;  // keep freed blocks for the next build
  H2_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
  pools[dev] = pool;
  return pool;
}

void* huge_take(size_t bytes, hipStream_t s) {
  int dev = 0;
  H2_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_huge_mu);
  // the smallest cached block that holds the request with at most 1/8 to spare
  size_t best = g_huge_free.size();
  for (size_t b = 0; b < g_huge_free.size(); ++b) {
    const HugeBlock& h = g_huge_free[b];
    if (h.dev == dev && h.s == s && h.bytes >= bytes && h.bytes - bytes <= bytes / 8 &&
        (best == g_huge_free.size() || h.bytes < g_huge_free[best].bytes))
      best = b;
  }
  if (best == g_huge_free.size()) return nullptr;
  const HugeBlock h = g_huge_free[best];
  g_huge_free.erase(g_huge_free.begin() + static_cast<std::ptrdiff_t>(best));
  g_huge_live[h.p] = h;
  g_huge_taken[dev] += static_cast<int64_t>(h.bytes);
  return h.p;
}

bool huge_put(void* p, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_huge_mu);
  auto it = g_huge_live.find(p);
  if (it == g_huge_live.end()) return false;
  HugeBlock h = it->second;
  g_huge_live.erase(it);
  h.s = s;  // the block's last use is ordered on s
  g_huge_free.push_back(h);
  return true;
}

void huge_trim(hipStream_t s) {
  std::vector<HugeBlock> drop;
  {
    std::lock_guard<std::mutex> lock(g_huge_mu);
    for (size_t b = 0; b < g_huge_free.size();) {
      if (!s || g_huge_free[b].s == s) {
        drop.push_back(g_huge_free[b]);
        g_huge_free.erase(g_huge_free.begin() + static_cast<std::ptrdiff_t>(b));
      } else {
        ++b;
      }
    }
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (const HugeBlock& h : drop) {
    (void)hipSetDevice(h.dev);
    if (!s) (void)hipStreamSynchronize(h.s);
    (void)hipFreeAsync(h.p, h.s);
  }
  (void)hipSetDevice(cur);
}

void* pool_alloc(size_t bytes, hipStream_t s) {
  if (bytes >= kHugeBytes) {
    if (void* p = huge_take(bytes, s)) return p;
  }
  const SmallArena* a = current_arena();
  const bool large = bytes >= kLargeBytes && !(a && a->large_default && a->serves(s));
  auto once = [&](void** p) {
    return large ? hipMallocFromPoolAsync(p, bytes, large_pool(), s) : hipMallocAsync(p, bytes, s);
  };
  void* p = nullptr;
  hipError_t e = once(&p);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    huge_trim(nullptr);
    H2_HIP(hipStreamSynchronize(s));
    int dev = 0;
    H2_HIP(hipGetDevice(&dev));
    hipMemPool_t def = nullptr;
    if (hipDeviceGetDefaultMemPool(&def, dev) == hipSuccess) (void)hipMemPoolTrimTo(def, 0);
    (void)hipMemPoolTrimTo(large_pool(), 0);
    e = once(&p);
  }
  H2_HIP(e);
  if (bytes >= kHugeBytes) {
    std::lock_guard<std::mutex> lock(g_huge_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    g_huge_live[p] = HugeBlock{p, bytes, s, dev};
  }
  return p;
}

SmallArena*& current_arena() {
  thread_local SmallArena* a = nullptr;
  return a;
}

void* SmallArena::take(size_t bytes, hipStream_t s) {
  if (s != stream_ || bytes > kMaxBytes) return nullptr;
  bytes = (bytes + 255) & ~size_t(255);
  if (used_ + bytes > cap_) {
    const size_t c = std::max(kChunkBytes, bytes);
    cur_ = static_cast<char*>(pool_alloc(c, stream_));
    chunks_.push_back(cur_);
    used_ = 0;
    cap_ = c;
  }
  void* p = cur_ + used_;
  used_ += bytes;
  return p;
}

SmallArena::~SmallArena() {
  for (void* c : chunks_) (void)hipFreeAsync(c, stream_);
}

void PanelWorkspace::ensure(int nodes, int max_m, int d, hipStream_t s) {
  const int64_t want = int64_t((max_m | 1) + 1) * int64_t((d | 1) + 1);
  if (want <= per && nodes <= nn) return;
  if (buf.size() < size_t(want) * nodes) buf.alloc(size_t(want) * nodes, s);
  per = want;
  nn = nodes;
  std::vector<int64_t> o(nodes);
  for (int i = 0; i < nodes; ++i) o[i] = want * i;
  off.upload(o, s);
}

void PrefixConvTest::init(hipStream_t s, int max_nodes, int inc, int oversample, double delta, size_t lds_limit) {
  inc_ = inc;
  ov_ = oversample;
  lds_ = lds_limit;
  zeros_.alloc(size_t(std::max(max_nodes, 1)), s);
  H2_HIP(h2dev::fill_i32(s, zeros_.get(), std::max(max_nodes, 1), 0));
  state_.alloc(4, s);
  delta_.upload(std::vector<double>{delta}, s);
}

int PrefixConvTest::first_converged(hipStream_t s, std::initializer_list<const Level*> levels, int d, int dsk,
                                    PanelWorkspace& ws) {
  int32_t* st = state_.get();
  H2_HIP(h2dev::fill_i32(s, st, 1, d));
  H2_HIP(h2dev::fill_i32(s, st + 1, 1, inc_));
  H2_HIP(h2dev::fill_i32(s, st + 2, 1, ov_));
  H2_HIP(h2dev::fill_i32(s, st + 3, 1, 0));
  for (const Level* L : levels) {
    if (size_t(L->max_m | 1) * size_t(dsk) * sizeof(double) > lds_) ws.ensure(L->nn, L->max_m, dsk, s);
    H2_HIP(h2dev::qr_first_conv(s, L->nn, L->rowoff.get(), L->y.get(), L->M, dsk, st + 1, st + 2, zeros_.get(), st,
                                delta_.get(), st + 3, L->max_m, lds_, ws.buf.get(), ws.off.get()));
  }
  const std::vector<int32_t> r = download(st, 4, s);
  return r[3] ? -1 : r[0];
}

// The context's second stream (default priority, created on first use and
// kept until the context is destroyed) for work that may overlap the build
// stream; none if not wanted, then work() is the build stream itself.  join() makes another stream wait for everything
// enqueued on it so far.
struct SideStream {
  hipStream_t s = nullptr;
  SideStream(h2_ctx* ctx, bool wanted) {
    if (!wanted) return;
    if (!ctx->side) H2_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    s = ctx->side;
  }
  hipStream_t work(hipStream_t build) const { return s ? s : build; }
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
  void join(hipStream_t other) {
    if (!s) return;
    hipEvent_t e = nullptr;
    H2_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, s);
    if (r == hipSuccess) r = hipStreamWaitEvent(other, e, 0);
    (void)hipEventDestroy(e);
    H2_HIP(r);
  }
};

int top_depth(const h2::Plan& p) {
  for (int t = 1; t <= p.depth; ++t)
    if (!p.far_idx[t].empty()) return t;
  return p.depth + 1;
}

// Every temporary of matvec_tree, in the order it takes them: the row-major
// staging copy of the block-sparse products, x_hat and y_hat per processed
// depth, and the leaf projection of a low-rank term.
template <typename Take>
static void matvec_temporaries(const h2_matrix& h, int64_t ldxt, int nc, bool trans, Take take, double** xr,
                               size_t* xr_cap, double** xh, double** yh, double** W) {
  const int D = h.plan.depth;
  trans = trans && h.two_sided();
  const std::vector<Level>& up = trans ? h.lv : h.col_levels();
  const std::vector<Level>& dn = trans ? h.col_levels() : h.lv;
  *xr_cap = h2dev::bsr_scratch_doubles(std::max<int64_t>(ldxt, h.plan.n), nc);
  *xr = take(*xr_cap);
  if (h.top <= D)
    for (int t = h.top; t <= D; ++t) {
      xh[t] = take(size_t(up[t].koff_h.back()) * nc);
      yh[t] = take(size_t(dn[t].koff_h.back()) * nc);
    }
  *W = h.lr_rank > 0 ? take(size_t(1 << D) * h.lr_rank * nc) : nullptr;
}

size_t matvec_tree_scratch(const h2_matrix& h, int nc, bool trans) {
  Workspace count(nullptr, 0);
  double* xh[32] = {};
  double* yh[32] = {};
  double *xr = nullptr, *W = nullptr;
  size_t cap = 0;
  matvec_temporaries(h, h.plan.n, nc, trans, [&](size_t d) { return count.take(d); }, &xr, &cap, xh, yh, &W);
  return count.used() / sizeof(double);
}

void matvec_tree(const h2_matrix& h, hipStream_t s, const double* xt, int64_t ldxt, double* yt, int64_t ldyt,
                 int nc, bool trans, Workspace* ws, bool near) {
  const int64_t n = h.plan.n;
  const int D = h.plan.depth;
  const int nleaves = 1 << D;
  if (nc <= 0) return;
  if (nc > 64) throw Error(H2_ERR_ARG, "matvec_tree: at most 64 columns");
  if (D > 30) throw Error(H2_ERR_ARG, "matvec_tree: tree too deep");
  // A symmetric build is its own transpose.  For a two-sided one, A^T x runs
  // up the row bases, applies B_{b,s}^T and goes down the column bases.
  trans = trans && h.two_sided();
  const std::vector<Level>& up = trans ? h.lv : h.col_levels();  // x_hat = (input-side basis)^T x
  const std::vector<Level>& dn = trans ? h.col_levels() : h.lv;  // y += (output-side basis) y_hat
  // temporaries: from the caller's workspace, else stream-ordered allocations
  DevArray<double> owned[2 * 32 + 2];
  int n_owned = 0;
  auto take = [&](size_t count) -> double* {
    if (ws) return ws->take(count);
    owned[n_owned].alloc(count, s);
    return owned[n_owned++].get();
  };
  double* xh[32] = {};
  double* yh[32] = {};
  double *xrp = nullptr, *W = nullptr;
  size_t xr_cap = 0;
  matvec_temporaries(h, ldxt, nc, trans, take, &xrp, &xr_cap, xh, yh, &W);
  if (h.top <= D) {
    for (int t = D; t >= h.top; --t) {  // upsweep
      const Level& L = up[t];
      const int64_t M = L.koff_h.back();
      const double* src = t == D ? xt : xh[t + 1];
      const int64_t lds = t == D ? ldxt : up[t + 1].koff_h.back();
      H2_HIP(h2dev::shrink_up(s, L.nn, L.rowoff.get(), L.koff.get(), L.J.get(), L.joff.get(), L.U.get(),
                              L.uoff.get(), nullptr, 0, src, lds, nullptr, 0, xh[t], M, nc, L.max_k));
      H2_HIP(h2dev::fill_zero(s, yh[t], dn[t].koff_h.back() * nc));
    }
    for (int t = h.top; t <= D; ++t) {  // couplings y_hat_s = sum_b B_{s,b} x_hat_b (or B_{b,s}^T)
      const Level& L = dn[t];
      const Level& C = up[t];
      const Level& R = h.lv[t];  // lists and blocks are stored with the row side
      H2_HIP(h2dev::bsr_gemm2(s, L.nn, R.fptr.get(), R.fidx.get(), L.koff.get(), C.koff.get(),
                              trans ? h.tpos[t].get() : nullptr, R.boff.get(), R.B.get(), xh[t],
                              C.koff_h.back(), yh[t], L.koff_h.back(), nc, 1.0,
                              std::max({L.max_k, C.max_k, 1}), xrp, xr_cap, 64, R.forder.get()));
    }
    for (int t = h.top; t <= D; ++t) {  // downsweep
      const Level& L = dn[t];
      double* dst = t == D ? yt : yh[t + 1];
      const int64_t ldd = t == D ? ldyt : dn[t + 1].koff_h.back();
      H2_HIP(h2dev::expand(s, L.nn, L.rowoff.get(), L.koff.get(), L.U.get(), L.uoff.get(), yh[t],
                           L.koff_h.back(), dst, ldd, nc));
    }
  }
  if (!near) return;
  int leaf_max = 0;
  for (int i = 0; i < nleaves; ++i) leaf_max = std::max(leaf_max, h.leafoff_h[i + 1] - h.leafoff_h[i]);
  H2_HIP(h2dev::bsr_gemm(s, nleaves, h.nptr.get(), h.nidx.get(), h.leafoff.get(), h.doff.get(), h.Dblk.get(), xt,
                         ldxt, yt, ldyt, nc, 1.0, leaf_max, xrp, xr_cap, 64, h.norder.get()));
  if (h.lr_rank > 0) {  // near-field part of the low-rank term: U_s sum_{b in N_s} V_b^T x_b (U, V swapped for A^T)
    const double* left = trans ? h.lrV.get() : h.lrU.get();
    const double* right = trans ? h.lrU.get() : h.lrV.get();
    H2_HIP(h2dev::lr_leaf_project(s, nleaves, h.leafoff.get(), right, n, h.lr_rank, xt, ldxt, nc, W));
    H2_HIP(h2dev::lr_apply(s, nleaves, h.nptr.get(), h.nidx.get(), h.leafoff.get(), n, left, n, h.lr_rank,
                           W, nc, yt, ldyt, 1.0));
  }
}

std::vector<int32_t> bsr_order(const std::vector<int32_t>& ptr) {
  const int rows = ptr.empty() ? 0 : static_cast<int>(ptr.size()) - 1;
  std::vector<int32_t> o(rows);
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b]; });
  return o;
}

}  // namespace h2i

namespace {

// The symmetric-tile sketch's scratch grows as 2 n^2 bytes.
void check_sym_size(int64_t n) {
  if (n > 163840) throw Error(H2_ERR_UNSUPPORTED, "H2_FP64_SYM needs about 2 n^2 bytes of scratch: n <= 163840");
}

void check_opts(const h2_opts* o) {
  H2_REQUIRE(o != nullptr, "opts is NULL");
  H2_REQUIRE(o->tol > 0.0 && std::isfinite(o->tol), "tol must be finite and > 0");
  H2_REQUIRE(o->leaf_size >= 2 && o->leaf_size <= 256, "leaf_size must be in [2, 256]");
  H2_REQUIRE(o->eta > 0.0 && std::isfinite(o->eta), "eta must be finite and > 0");
  H2_REQUIRE(o->d0 >= 1 && o->d0 <= 256, "d0 must be in [1, 256]");
  H2_REQUIRE(o->d_inc >= 0 && o->d_inc <= 128, "d_inc must be in [0, 128]");
  H2_REQUIRE(o->d_max >= o->d0 && o->d_max <= 256, "d_max must be in [d0, 256]");
  H2_REQUIRE(o->precision == H2_FP64 || o->precision == H2_FP32 || o->precision == H2_BF16X3 ||
                 o->precision == H2_FP32E || o->precision == H2_BF16X6 || o->precision == H2_FP64_SYM,
             "unknown precision");
  H2_REQUIRE(o->norm_mode == H2_NORM_FRO_SCALED || o->norm_mode == H2_NORM_LITERAL, "unknown norm_mode");
  H2_REQUIRE(o->sketch_ahead >= 0 && o->sketch_ahead <= 256, "sketch_ahead must be in [0, 256]");
  H2_REQUIRE(o->oversample >= 0 && o->oversample <= 64, "oversample must be in [0, 64]");
}


// The matrix given to Alg. 1: a built-in kernel (dense on-the-fly sketch and
// kernel entries) and/or the user's black box and entry evaluator.
struct Operator {
  const h2_kernel* kernel = nullptr;
  h2_sketch_fn sketch = nullptr;
  void* sketch_user = nullptr;
  h2_entry_fn entry = nullptr;
  void* entry_user = nullptr;
};

class Builder {
 public:
  Builder(h2_ctx* ctx, h2_matrix* h, const Operator& op)
      : ctx_(ctx), h_(h), s_(ctx->stream), timer_(ctx->stream), op_(op) {}

  void run(int64_t n, int dim, const double* points) {
    pool_peak_reset(ctx_->device);
    const int64_t used0 = pool_bytes(ctx_->device, false);
    hipEvent_t t0, t1;
    H2_HIP(hipEventCreate(&t0));
    H2_HIP(hipEventCreate(&t1));
    H2_HIP(hipEventRecord(t0, s_));
    try {
      run_inner(n, dim, points);
    } catch (...) {
      (void)hipStreamSynchronize(s_);
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      throw;
    }
    H2_HIP(hipEventRecord(t1, s_));
    H2_HIP(hipStreamSynchronize(s_));
    float ms = 0;
    H2_HIP(hipEventElapsedTime(&ms, t0, t1));
    h_->total_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    timer_.totals(h_->phase_ms, kNumPhase);
    // pool growth plus the cached huge blocks the build took (already counted in used0)
    h_->bytes_peak = pool_bytes(ctx_->device, true) - used0 + huge_taken(ctx_->device);
    // drop the build-only sample buffers
    for (auto& L : h_->lv) {
      L.om.release();
      L.y.release();
    }
  }

 private:
  h2_ctx* ctx_;
  h2_matrix* h_;
  hipStream_t s_;
  PhaseTimer timer_;
  Operator op_;
  h2dev::KernelFn kf_{};
  int dcap_ = 0, d_ = 0, dsk_ = 0, ahead_ = 0;
  const double* points_ = nullptr;  // caller's points, original order (borrowed for the build)
  PanelWorkspace ws_;
  PrefixConvTest conv_;
  BsrScratch xr_;

  int64_t n_ = 0;
  int dim_ = 0;

  void run_inner(int64_t n, int dim, const double* points) {
    n_ = n;
    dim_ = dim;
    h2_matrix& h = *h_;
    const h2_opts& o = h.opts;
    if (op_.kernel) kf_ = kernel_fn(*op_.kernel);
    points_ = points;
    dcap_ = o.d_max;
    ahead_ = o.d_inc > 0 ? o.sketch_ahead : 0;  // a fixed sample size draws d0 columns once
    std::vector<double> pts_h(static_cast<size_t>(n) * dim);
    H2_HIP(hipMemcpyAsync(pts_h.data(), points, pts_h.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
    H2_HIP(hipStreamSynchronize(s_));

    // ---- first sketch Y = K Omega (Alg. 1 batchedRand + black box), enqueued in
    // ORIGINAL point order so that it runs while the host builds the tree:
    // Omega(i, j) depends on the original index i only.
    int ph = timer_.begin(kSample);
    const int first = std::min(o.d0 + ahead_, dcap_);
    DevArray<double> om0, y0, part;
    om0.alloc(static_cast<size_t>(n) * first, s_);
    y0.alloc(static_cast<size_t>(n) * first, s_);
    H2_HIP(h2dev::gaussian(s_, o.seed, n, nullptr, 0, first, om0.get(), n));
    sketch_pass(om0.get(), y0.get(), first);
    const int nb = 512;
    part.alloc(nb, s_);
    // nu = ||Y_0||_F / sqrt(d0) from the first d0 columns: deterministic two-stage sum
    H2_HIP(h2dev::sumsq_partial(s_, n, o.d0, y0.get(), n, part.get(), nb));
    timer_.end(ph);

    // ---- plan (host): tree + lists, overlapping the sketch on the device
    const auto th0 = std::chrono::steady_clock::now();
    h.plan = h2::make_plan(n, dim, pts_h.data(), o.leaf_size, o.eta);
    h.host_plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
    const h2::Plan& p = h.plan;
    const int D = p.depth;
    const int nleaves = 1 << D;
    h.leafoff_h.assign(nleaves + 1, 0);
    for (int i = 0; i < nleaves; ++i) h.leafoff_h[i] = p.begin[p.level_begin(D) + i];
    h.leafoff_h[nleaves] = static_cast<int32_t>(n);
    std::vector<int64_t> dsz(p.near_idx.size());
    for (int s = 0; s < nleaves; ++s) {
      const int ms = h.leafoff_h[s + 1] - h.leafoff_h[s];
      for (int j = p.near_ptr[s]; j < p.near_ptr[s + 1]; ++j) {
        const int b = p.near_idx[j];
        dsz[j] = int64_t(ms) * (h.leafoff_h[b + 1] - h.leafoff_h[b]);
      }
    }
    h.doff_h = prefix(dsz);

    // ---- tree-ordered points and the dense near-field blocks
    // D_{tau,b} = K(I_tau, I_b) (Alg. 1 batchedGen) depend on the tree only.
    // With the split-bf16 sketches they are produced on a side stream while
    // the first sketch still runs on the build stream, which then waits for
    // them; their arrays are handed to the build stream, which orders their
    // later release.  The FP64 and FP32E sketches use the FP64 units that the
    // FP64 block generation needs, and run faster alone (measured: overlapping
    // them slowed the FP64 build by about 10 %).
    SideStream side(ctx_, o.precision == H2_BF16X3 || o.precision == H2_BF16X6);
    const hipStream_t gs = side.work(s_);
    auto adopt_all = [&] {
      h.perm.adopt(s_);
      h.X.adopt(s_);
      h.nptr.adopt(s_);
      h.norder.adopt(s_);
      h.nidx.adopt(s_);
      h.leafoff.adopt(s_);
      h.doff.adopt(s_);
      h.Dblk.adopt(s_);
    };
    try {
      ph = timer_.begin(kTree, gs);
      h.perm.upload(p.perm, gs);
      h.X.alloc(static_cast<size_t>(n) * dim, gs);
      H2_HIP(h2dev::permute_rows(gs, n, h.perm.get(), false, points, n, h.X.get(), n, dim));
      timer_.end(ph, gs);
      ph = timer_.begin(kNearGen, gs);
      h.nptr.upload(p.near_ptr, gs);
      h.norder.upload(bsr_order(p.near_ptr), gs);
      h.nidx.upload(p.near_idx, gs);
      h.leafoff.upload(h.leafoff_h, gs);
      h.doff.upload(h.doff_h, gs);
      h.Dblk.alloc(static_cast<size_t>(h.doff_h.back()), gs);
      if (op_.entry) {
        // D_{tau,b} = A(I_tau, I_b) from the entry callback: block j of the near
        // list is rows leafoff[s].. and columns leafoff[b].. of perm
        const size_t nnz = p.near_idx.size();
        std::vector<int64_t> rb(nnz), cb(nnz);
        std::vector<int32_t> rc(nnz), cc(nnz);
        int mmax = 0;
        for (int sl = 0; sl < nleaves; ++sl)
          for (int j = p.near_ptr[sl]; j < p.near_ptr[sl + 1]; ++j) {
            const int b = p.near_idx[j];
            rb[j] = h.leafoff_h[sl];
            rc[j] = h.leafoff_h[sl + 1] - h.leafoff_h[sl];
            cb[j] = h.leafoff_h[b];
            cc[j] = h.leafoff_h[b + 1] - h.leafoff_h[b];
            mmax = std::max(mmax, rc[j]);
          }
        DevArray<int64_t> rb_d, cb_d;
        DevArray<int32_t> rc_d, cc_d;
        rb_d.upload(rb, gs);
        cb_d.upload(cb, gs);
        rc_d.upload(rc, gs);
        cc_d.upload(cc, gs);
        call_entries(op_.entry, op_.entry_user, static_cast<int>(nnz), h.perm.get(), rb_d.get(), rc_d.get(),
                     cb_d.get(), cc_d.get(), h.doff.get(), h.Dblk.get(), mmax, mmax, gs);
      } else {
        H2_HIP(h2dev::gen_blocks(gs, nleaves, h.nptr.get(), h.nidx.get(), h.leafoff.get(), h.doff.get(), dim,
                                 h.X.get(), n, kf_, h.Dblk.get()));
      }
      timer_.end(ph, gs);
      side.join(s_);
    } catch (...) {
      (void)hipStreamSynchronize(gs);
      adopt_all();
      throw;
    }
    adopt_all();

    h.lv.clear();
    h.lv.resize(D + 1);
    for (int t = 0; t <= D; ++t) {
      h.lv[t].t = t;
      h.lv[t].nn = 1 << t;
    }
    h.top = top_depth(p);
    if (h.top > D) {  // no admissible block: the dense blocks are the whole matrix
      h.sketch_flops = h.sketch_entries = 0;
      h.sketch_calls = 0;
      return;
    }

    // ---- the first sketch in tree order; threshold from its first d0 columns
    ph = timer_.begin(kSample);
    Level& leaf = h.lv[D];
    leaf.M = n;
    leaf.om.alloc(static_cast<size_t>(n) * dcap_, s_);
    leaf.y.alloc(static_cast<size_t>(n) * dcap_, s_);
    H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, om0.get(), n, leaf.om.get(), n, first));
    H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, y0.get(), n, leaf.y.get(), n, first));
    std::vector<double> part_h = download(part.get(), nb, s_);
    double ss = 0;
    for (double v : part_h) ss += v;
    h.nu = std::sqrt(ss) / std::sqrt(double(o.d0));
    h.delta = o.norm_mode == H2_NORM_FRO_SCALED ? o.tol * h.nu / std::sqrt(double(nleaves)) : o.tol * h.nu;
    om0.release();
    y0.release();
    dsk_ = first;
    d_ = o.d0;
    timer_.end(ph);

    if (o.d_inc > 0) conv_.init(s_, nleaves, o.d_inc, o.oversample, h.delta, ctx_->lds_limit);

    for (int t = D; t >= h.top; --t) level(t);
    h.samples = d_;
    h.sketched = dsk_;
  }

  // Omega columns [c0, c0+nc) and Y = K Omega for them, computed in ORIGINAL
  // point order (like the first pass) and then gathered into tree order, so
  // every column is evaluated identically whichever pass produced it.
  void draw(int c0, int nc) {
    h2_matrix& h = *h_;
    Level& leaf = h.lv[h.plan.depth];
    const int64_t n = h.plan.n;
    DevArray<double> om, y;
    om.alloc(static_cast<size_t>(n) * nc, s_);
    y.alloc(static_cast<size_t>(n) * nc, s_);
    H2_HIP(h2dev::gaussian(s_, h.opts.seed, n, nullptr, c0, nc, om.get(), n));
    sketch_pass(om.get(), y.get(), nc);
    H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, om.get(), n, leaf.om.get() + int64_t(c0) * n, n, nc));
    H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, y.get(), n, leaf.y.get() + int64_t(c0) * n, n, nc));
  }

  // One pass of the black box Y = A Omega on nc columns in ORIGINAL order.
  void sketch_pass(const double* om, double* y, int nc) {
    h2_matrix& h = *h_;
    const int64_t n = n_;
    if (op_.sketch) {
      call_sketch(op_.sketch, op_.sketch_user, n, nc, om, n, y, n, s_);
    } else {
      DevArray<double> zs;  // the symmetric-tile sketch's scratch (kept by the huge-block cache)
      if (h.opts.precision == H2_FP64_SYM) zs.alloc(h2dev::sketch_sym_scratch_bytes(n) / sizeof(double), s_);
      H2_HIP(h2dev::sketch(s_, h.opts.precision, n, dim_, points_, n, kf_, nc, om, n, y, n, zs.get()));
      h.sketch_flops += 2.0 * double(n) * double(n) * nc;
      h.sketch_entries += double(n) * double(n);
    }
    h.sketch_calls++;
  }

  // Y_loc = Y^l - (near or far contributions) on columns [c0, c0+nc) at depth t.
  void subtract(int t, int c0, int nc) {
    h2_matrix& h = *h_;
    const int D = h.plan.depth;
    Level& L = h.lv[t];
    double* xr = xr_.get(L.M, nc, s_);
    if (t == D) {
      H2_HIP(h2dev::bsr_gemm(s_, L.nn, h.nptr.get(), h.nidx.get(), h.leafoff.get(), h.doff.get(), h.Dblk.get(),
                             L.om.get() + int64_t(c0) * L.M, L.M, L.y.get() + int64_t(c0) * L.M, L.M, nc, -1.0,
                             L.max_m, xr, xr_.cap(), 64, h.norder.get()));
    } else {
      Level& C = h.lv[t + 1];
      H2_HIP(h2dev::bsr_gemm(s_, C.nn, C.fptr.get(), C.fidx.get(), C.koff.get(), C.boff.get(), C.B.get(),
                             L.om.get() + int64_t(c0) * L.M, L.M, L.y.get() + int64_t(c0) * L.M, L.M, nc, -1.0,
                             std::max(C.max_k, 1), xr, xr_.cap(), 64, C.forder.get()));
    }
  }

  // Shrink + upsweep of depth t (its ID already computed) on columns [c0, c0+nc).
  void upsweep(int t, int c0, int nc) {
    h2_matrix& h = *h_;
    Level& L = h.lv[t];
    Level& P = h.lv[t - 1];
    H2_HIP(h2dev::shrink_up(s_, L.nn, L.rowoff.get(), L.koff.get(), L.J.get(), L.joff.get(), L.U.get(), L.uoff.get(),
                            L.y.get() + int64_t(c0) * L.M, L.M, L.om.get() + int64_t(c0) * L.M, L.M,
                            P.y.get() + int64_t(c0) * P.M, P.M, P.om.get() + int64_t(c0) * P.M, P.M, nc,
                            L.max_k));
  }


  void level(int t) {
    h2_matrix& h = *h_;
    const h2::Plan& p = h.plan;
    const int D = p.depth;
    Level& L = h.lv[t];
    L.processed = true;
    // in-rows of the clusters at depth t
    if (t == D) {
      L.rowoff_h = h.leafoff_h;
    } else {
      const Level& C = h.lv[t + 1];
      L.rowoff_h.resize(L.nn + 1);
      for (int i = 0; i <= L.nn; ++i) L.rowoff_h[i] = C.koff_h[2 * i];
      L.M = C.koff_h.back();
    }
    L.max_m = 0;
    for (int i = 0; i < L.nn; ++i) L.max_m = std::max(L.max_m, L.rowoff_h[i + 1] - L.rowoff_h[i]);
    L.rowoff.upload(L.rowoff_h, s_);

    int ph = timer_.begin(kSubtract);
    subtract(t, 0, dsk_);  // every sketched column, used or not yet
    timer_.end(ph);

    // adaptive sampling (Sec. III-B): the counts d_, d_ + d_inc, ... are
    // tested together on every sketched column (prefix test), then more
    // columns are sketched if none of them converges
    const int inc = h.opts.d_inc;
    while (inc > 0) {  // a fixed sample size (inc = 0) takes the d0 columns as they are
      ph = timer_.begin(kConv);
      const int dconv = conv_.first_converged(s_, {&L}, d_, dsk_, ws_);
      timer_.end(ph);
      if (dconv > 0) {
        h.rounds += (dconv - d_) / inc;
        d_ = dconv;
        break;
      }
      // every count up to the sketched columns fails: continue from the last one
      const int gmax = d_ + ((dsk_ - d_) / inc) * inc;
      h.rounds += (gmax - d_) / inc;
      d_ = gmax;
      if (d_ + inc > h.opts.d_max)
        throw Error(H2_ERR_SAMPLES, "adaptive sampling did not converge within d_max = " +
                                        std::to_string(h.opts.d_max) + " columns at depth " + std::to_string(t));
      const int need = d_ + inc;
      if (need > dsk_) {
        // sketch the missing columns plus the look-ahead, then updateSamples:
        // sweep them up through the finished levels
        const int c0 = dsk_, nc = std::min(need - dsk_ + ahead_, dcap_ - dsk_);
        ph = timer_.begin(kSample);
        draw(c0, nc);
        timer_.end(ph);
        for (int tt = D; tt >= t; --tt) {
          ph = timer_.begin(kSubtract);
          subtract(tt, c0, nc);
          timer_.end(ph);
          if (tt > t) {
            ph = timer_.begin(kUpsweep);
            upsweep(tt, c0, nc);
            timer_.end(ph);
          }
        }
        dsk_ += nc;
      }
      d_ = need;
      h.rounds++;
    }

    // row ID of every cluster (batchedID)
    ph = timer_.begin(kId);
    std::vector<int64_t> jsz(L.nn), usz(L.nn);
    for (int i = 0; i < L.nn; ++i) {
      const int m = L.rowoff_h[i + 1] - L.rowoff_h[i];
      jsz[i] = std::min(m, d_);
      usz[i] = int64_t(m) * std::min(m, d_);
    }
    L.joff_h = prefix(jsz);
    L.uoff_h = prefix(usz);
    L.joff.upload(L.joff_h, s_);
    L.uoff.upload(L.uoff_h, s_);
    L.J.alloc(static_cast<size_t>(L.joff_h.back()), s_);
    L.U.alloc(static_cast<size_t>(L.uoff_h.back()), s_);
    DevArray<int32_t> kdev;
    kdev.alloc(L.nn, s_);
    const size_t cbytes = size_t(3) * L.max_m * sizeof(double) + size_t(d_ | 1) * L.max_m * sizeof(double);
    if (cbytes > ctx_->lds_limit) ws_.ensure(L.nn, L.max_m, d_, s_);
    H2_HIP(h2dev::cpqr_id(s_, L.nn, L.rowoff.get(), L.y.get(), L.M, d_, h.delta, kdev.get(), L.J.get(), L.joff.get(),
                          L.U.get(), L.uoff.get(), L.max_m, ctx_->lds_limit, ws_.buf.get(), ws_.off.get()));
    L.k_h = download(kdev.get(), L.nn, s_);
    L.koff_h = prefix(L.k_h);
    L.koff.upload(L.koff_h, s_);
    L.max_k = 0;
    for (int k : L.k_h) L.max_k = std::max(L.max_k, k);
    timer_.end(ph);

    // shrink + upsweep into the next level's row space R_{t-1}
    ph = timer_.begin(kUpsweep);
    const int64_t Mn = L.koff_h.back();
    Level& P = h.lv[t - 1];
    if (t > h.top) {
      P.M = Mn;
      P.om.alloc(static_cast<size_t>(Mn) * dcap_, s_);
      P.y.alloc(static_cast<size_t>(Mn) * dcap_, s_);
      upsweep(t, 0, dsk_);
    }
    // skeleton tree positions and coordinates
    L.pos_out.alloc(static_cast<size_t>(Mn), s_);
    const int32_t* pos_in = (t == D) ? nullptr : h.lv[t + 1].pos_out.get();
    if (op_.entry) {  // entries come from the callback: no skeleton coordinates needed
      H2_HIP(h2dev::skeleton(s_, L.nn, L.rowoff.get(), L.koff.get(), L.J.get(), L.joff.get(), pos_in,
                             L.pos_out.get(), 0, nullptr, 0, nullptr, 0));
    } else {
      L.xs_out.alloc(static_cast<size_t>(Mn) * p.dim, s_);
      H2_HIP(h2dev::skeleton(s_, L.nn, L.rowoff.get(), L.koff.get(), L.J.get(), L.joff.get(), pos_in,
                             L.pos_out.get(), p.dim, h.X.get(), p.n, L.xs_out.get(), Mn));
    }
    timer_.end(ph);

    // coupling matrices B_{tau,b} = K(I~_tau, I~_b), b in F_tau  (batchedGen)
    ph = timer_.begin(kCoupling);
    L.fptr_h = p.far_ptr[t];
    L.fidx_h = p.far_idx[t];
    std::vector<int64_t> bsz(L.fidx_h.size());
    for (int s = 0; s < L.nn; ++s)
      for (int j = L.fptr_h[s]; j < L.fptr_h[s + 1]; ++j) bsz[j] = int64_t(L.k_h[s]) * L.k_h[L.fidx_h[j]];
    L.boff_h = prefix(bsz);
    L.fptr.upload(L.fptr_h, s_);
    L.forder.upload(bsr_order(L.fptr_h), s_);
    L.fidx.upload(L.fidx_h, s_);
    L.boff.upload(L.boff_h, s_);
    L.B.alloc(static_cast<size_t>(L.boff_h.back()), s_);
    if (op_.entry) {
      // B_{tau,b} = A(I~_tau, I~_b): the skeletons' original indices, block j of
      // the far list is rows koff[s].. and columns koff[b].. of them
      DevArray<int32_t> sk;
      sk.alloc(static_cast<size_t>(std::max<int64_t>(Mn, 1)), s_);
      H2_HIP(h2dev::gather_idx(s_, Mn, L.pos_out.get(), h.perm.get(), sk.get()));
      const size_t nnz = L.fidx_h.size();
      std::vector<int64_t> rb(nnz), cb(nnz);
      std::vector<int32_t> rc(nnz), cc(nnz);
      for (int a = 0; a < L.nn; ++a)
        for (int j = L.fptr_h[a]; j < L.fptr_h[a + 1]; ++j) {
          const int b = L.fidx_h[j];
          rb[j] = L.koff_h[a];
          rc[j] = L.k_h[a];
          cb[j] = L.koff_h[b];
          cc[j] = L.k_h[b];
        }
      DevArray<int64_t> rb_d, cb_d;
      DevArray<int32_t> rc_d, cc_d;
      rb_d.upload(rb, s_);
      cb_d.upload(cb, s_);
      rc_d.upload(rc, s_);
      cc_d.upload(cc, s_);
      call_entries(op_.entry, op_.entry_user, static_cast<int>(nnz), sk.get(), rb_d.get(), rc_d.get(), cb_d.get(),
                   cc_d.get(), L.boff.get(), L.B.get(), L.max_k, L.max_k, s_);
    } else {
      H2_HIP(h2dev::gen_blocks(s_, L.nn, L.fptr.get(), L.fidx.get(), L.koff.get(), L.boff.get(), p.dim,
                               L.xs_out.get(), Mn, kf_, L.B.get()));
    }
    timer_.end(ph);
  }
};

// Copies `bytes` from src (device memory when src_dev) to dst (device memory
// when dst_dev); dst == NULL only reports the size.
size_t copy_part(const void* src, size_t bytes, void* dst, size_t dst_bytes, size_t* needed, bool src_dev,
                 bool dst_dev, hipStream_t s) {
  if (needed) *needed = bytes;
  if (!dst) return bytes;
  if (dst_bytes < bytes) throw Error(H2_ERR_ARG, "destination too small");
  if (bytes == 0) return 0;
  if (src_dev || dst_dev) {
    const hipMemcpyKind kind = src_dev ? (dst_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost)
                                       : hipMemcpyHostToDevice;
    H2_HIP(hipMemcpyAsync(dst, src, bytes, kind, s));
    H2_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(dst, src, bytes);
  }
  return bytes;
}

void export_plan_part(const h2::Plan& p, int32_t part, int32_t depth, void* dst, size_t dst_bytes, size_t* needed,
                      bool dst_dev = false, hipStream_t s = nullptr) {
  switch (part) {
    case H2_PART_DEPTH: {
      const int32_t d = p.depth;
      copy_part(&d, sizeof d, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    }
    case H2_PART_PERM:
      copy_part(p.perm.data(), p.perm.size() * 4, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    case H2_PART_NODES: {
      std::vector<int32_t> v(2 * p.begin.size());
      for (size_t i = 0; i < p.begin.size(); ++i) {
        v[2 * i] = p.begin[i];
        v[2 * i + 1] = p.end[i];
      }
      copy_part(v.data(), v.size() * 4, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    }
    case H2_PART_BOXES: {
      std::vector<double> v;
      v.reserve(p.lo.size() * 2);
      for (int i = 0; i < p.num_nodes(); ++i) {
        for (int a = 0; a < p.dim; ++a) v.push_back(p.lo[size_t(i) * p.dim + a]);
        for (int a = 0; a < p.dim; ++a) v.push_back(p.hi[size_t(i) * p.dim + a]);
      }
      copy_part(v.data(), v.size() * 8, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    }
    case H2_PART_NEAR_PTR:
      copy_part(p.near_ptr.data(), p.near_ptr.size() * 4, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    case H2_PART_NEAR_IDX:
      copy_part(p.near_idx.data(), p.near_idx.size() * 4, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    case H2_PART_FAR_PTR:
    case H2_PART_FAR_IDX: {
      H2_REQUIRE(depth >= 0 && depth <= p.depth, "depth out of range");
      const auto& v = part == H2_PART_FAR_PTR ? p.far_ptr[depth] : p.far_idx[depth];
      copy_part(v.data(), v.size() * 4, dst, dst_bytes, needed, false, dst_dev, s);
      return;
    }
    default:
      throw Error(H2_ERR_STATE, "part not available for this object");
  }
}

}  // namespace

// ------------------------------------------- no-allocation product scratch
// h2_matvec_noalloc keeps its temporaries in this array instead of allocating.
// Each device holds its own copy (placed when the code object is loaded) until
// the process ends.  In host code the array's name is a host-side stand-in:
// kernels get the device address that hipGetSymbolAddress returned for the
// current device, looked up once per device when a context is created.
namespace {
constexpr size_t kNoAllocScratchBytes = H2_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `device`'s scratch array; `device` must be current.
void* scratch_address(int device) {
  H2_REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    H2_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    H2_REQUIRE(ptr != nullptr, "no device address for the scratch array");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}
}  // namespace

// =================================================================== C ABI

extern "C" {

h2_status h2_opts_default(h2_opts* o) {
  return guarded([&] {
    H2_REQUIRE(o != nullptr, "opts is NULL");
    o->tol = 1e-6;
    o->leaf_size = 64;
    o->eta = 0.7;
    o->d0 = 32;
    o->d_inc = 16;
    o->d_max = 256;
    o->seed = 1000;
    o->precision = H2_FP64;
    o->norm_mode = H2_NORM_FRO_SCALED;
    o->sketch_ahead = 32;
    o->oversample = 0;
  });
}

const char* h2_status_string(h2_status s) {
  switch (s) {
    case H2_OK: return "ok";
    case H2_ERR_ARG: return "invalid argument";
    case H2_ERR_HIP: return "HIP runtime error";
    case H2_ERR_OOM: return "out of device memory";
    case H2_ERR_CALLBACK: return "callback failed";
    case H2_ERR_SAMPLES: return "adaptive sampling reached d_max";
    case H2_ERR_STATE: return "invalid state";
    case H2_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* h2_last_error(void) { return g_last_error.c_str(); }

h2_status h2_ctx_create(int device, void* stream, h2_ctx** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    H2_REQUIRE(out != nullptr, "out is NULL");
    int count = 0;
    H2_HIP(hipGetDeviceCount(&count));
    H2_REQUIRE(device >= 0 && device < count, "device out of range");
    H2_HIP(hipSetDevice(device));
    auto c = std::make_unique<h2_ctx>();
    c->device = device;
    c->scratch = scratch_address(device);
    c->stream = static_cast<hipStream_t>(stream);
    int lds = 0;
    H2_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    c->lds_limit = lds > 2048 ? size_t(lds) - 1024 : size_t(lds);
    H2_HIP(h2dev::prepare_kernels(c->lds_limit));
    // keep freed device memory in the stream-ordered pool between builds
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    *out = c.release();
  });
}

h2_status h2_ctx_destroy(h2_ctx* ctx) {
  return guarded([&] {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) {
      (void)hipStreamSynchronize(ctx->side);
      huge_trim(ctx->side);
      (void)hipStreamDestroy(ctx->side);
    }
    huge_trim(ctx->stream);  // the stream is borrowed: keep no block ordered on it
    delete ctx;
  });
}

h2_status h2_plan_create(int64_t n, int32_t dim, const double* points_host, int32_t leaf_size, double eta,
                         h2_plan** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    H2_REQUIRE(out != nullptr, "out is NULL");
    auto p = std::make_unique<h2_plan>();
    p->plan = h2::make_plan(n, dim, points_host, leaf_size, eta);
    *out = p.release();
  });
}

h2_status h2_plan_create_device(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, int32_t leaf_size,
                                double eta, h2_plan** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && out != nullptr, "NULL argument");
    H2_HIP(hipSetDevice(ctx->device));
    auto p = std::make_unique<h2_plan>();
    p->plan = h2::make_plan_device(ctx->stream, n, dim, points, leaf_size, eta);
    *out = p.release();
  });
}

h2_status h2_plan_free(h2_plan* plan) {
  return guarded([&] { delete plan; });
}

h2_status h2_plan_export(const h2_plan* plan, int32_t part, int32_t depth, void* dst, size_t dst_bytes,
                         size_t* needed) {
  return guarded([&] {
    H2_REQUIRE(plan != nullptr, "plan is NULL");
    export_plan_part(plan->plan, part, depth, dst, dst_bytes, needed);
  });
}

h2_status h2_gaussian(h2_ctx* ctx, uint64_t seed, int64_t nrows, const int32_t* rows, int64_t col0, int32_t ncols,
                      double* out, int64_t ldo) {
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr, "ctx is NULL");
    H2_REQUIRE(nrows >= 0 && ncols >= 0 && col0 >= 0, "negative size");
    H2_REQUIRE(ldo >= std::max<int64_t>(nrows, 1), "ldo < nrows");
    H2_REQUIRE((rows && out) || nrows * int64_t(ncols) == 0, "NULL pointer");
    H2_HIP(hipSetDevice(ctx->device));
    H2_HIP(h2dev::gaussian(ctx->stream, seed, nrows, rows, col0, ncols, out, ldo));
  });
}

h2_status h2_sketch(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, const h2_kernel* kernel,
                    int32_t precision, int32_t ncols, const double* omega, int64_t ldo, double* y, int64_t ldy) {
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr, "ctx is NULL");
    check_kernel(kernel);
    H2_REQUIRE(precision == H2_FP64 || precision == H2_FP32 || precision == H2_BF16X3 || precision == H2_FP32E ||
                 precision == H2_BF16X6 || precision == H2_FP64_SYM,
               "unknown precision");
    H2_REQUIRE(n >= 0 && n < (int64_t{1} << 31), "n out of range");
    H2_REQUIRE(dim >= 1 && dim <= 3, "dim must be 1..3");
    H2_REQUIRE(ncols >= 0 && ncols <= 128, "ncols must be in [0, 128]");
    H2_REQUIRE(ldo >= std::max<int64_t>(n, 1) && ldy >= std::max<int64_t>(n, 1), "ld < n");
    H2_REQUIRE((points && omega && y) || n * int64_t(ncols) == 0, "NULL pointer");
    if (kernel->kind == H2_K_HELMHOLTZ && precision != H2_FP64 && precision != H2_FP64_SYM)
      throw Error(H2_ERR_UNSUPPORTED, "the Helmholtz kernel is evaluated in FP64 only");
    if (precision == H2_FP64_SYM) check_sym_size(n);
    H2_HIP(hipSetDevice(ctx->device));
    DevArray<double> zs;  // the symmetric-tile sketch's scratch (kept by the huge-block cache)
    if (precision == H2_FP64_SYM && ncols > 0)
      zs.alloc(h2dev::sketch_sym_scratch_bytes(n) / sizeof(double), ctx->stream);
    H2_HIP(h2dev::sketch(ctx->stream, precision, n, dim, points, n, kernel_fn(*kernel), ncols, omega, ldo, y, ldy,
                         zs.get()));
  });
}

h2_status h2_build(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, const h2_kernel* kernel,
                   h2_sketch_fn sketch, void* sketch_user, h2_entry_fn entry, void* entry_user,
                   const h2_opts* opts, h2_matrix** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && out != nullptr, "NULL argument");
    H2_REQUIRE(points != nullptr, "points is NULL");
    H2_REQUIRE(n >= 1 && n <= (int64_t{1} << 30), "n must be in [1, 2^30]");
    H2_REQUIRE(dim >= 1 && dim <= 3, "dim must be 1..3");
    if (kernel) {
      check_kernel(kernel);
      H2_REQUIRE(entry == nullptr, "entry callback given together with a kernel");
    } else {
      H2_REQUIRE(sketch != nullptr && entry != nullptr, "without a kernel both callbacks are required");
    }
    check_opts(opts);
    if (sketch && opts->precision != H2_FP64)
      throw Error(H2_ERR_UNSUPPORTED, "the precision modes apply to the built-in sketches only");
    if (kernel && kernel->kind == H2_K_HELMHOLTZ && opts->precision != H2_FP64 && opts->precision != H2_FP64_SYM)
      throw Error(H2_ERR_UNSUPPORTED, "the Helmholtz kernel is evaluated in FP64 only");
    if (opts->precision == H2_FP64_SYM) check_sym_size(n);
    H2_HIP(hipSetDevice(ctx->device));
    auto h = std::make_unique<h2_matrix>();
    h->device = ctx->device;
    h->stream = ctx->stream;
    if (kernel) h->kernel = *kernel;
    h->opts = *opts;
    h->small = std::make_shared<SmallArena>(ctx->stream);
    h->small->large_default = !(opts->precision == H2_BF16X3 || opts->precision == H2_BF16X6);
    Operator op;
    op.kernel = kernel;
    op.sketch = sketch;
    op.sketch_user = sketch_user;
    op.entry = entry;
    op.entry_user = entry_user;
    {
      ArenaScope scope(h->small.get());
      Builder b(ctx, h.get(), op);
      b.run(n, dim, points);
    }
    *out = h.release();
  });
}

h2_status h2_matvec(h2_ctx* ctx, const h2_matrix* hm, int32_t trans, int32_t nrhs, const double* x, int64_t ldx,
                    double* y, int64_t ldy) {
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && hm != nullptr, "NULL argument");
    H2_REQUIRE(trans == 0 || trans == 1, "trans must be 0 or 1");
    const h2_matrix& h = *hm;
    const int64_t n = h.plan.n;
    H2_REQUIRE(nrhs >= 0, "nrhs < 0");
    if (nrhs == 0) return;
    H2_REQUIRE(x && y, "NULL vector");
    H2_REQUIRE(ldx >= n && ldy >= n, "ld < n");
    H2_HIP(hipSetDevice(ctx->device));
    ArenaScope none(nullptr);  // temporaries of a matvec called inside a build are not the build's
    hipStream_t s = ctx->stream;
    const int chunk = 64;
    DevArray<double> xt, yt;
    xt.alloc(size_t(n) * chunk, s);
    yt.alloc(size_t(n) * chunk, s);
    for (int c0 = 0; c0 < nrhs; c0 += chunk) {
      const int nc = std::min(chunk, nrhs - c0);
      H2_HIP(h2dev::permute_rows(s, n, h.perm.get(), false, x + int64_t(c0) * ldx, ldx, xt.get(), n, nc));
      H2_HIP(h2dev::fill_zero(s, yt.get(), n * nc));
      matvec_tree(h, s, xt.get(), n, yt.get(), n, nc, trans != 0);
      H2_HIP(h2dev::permute_rows(s, n, h.perm.get(), true, yt.get(), n, y + int64_t(c0) * ldy, ldy, nc));
    }
    // temporaries are released stream-ordered; inputs stay valid until the stream passes this point
  });
}

h2_status h2_matvec_noalloc(h2_ctx* ctx, const h2_matrix* hm, int32_t trans, int32_t nrhs, const double* x,
                            int64_t ldx, double* y, int64_t ldy) {
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && hm != nullptr, "NULL argument");
    H2_REQUIRE(trans == 0 || trans == 1, "trans must be 0 or 1");
    const h2_matrix& h = *hm;
    const int64_t n = h.plan.n;
    H2_REQUIRE(nrhs >= 0, "nrhs < 0");
    if (nrhs == 0) return;
    H2_REQUIRE(x && y, "NULL vector");
    H2_REQUIRE(ldx >= n && ldy >= n, "ld < n");
    H2_REQUIRE(ctx->scratch != nullptr, "context has no scratch array");
    H2_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // the widest column chunk (<= 64) whose temporaries fit: tree-ordered x
    // and y, then matvec_tree's own
    auto need = [&](int nc) {
      return 2 * ((size_t(n) * nc * sizeof(double) + 255) & ~size_t(255)) +
             matvec_tree_scratch(h, nc, trans != 0) * sizeof(double);
    };
    int chunk = std::min(64, nrhs);
    while (chunk > 1 && need(chunk) > kNoAllocScratchBytes) --chunk;
    if (need(chunk) > kNoAllocScratchBytes)
      throw Error(H2_ERR_ARG, "h2_matvec_noalloc: one column needs " + std::to_string(need(1)) +
                                  " bytes of scratch, more than the " + std::to_string(kNoAllocScratchBytes) +
                                  " bytes it has (use h2_matvec)");
    char* base = static_cast<char*>(ctx->scratch);
    Workspace io(base, kNoAllocScratchBytes);
    double* xt = io.take(size_t(n) * chunk);
    double* yt = io.take(size_t(n) * chunk);
    for (int c0 = 0; c0 < nrhs; c0 += chunk) {
      const int nc = std::min(chunk, nrhs - c0);
      Workspace tree(base + io.used(), kNoAllocScratchBytes - io.used());
      H2_HIP(h2dev::permute_rows(s, n, h.perm.get(), false, x + int64_t(c0) * ldx, ldx, xt, n, nc));
      H2_HIP(h2dev::fill_zero(s, yt, n * nc));
      matvec_tree(h, s, xt, n, yt, n, nc, trans != 0, &tree);
      H2_HIP(h2dev::permute_rows(s, n, h.perm.get(), true, yt, n, y + int64_t(c0) * ldy, ldy, nc));
    }
  });
}

h2_status h2_export(const h2_matrix* hm, int32_t part, int32_t depth, int32_t on_device, void* dst,
                    size_t dst_bytes, size_t* needed) {
  return guarded([&] {
    H2_REQUIRE(hm != nullptr, "matrix is NULL");
    H2_REQUIRE(on_device == 0 || on_device == 1, "on_device must be 0 or 1");
    const h2_matrix& h = *hm;
    const h2::Plan& p = h.plan;
    hipStream_t s = h.stream;
    const bool dd = on_device != 0;
    if (dd) H2_HIP(hipSetDevice(h.device));
    if (part <= H2_PART_FAR_IDX) {
      export_plan_part(p, part, depth, dst, dst_bytes, needed, dd, s);
      return;
    }
    if (part == H2_PART_TOP) {
      const int32_t v = h.top;
      copy_part(&v, 4, dst, dst_bytes, needed, false, dd, s);
      return;
    }
    if (part == H2_PART_DENSE) {
      if (h.lr_rank == 0 || !dst) {
        copy_part(h.Dblk.get(), h.Dblk.bytes(), dst, dst_bytes, needed, true, dd, s);
        return;
      }
      // an update keeps D_old and the factors of U V^T: write the blocks out
      DevArray<double> tmp;
      tmp.alloc(h.Dblk.size(), s);
      H2_HIP(h2dev::dense_lowrank(s, 1 << p.depth, h.nptr.get(), h.nidx.get(), h.leafoff.get(), h.doff.get(),
                                  h.Dblk.get(), h.lrU.get(), p.n, h.lrV.get(), p.n, h.lr_rank, tmp.get()));
      copy_part(tmp.get(), tmp.bytes(), dst, dst_bytes, needed, true, dd, s);
      return;
    }
    H2_REQUIRE(depth >= 0 && depth <= p.depth, "depth out of range");
    const bool col = part >= H2_PART_RANKS_C && part <= H2_PART_SKEL_POS_C;
    if (col) part = part == H2_PART_RANKS_C  ? H2_PART_RANKS
                    : part == H2_PART_SKEL_C ? H2_PART_SKEL
                    : part == H2_PART_BASIS_C ? H2_PART_BASIS
                                              : H2_PART_SKEL_POS;
    const Level& L = col ? h.col_levels()[depth] : h.lv[depth];
    const Level& Lc = h.col_levels()[depth];
    const bool have = L.processed;
    switch (part) {
      case H2_PART_RANKS: {
        std::vector<int32_t> k(size_t(1) << depth, 0);
        if (have) k = L.k_h;
        copy_part(k.data(), k.size() * 4, dst, dst_bytes, needed, false, dd, s);
        return;
      }
      case H2_PART_SKEL:
      case H2_PART_SKEL_POS: {
        if (!have) {
          copy_part(nullptr, 0, dst, dst_bytes, needed, false, dd, s);
          return;
        }
        std::vector<int32_t> pos(L.pos_out.size());
        if (!pos.empty()) {
          H2_HIP(hipMemcpyAsync(pos.data(), L.pos_out.get(), pos.size() * 4, hipMemcpyDeviceToHost, s));
          H2_HIP(hipStreamSynchronize(s));
        }
        if (part == H2_PART_SKEL)
          for (auto& v : pos) v = p.perm[v];
        copy_part(pos.data(), pos.size() * 4, dst, dst_bytes, needed, false, dd, s);
        return;
      }
      case H2_PART_BASIS: {
        if (!have) {
          copy_part(nullptr, 0, dst, dst_bytes, needed, false, dd, s);
          return;
        }
        // packed m x k per node (U is stored with capacity m x min(m, d))
        std::vector<double> all(L.U.size());
        if (!all.empty()) {
          H2_HIP(hipMemcpyAsync(all.data(), L.U.get(), all.size() * 8, hipMemcpyDeviceToHost, s));
          H2_HIP(hipStreamSynchronize(s));
        }
        std::vector<double> packed;
        for (int i = 0; i < L.nn; ++i) {
          const int64_t m = L.rowoff_h[i + 1] - L.rowoff_h[i];
          const int64_t k = L.k_h[i];
          packed.insert(packed.end(), all.begin() + L.uoff_h[i], all.begin() + L.uoff_h[i] + m * k);
        }
        copy_part(packed.data(), packed.size() * 8, dst, dst_bytes, needed, false, dd, s);
        return;
      }
      case H2_PART_COUPLING: {
        if (!have) {
          copy_part(nullptr, 0, dst, dst_bytes, needed, false, dd, s);
          return;
        }
        // packed k_s x k_b per far pair in CSR order (storage may hold gaps)
        std::vector<double> all(L.B.size());
        if (!all.empty()) {
          H2_HIP(hipMemcpyAsync(all.data(), L.B.get(), all.size() * 8, hipMemcpyDeviceToHost, s));
          H2_HIP(hipStreamSynchronize(s));
        }
        std::vector<double> packed;
        for (int a = 0; a < L.nn; ++a)
          for (int j = L.fptr_h[a]; j < L.fptr_h[a + 1]; ++j) {
            const int64_t sz = int64_t(L.k_h[a]) * Lc.k_h[L.fidx_h[j]];
            packed.insert(packed.end(), all.begin() + L.boff_h[j], all.begin() + L.boff_h[j] + sz);
          }
        copy_part(packed.data(), packed.size() * 8, dst, dst_bytes, needed, false, dd, s);
        return;
      }
      default:
        throw Error(H2_ERR_ARG, "unknown part");
    }
  });
}

h2_status h2_query(const h2_matrix* hm, h2_info* info) {
  return guarded([&] {
    H2_REQUIRE(hm != nullptr && info != nullptr, "NULL argument");
    const h2_matrix& h = *hm;
    h2_info r{};
    r.n = h.plan.n;
    r.dim = h.plan.dim;
    r.depth = h.plan.depth;
    r.top = h.top;
    r.samples = h.samples;
    r.sketched = h.sketched;
    r.t_host_plan = h.host_plan_ms;
    r.rounds = h.rounds;
    r.delta = h.delta;
    r.norm_estimate = h.nu;
    r.rank_min = 1 << 30;
    r.rank_max = 0;
    r.near_blocks = static_cast<int64_t>(h.plan.near_idx.size());
    r.bytes_dense = static_cast<int64_t>(h.Dblk.bytes());
    for (const Level& L : h.lv) {
      if (!L.processed) continue;
      for (int k : L.k_h) {
        r.rank_min = std::min(r.rank_min, k);
        r.rank_max = std::max(r.rank_max, k);
      }
      r.far_blocks += static_cast<int64_t>(L.fidx_h.size());
      r.bytes_coupling += static_cast<int64_t>(L.B.bytes());
      r.bytes_basis += static_cast<int64_t>(L.U.bytes());
    }
    for (const Level& L : h.lvc) {  // column side of a two-sided matrix
      if (!L.processed) continue;
      for (int k : L.k_h) {
        r.rank_min = std::min(r.rank_min, k);
        r.rank_max = std::max(r.rank_max, k);
      }
      r.bytes_basis += static_cast<int64_t>(L.U.bytes());
    }
    r.bytes_dense += static_cast<int64_t>(h.lrU.bytes() + h.lrV.bytes());
    if (r.rank_max == 0 && r.rank_min == (1 << 30)) r.rank_min = 0;
    r.t_total = h.total_ms;
    r.t_tree = h.phase_ms[kTree];
    r.t_sample = h.phase_ms[kSample];
    r.t_near_gen = h.phase_ms[kNearGen];
    r.t_subtract = h.phase_ms[kSubtract];
    r.t_convtest = h.phase_ms[kConv];
    r.t_id = h.phase_ms[kId];
    r.t_upsweep = h.phase_ms[kUpsweep];
    r.t_coupling = h.phase_ms[kCoupling];
    double acc = 0;
    for (int ph = 0; ph < kNumPhase; ++ph) acc += h.phase_ms[ph];
    r.t_misc = std::max(0.0, h.total_ms - acc);
    r.sketch_flops = h.sketch_flops;
    r.sketch_entries = h.sketch_entries;
    r.sketch_calls = h.sketch_calls;
    r.fixed_samples = h.opts.d_inc == 0 ? 1 : 0;
    r.bytes_peak = h.bytes_peak;
    *info = r;
  });
}

h2_status h2_free(h2_matrix* h) {
  return guarded([&] {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    delete h;
    // releases are stream-ordered; nothing else to wait for
  });
}

}  // extern "C"
