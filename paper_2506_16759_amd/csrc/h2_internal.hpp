// Internal types shared by the C ABI translation units: error handling,
// stream-ordered device arrays, per-depth level data and the matrix object.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <initializer_list>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "h2.h"
#include "h2_device.hpp"
#include "h2_plan.hpp"

namespace h2i {

extern thread_local std::string g_last_error;

struct Error : std::runtime_error {
  h2_status status;
  Error(h2_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

#define H2_HIP(expr)                                                                                    \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      throw ::h2i::Error(e_ == hipErrorOutOfMemory ? H2_ERR_OOM : H2_ERR_HIP,                           \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                            \
  } while (0)

#define H2_REQUIRE(cond, msg)                          \
  do {                                                 \
    if (!(cond)) throw ::h2i::Error(H2_ERR_ARG, msg);  \
  } while (0)

template <typename F>
h2_status guarded(F&& f) {
  try {
    f();
    return H2_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::invalid_argument& e) {
    g_last_error = e.what();
    return H2_ERR_ARG;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return H2_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return H2_ERR_HIP;
  }
}

// Stream-ordered pool of the current device for large arrays (>= 64 MB).
// Keeping them apart from the small per-level arrays stops the small ones from
// splitting a freed large block, so a repeated build of the same size gets its
// large blocks back without mapping new memory.  Single builds, whose small
// arrays come from an arena (below), take their large arrays on the build
// stream from the default pool too: releasing a block there is about ten times
// cheaper (a 131072-point matrix: 0.35 instead of 3.4 ms).  Builds that use
// the side stream keep every large array in the large pool: there the default
// pool's releases measured slower instead (about 6.6 ms per matrix).
hipMemPool_t large_pool();
constexpr size_t kLargeBytes = size_t(64) << 20;
// Device blocks of 1 GiB and more (dense near-field blocks, the largest
// coupling levels) are kept by the library when released and handed to the
// next request of about their size on the same device and stream: the
// stream-ordered pool does not reliably return a freed block of tens of GB to
// a later request of the same size (a build's smaller arrays may be carved out
// of it first), and mapping that much memory anew stalls the host about a
// second per 30 GB.  huge_take returns nullptr when no cached block fits;
// huge_put keeps a released block (false: not one of its blocks, the caller
// frees it); huge_trim frees the cached blocks of a stream (nullptr: of every
// stream, after synchronising them).
constexpr size_t kHugeBytes = size_t(1) << 30;
void* huge_take(size_t bytes, hipStream_t s);
bool huge_put(void* p, hipStream_t s);
void huge_trim(hipStream_t s);
// Stream-ordered allocation from the matching pool; on exhaustion the pools'
// cached free blocks are released (after the stream drains) and it retries once.
void* pool_alloc(size_t bytes, hipStream_t s);

// Device chunks for the many small arrays of one single build (index arrays,
// offsets, per-level scratch), released together with the matrix: one free
// per chunk instead of one per array.  Only allocations on the arena's stream
// and of at most kMaxBytes are served; others return nullptr.
class SmallArena {
 public:
  static constexpr size_t kMaxBytes = size_t(4) << 20;
  static constexpr size_t kChunkBytes = size_t(32) << 20;
  explicit SmallArena(hipStream_t s) : stream_(s) {}
  SmallArena(const SmallArena&) = delete;
  SmallArena& operator=(const SmallArena&) = delete;
  ~SmallArena();
  void* take(size_t bytes, hipStream_t s);
  bool serves(hipStream_t s) const { return s == stream_; }
  // large arrays on the arena's stream from the default pool (see large_pool)
  bool large_default = true;

 private:
  hipStream_t stream_;
  std::vector<void*> chunks_;
  char* cur_ = nullptr;
  size_t used_ = 0, cap_ = 0;
};
// The arena that DevArray::alloc draws from on this host thread (nullptr: none).
SmallArena*& current_arena();
// Sets the current arena for a scope.
struct ArenaScope {
  SmallArena* prev;
  explicit ArenaScope(SmallArena* a) : prev(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};

// Stream-ordered device array; borrow() makes it a non-owning view.  Small
// arrays allocated while an arena is current are views into it.
template <typename T>
class DevArray {
 public:
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  DevArray(DevArray&& o) noexcept { *this = std::move(o); }
  DevArray& operator=(DevArray&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_;
      n_ = o.n_;
      s_ = o.s_;
      owned_ = o.owned_;
      o.p_ = nullptr;
      o.n_ = 0;
    }
    return *this;
  }
  ~DevArray() { release(); }

  void alloc(size_t n, hipStream_t s) {
    release();
    s_ = s;
    n_ = n;
    owned_ = true;
    if (n == 0) return;
    if (SmallArena* a = current_arena()) {
      if (void* q = a->take(n * sizeof(T), s)) {
        p_ = static_cast<T*>(q);
        owned_ = false;
        return;
      }
    }
    p_ = static_cast<T*>(pool_alloc(n * sizeof(T), s));
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size(), s);
    if (!h.empty()) H2_HIP(hipMemcpyAsync(p_, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void borrow(T* p, size_t n) {
    release();
    p_ = n ? p : nullptr;
    n_ = n;
    owned_ = false;
  }
  void release() {
    if (p_ && owned_ && !huge_put(p_, s_)) (void)hipFreeAsync(p_, s_);
    p_ = nullptr;
    n_ = 0;
  }
  // Later releases are ordered on stream s; the caller has made s wait for
  // every use of the array on the stream it was allocated on.
  void adopt(hipStream_t s) { s_ = s; }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  hipStream_t s_ = nullptr;
  bool owned_ = true;
};

// Row-major staging buffer of the block-sparse products, grown on demand on
// the stream that uses it.
struct BsrScratch {
  DevArray<double> buf;
  double* get(int64_t ldx, int nc, hipStream_t s) {
    const size_t need = h2dev::bsr_scratch_doubles(ldx, nc);
    if (buf.size() < need) buf.alloc(need, s);
    return buf.get();
  }
  size_t cap() const { return buf.size(); }
};

template <typename T>
std::vector<T> download(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    H2_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
  }
  return h;
}

template <typename T>
std::vector<T> prefix(const std::vector<T>& sizes) {
  std::vector<T> off(sizes.size() + 1, 0);
  for (size_t i = 0; i < sizes.size(); ++i) off[i + 1] = off[i] + sizes[i];
  return off;
}

// Phase timer on HIP events: record pairs, resolve after the stream is synchronised.
class PhaseTimer {
 public:
  explicit PhaseTimer(hipStream_t s) : s_(s) {}
  ~PhaseTimer() {
    for (auto& r : recs_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
  // A phase is timed on the timer's stream or on another stream `on`, which
  // must have been joined into the timer's stream before totals().
  int begin(int phase, hipStream_t on = nullptr) {
    Rec r{phase, nullptr, nullptr};
    H2_HIP(hipEventCreate(&r.a));
    H2_HIP(hipEventCreate(&r.b));
    H2_HIP(hipEventRecord(r.a, on ? on : s_));
    recs_.push_back(r);
    return static_cast<int>(recs_.size()) - 1;
  }
  void end(int h, hipStream_t on = nullptr) { H2_HIP(hipEventRecord(recs_[h].b, on ? on : s_)); }
  void totals(double* out, int nphase) {
    H2_HIP(hipStreamSynchronize(s_));
    for (int p = 0; p < nphase; ++p) out[p] = 0;
    for (auto& r : recs_) {
      float ms = 0;
      H2_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      out[r.phase] += ms;
    }
  }

 private:
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  hipStream_t s_;
  std::vector<Rec> recs_;
};

enum Phase { kTree, kSample, kNearGen, kSubtract, kConv, kId, kUpsweep, kCoupling, kMisc, kNumPhase };

// Per-depth results of the construction.  Rows of depth t live in row space
// R_t (in-rows, `rowoff`) and the skeleton rows in R_{t-1} (`koff`).  Block
// and basis storage is addressed through the offset arrays (joff, uoff, boff),
// which may leave gaps (batched builds reserve capacity per cluster).
struct Level {
  int t = 0, nn = 0;
  bool processed = false;
  std::vector<int32_t> rowoff_h, k_h, koff_h;
  std::vector<int64_t> joff_h, uoff_h;
  int max_m = 0, max_k = 0;
  DevArray<int32_t> rowoff, koff, J, pos_out;
  DevArray<int64_t> joff, uoff;
  DevArray<double> U, xs_out;
  // far blocks at this depth
  std::vector<int32_t> fptr_h, fidx_h;
  std::vector<int64_t> boff_h;
  DevArray<int32_t> fptr, fidx;
  DevArray<int32_t> forder;  // block rows of the far lists, longest first (may be empty)
  DevArray<int64_t> boff;
  DevArray<double> B;
  // sample buffers of row space R_t (capacity columns), only during a build
  DevArray<double> om, y;
  int64_t M = 0;
};

// Rows of a CSR list (ptr, rows + 1 entries) by decreasing length, ties in row
// order: the launch order that balances a block-sparse product over the CUs.
std::vector<int32_t> bsr_order(const std::vector<int32_t>& ptr);

h2dev::KernelFn kernel_fn(const h2_kernel& k);
void check_kernel(const h2_kernel* k);
int top_depth(const h2::Plan& p);

// Per-cluster panels for the kernels whose panel (QR test, CPQR) exceeds LDS:
// one panel of `per` doubles per cluster.  The offsets are laid out again
// whenever a call needs a larger stride or more clusters: a buffer that is
// large enough in total but laid out with a smaller stride would hand
// overlapping panels to the clusters of a later level (fewer, larger clusters).
struct PanelWorkspace {
  DevArray<double> buf;
  DevArray<int64_t> off;
  int64_t per = 0;
  int nn = 0;
  void ensure(int nodes, int max_m, int d, hipStream_t s);
};

// Adaptive stopping test (Sec. III-B) on every sketched column at once: the
// smallest count d' on the grid d, d + inc, ... (d' <= dsk) at which every
// cluster of the given levels is converged, or -1 if some cluster is not
// converged within the dsk sketched columns.  The leading diagonal entries of
// a cluster's QR do not depend on later columns, so a converged count stays
// converged and the result equals testing d, d + inc, ... one at a time.
class PrefixConvTest {
 public:
  void init(hipStream_t s, int max_nodes, int inc, int oversample, double delta, size_t lds_limit);
  int first_converged(hipStream_t s, std::initializer_list<const Level*> levels, int d, int dsk,
                      PanelWorkspace& ws);

 private:
  DevArray<int32_t> zeros_, state_;  // state: d (raised in place), inc, oversample, exhausted
  DevArray<double> delta_;
  int inc_ = 16, ov_ = 0;
  size_t lds_ = 0;
};

}  // namespace h2i

struct h2_matrix;
namespace h2i {
// Bump allocator over device memory the caller owns: take() hands out
// consecutive 256-byte aligned slices and never allocates.  With base ==
// nullptr it only counts (used() is then the size a later run needs).
class Workspace {
 public:
  Workspace(void* base, size_t cap_bytes) : base_(static_cast<char*>(base)), cap_(cap_bytes) {}
  double* take(size_t doubles) {
    const size_t bytes = (doubles * sizeof(double) + 255) & ~size_t(255);
    if (base_ && used_ + bytes > cap_) throw Error(H2_ERR_ARG, "workspace exhausted");
    double* p = base_ ? reinterpret_cast<double*>(base_ + used_) : nullptr;
    used_ += bytes;
    return p;
  }
  size_t used() const { return used_; }

 private:
  char* base_;
  size_t cap_, used_ = 0;
};

// yt += A xt (or A^T xt when trans) for nc <= 64 columns, both in TREE order
// (ld >= n): the standard H^2 product (upsweep through the column bases,
// couplings, downsweep through the row bases) plus the near field (left out
// when near is false: the far-field part alone).  Stream-ordered on s.
// Temporaries come from ws when given (no allocation), else from the
// stream-ordered pools.
void matvec_tree(const h2_matrix& h, hipStream_t s, const double* xt, int64_t ldxt, double* yt, int64_t ldyt, int nc,
                 bool trans = false, Workspace* ws = nullptr, bool near = true);
// Doubles of workspace matvec_tree takes for nc columns with ldxt = n.
size_t matvec_tree_scratch(const h2_matrix& h, int nc, bool trans);
}  // namespace h2i

struct h2_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // created on first use, default priority, kept until h2_ctx_destroy
  size_t lds_limit = 65536;
  void* scratch = nullptr;  // device address of this device's no-allocation scratch array
};

struct h2_plan {
  h2::Plan plan;
};

struct h2_matrix {
  int device = 0;
  hipStream_t stream = nullptr;
  h2::Plan plan;
  h2_kernel kernel{};
  h2_opts opts{};
  int top = 1;
  double delta = 0, nu = 0;
  int samples = 0, sketched = 0, rounds = 0;
  double host_plan_ms = 0;
  h2i::DevArray<int32_t> perm;
  h2i::DevArray<double> X;  // tree-ordered SoA points (single builds)
  h2i::DevArray<int32_t> nptr, nidx, leafoff;
  h2i::DevArray<int32_t> norder;  // leaves by near-list length, longest first (may be empty)
  h2i::DevArray<int64_t> doff;
  std::vector<int64_t> doff_h;
  std::vector<int32_t> leafoff_h;
  h2i::DevArray<double> Dblk;
  std::vector<h2i::Level> lv;  // indexed by depth
  double phase_ms[h2i::kNumPhase] = {};
  double total_ms = 0;
  double sketch_flops = 0, sketch_entries = 0;
  int sketch_calls = 0;
  int64_t bytes_peak = 0;
  std::shared_ptr<void> keep;    // storage shared with other matrices of a batched build
  std::shared_ptr<void> keep_d;  // owner of Dblk when it is shared with an update
  std::shared_ptr<h2i::SmallArena> small;       // small arrays of a single build
  std::shared_ptr<h2i::SmallArena> keep_small;  // the arena of the matrix an update shares Dblk with
  // Two-sided matrices (low-rank updates): column-side levels, empty when the
  // matrix is symmetric (column bases = row bases).
  std::vector<h2i::Level> lvc;
  // Near blocks of an update are Dblk + U_s V_b^T: factors n x lr_rank, tree order.
  int lr_rank = 0;
  h2i::DevArray<double> lrU, lrV;
  // Two-sided matrices, per depth: CSR position of the mirrored far pair
  // (b, s) for every stored pair (s, b), for products with B^T.
  std::vector<h2i::DevArray<int64_t>> tpos;
  // Nested-basis rows of every point, expanded on the first h2_entries call.
  mutable std::shared_ptr<void> entry_cache;
  bool two_sided() const { return !lvc.empty(); }
  const std::vector<h2i::Level>& col_levels() const { return lvc.empty() ? lv : lvc; }
};

namespace h2 {
// The plan of make_plan built by device kernels on stream s from DEVICE points
// ((dim x n) SoA, original order); the same plan bit for bit.  Synchronises s.
// Throws std::invalid_argument like make_plan, Error on a HIP failure.
Plan make_plan_device(hipStream_t s, int64_t n, int dim, const double* points, int leaf_size, double eta);
}  // namespace h2
