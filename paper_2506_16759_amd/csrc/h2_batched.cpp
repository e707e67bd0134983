// Batched construction of many independent H^2 matrices (Alg. 1 with the
// adaptive sampling of Sec. III-B) in one launch sequence.
//
// Problems are ordered by the number of levels they process (descending), so
// the problems still active at any level are a prefix of that order and each
// level's clusters and row space are contiguous.  Every stage of a level is one
// kernel over the clusters of all active problems.  All d_max columns are
// sketched up front; the adaptive loop then only picks each problem's column
// count, from one prefix QR per cluster (qr_first_conv), so the device needs no
// host decision.  Storage uses static per-cluster capacities (k <= min(m,
// d_max)) except the compact skeleton rows, whose offsets come from a device
// scan.  With use_graph the whole sequence is captured in one hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <tuple>

#include "h2_internal.hpp"
#include "h2_pool.hpp"

using namespace h2i;

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// One device block carved into 256-byte aligned arrays.  A batch uses two:
// the factors the matrices keep (dense blocks, IDs, couplings) and the
// build's working set, released after the build.  Equal-sized blocks on
// repeated builds come straight back from the stream-ordered pool.
struct PinnedStage;

struct Arena {
  struct Item {
    size_t off, bytes;
    std::function<void(char*)> bind;
    const void* src;
  };
  std::vector<Item> items;
  size_t total = 0;
  DevArray<char> block;
  template <typename T>
  void want(DevArray<T>& a, size_t n) {
    add(a, n, nullptr);
  }
  template <typename T>
  void want(DevArray<T>& a, const std::vector<T>& h) {
    add(a, h.size(), h.data());
  }
  template <typename T>
  void add(DevArray<T>& a, size_t n, const void* src) {
    const size_t b = n * sizeof(T);
    DevArray<T>* pa = &a;
    items.push_back({total, b, [pa, n](char* p) { pa->borrow(reinterpret_cast<T*>(p), n); }, src});
    total += (b + 255) & ~size_t(255);
  }
  // allocate, bind every array and enqueue the uploads (host sources must stay
  // alive until the stream is synchronised)
  void commit(hipStream_t s) {
    block.alloc(std::max<size_t>(total, 256), s);
    for (auto& it : items) {
      it.bind(block.get() + it.off);
      if (it.src && it.bytes)
        H2_HIP(hipMemcpyAsync(block.get() + it.off, it.src, it.bytes, hipMemcpyHostToDevice, s));
    }
  }
  // The same through a pinned staging buffer: the arrays with host sources
  // are laid out first and sent in one asynchronous copy, so the call does not
  // wait for earlier work on the stream (a copy from pageable memory does).
  // The staging buffer must not be reused before the stream is synchronised.
  void commit_staged(hipStream_t s, PinnedStage& stage);
};

// A pinned host buffer, grown on demand (one per host thread and use).
struct PinnedStage {
  char* p = nullptr;
  size_t cap = 0;
  PinnedStage() = default;
  PinnedStage(const PinnedStage&) = delete;
  PinnedStage& operator=(const PinnedStage&) = delete;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
  char* get(size_t bytes) {
    if (bytes > cap) {
      const size_t want = std::max(bytes, cap * 2);
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      H2_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), want, hipHostMallocDefault));
      cap = want;
    }
    return p;
  }
};

void Arena::commit_staged(hipStream_t s, PinnedStage& stage) {
  size_t up = 0;
  for (auto& it : items)
    if (it.src) {
      it.off = up;
      up += (it.bytes + 255) & ~size_t(255);
    }
  size_t off = up;
  for (auto& it : items)
    if (!it.src) {
      it.off = off;
      off += (it.bytes + 255) & ~size_t(255);
    }
  block.alloc(std::max<size_t>(total, 256), s);
  char* h = up ? stage.get(up) : nullptr;
  for (auto& it : items) {
    it.bind(block.get() + it.off);
    if (it.src && it.bytes) std::memcpy(h + it.off, it.src, it.bytes);
  }
  if (up) H2_HIP(hipMemcpyAsync(block.get(), h, up, hipMemcpyHostToDevice, s));
}

// Small host arrays for many matrices, staged into one host buffer as they
// are added and sent to the device in one copy: each array is a view into one
// device block (256-byte aligned slices).  The staging buffer is kept per host
// thread and reused, so repeated batches neither grow nor fault in fresh pages.
std::vector<char>& packed_staging() {
  thread_local std::vector<char> buf;
  return buf;
}

struct Packed {
  std::vector<char>& host = packed_staging();
  Packed() { host.clear(); }
  std::vector<std::function<void(char*)>> bind;
  DevArray<char> block;
  template <typename T>
  void add(DevArray<T>& a, const std::vector<T>& h) {
    const size_t off = host.size(), b = h.size() * sizeof(T);
    host.resize(off + ((b + 255) & ~size_t(255)));
    if (b) std::memcpy(host.data() + off, h.data(), b);
    DevArray<T>* pa = &a;
    const size_t n = h.size();
    bind.push_back([pa, off, n](char* p) { pa->borrow(reinterpret_cast<T*>(p + off), n); });
  }
  // the host buffer must stay alive until the stream is synchronised
  void commit(hipStream_t s) {
    block.alloc(std::max<size_t>(host.size(), 256), s);
    if (!host.empty()) H2_HIP(hipMemcpyAsync(block.get(), host.data(), host.size(), hipMemcpyHostToDevice, s));
    for (auto& f : bind) f(block.get());
    bind.clear();
  }
};

struct Prob {
  int orig = 0;
  h2_problem in{};
  h2::Plan plan;
  int D = 0, top = 1, L = 0;  // tree depth, coarsest processed depth, processed levels
  int64_t base = 0;           // first global row
  int leafbase = 0;           // first global leaf
  int64_t dbase = 0;          // first dense-block entry
};

struct LevelB {
  int G = 0;
  std::vector<int32_t> nodeprob, childfirst, nodebase, mcap, kcap, fptr, fidx;
  std::vector<int64_t> joff, uoff, boff;
  int max_m = 0, max_k = 0;
  int64_t rcap = 0;       // rows of R_l (this level's in-rows)
  int64_t rcap_next = 0;  // rows of R_{l+1} (skeletons of this level)
  DevArray<int32_t> d_nodeprob, d_childfirst, rowoff, k, koff, J, pos, d_fptr, d_fidx;
  DevArray<int64_t> d_joff, d_uoff, d_boff, gws_off;
  DevArray<double> U, B, xs, om, y, gws;
  std::vector<int32_t> k_h, koff_h, rowoff_h;
  std::vector<int64_t> gws_off_h;
};

struct BatchStore {
  std::vector<LevelB> lv;  // index l-1
  DevArray<double> Xo, Xt, Om0, Y0, Dblk;
  DevArray<int32_t> perm_g, rowprob_o, rowlocal_o, leafoff, nptr, nidx, leafprob, kinds, dprob, incprob, ovprob,
      exhausted;
  DevArray<int64_t> doff;
  DevArray<uint64_t> seeds;
  DevArray<double> c2s, nu, delta;
  DevArray<double> xr;  // row-major staging of the block-sparse products (every level's row space fits)
  DevArray<char> sjobs, tjobs;
  DevArray<int32_t> tiles;
  Arena keep, work;  // factors kept by the matrices; the build's working set
  Arena pre;         // the original-order sketch's arrays (allocated before planning)
  Packed meta;       // the matrices' index arrays (permutation, offsets, lists)
  int64_t bytes = 0;
};

void check_problem(const h2_problem& p) {
  H2_REQUIRE(p.points != nullptr, "problem points are NULL");
  H2_REQUIRE(p.n >= 1 && p.n <= (int64_t{1} << 30), "problem n must be in [1, 2^30]");
  H2_REQUIRE(p.dim >= 1 && p.dim <= 3, "problem dim must be 1..3");
  check_kernel(&p.kernel);
  if (p.kernel.kind == H2_K_HELMHOLTZ)
    throw Error(H2_ERR_UNSUPPORTED, "batched builds take the covariance kernels only");
  H2_REQUIRE(p.tol > 0.0 && std::isfinite(p.tol), "problem tol must be finite and > 0");
  H2_REQUIRE(p.leaf_size >= 2 && p.leaf_size <= 256, "problem leaf_size must be in [2, 256]");
  H2_REQUIRE(p.eta > 0.0 && std::isfinite(p.eta), "problem eta must be finite and > 0");
  H2_REQUIRE(p.d0 >= 1 && p.d_inc >= 1, "problem d0, d_inc must be >= 1");
  H2_REQUIRE(p.norm_mode == H2_NORM_FRO_SCALED || p.norm_mode == H2_NORM_LITERAL, "unknown norm_mode");
  H2_REQUIRE(p.oversample >= 0 && p.oversample <= 64, "problem oversample must be in [0, 64]");
}

// Tile shapes of one launch sequence (columns per sketch launch, column-tile
// width of the block-sparse products).
struct Tiles {
  int sketch_cols = 64;
  int bsr_cols = 64;
};

// One launch sequence over `count` problems with dcap columns sketched up
// front.  A problem not converged within dcap columns gets no matrix (out[i]
// stays nullptr) and is listed in `exhausted`.  Arguments are validated by
// the caller.
//
// The dense sketch works in the problems' original point order and input
// order, so it needs no plan: it is enqueued first, and the host plans and
// lays out the batch while the device sketches.  Everything after it (tree
// order, near field, the levels) is one launch sequence, captured in a graph.

void build_pass(h2_ctx* ctx, int32_t count, const h2_problem* problems, int prec, int dcap, bool use_graph,
                const Tiles& tiles_shape, h2_matrix** out, std::vector<int>& exhausted, h2_batch_info* info) {
  {
    const auto t_start = Clock::now();
    H2_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    auto store = std::make_shared<BatchStore>();
    BatchStore& B = *store;
    int64_t& bytes = B.bytes;

    auto t0 = Clock::now();
    std::vector<Prob> P(count);
    for (int i = 0; i < count; ++i) {
      P[i].orig = i;
      P[i].in = problems[i];
    }

    // ---- the dense sketch in original order (problems in input order: rows
    // [base0[i], base0[i] + n_i) belong to problem i)
    std::vector<int64_t> base0(count + 1, 0);
    for (int i = 0; i < count; ++i) base0[i + 1] = base0[i] + problems[i].n;
    const int64_t NT = base0[count];
    H2_REQUIRE(NT < (int64_t{1} << 31), "total points must be < 2^31");
    // device events around the whole device work of this call
    struct Events {
      hipEvent_t e0 = nullptr, e1 = nullptr, ready = nullptr;
      ~Events() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ready) (void)hipEventDestroy(ready);
      }
    } ev;
    H2_HIP(hipEventCreate(&ev.e0));
    H2_HIP(hipEventCreate(&ev.e1));
    H2_HIP(hipEventCreateWithFlags(&ev.ready, hipEventDisableTiming));
    H2_HIP(hipEventRecord(ev.ready, s));  // the caller's earlier work on the stream (the points)
    // host sources of the uploads live until the end of the call
    std::vector<int32_t> tiles, rowprob_o(NT), rowlocal_o(NT);
    std::vector<uint64_t> seeds(count);
    std::vector<char> sj(h2dev::sketch_job_bytes() * count);
    // on an error after this point, let the enqueued work finish before the
    // host sources and the arrays it uses go away
    struct SyncOnUnwind {
      hipStream_t s;
      int n = std::uncaught_exceptions();
      ~SyncOnUnwind() {
        if (std::uncaught_exceptions() > n) (void)hipStreamSynchronize(s);
      }
    } unwind{s};
    {
      for (int i = 0; i < count; ++i)
        for (int64_t r = 0; r < problems[i].n; ++r) {
          rowprob_o[base0[i] + r] = i;
          rowlocal_o[base0[i] + r] = static_cast<int32_t>(r);
        }
      std::vector<std::pair<int64_t, int>> order(count);
      for (int i = 0; i < count; ++i) {
        seeds[i] = problems[i].seed;
        const h2dev::KernelFn kf = kernel_fn(problems[i].kernel);
        h2dev::pack_sketch_job(sj.data() + i * h2dev::sketch_job_bytes(), problems[i].n, base0[i], kf.kind,
                               kf.scale);
        order[i] = {problems[i].n, i};
      }
      // sketch tiles, largest problems first
      std::stable_sort(order.begin(), order.end(), [](auto& a, auto& b) { return a.first > b.first; });
      for (auto& o : order)
        for (int64_t r0 = 0; r0 < o.first; r0 += 128) {
          tiles.push_back(o.second);
          tiles.push_back(static_cast<int32_t>(r0));
        }
      B.pre.want(B.Xo, size_t(3) * NT);
      B.pre.want(B.Om0, size_t(NT) * dcap);
      B.pre.want(B.Y0, size_t(NT) * dcap);
      B.pre.want(B.rowprob_o, rowprob_o);
      B.pre.want(B.rowlocal_o, rowlocal_o);
      B.pre.want(B.seeds, seeds);
      B.pre.want(B.sjobs, sj);
      B.pre.want(B.tiles, tiles);
      B.pre.commit(s);
      H2_HIP(hipEventRecord(ev.e0, s));
      H2_HIP(h2dev::fill_zero(s, B.Xo.get(), 3 * NT));
      for (int i = 0; i < count; ++i)
        for (int a = 0; a < problems[i].dim; ++a)
          H2_HIP(hipMemcpyAsync(B.Xo.get() + a * NT + base0[i], problems[i].points + a * problems[i].n,
                                problems[i].n * sizeof(double), hipMemcpyDeviceToDevice, s));
      H2_HIP(h2dev::gaussian_batched(s, NT, B.rowlocal_o.get(), B.rowprob_o.get(), B.seeds.get(), 0, dcap,
                                     B.Om0.get(), NT));
      H2_HIP(h2dev::sketch_batched(s, prec, static_cast<int>(tiles.size() / 2), B.sjobs.get(), B.tiles.get(),
                                   B.Xo.get(), NT, dcap, B.Om0.get(), NT, B.Y0.get(), NT, tiles_shape.sketch_cols));
    }

    // ---- points to the host for planning, on the side stream (after the
    // caller's earlier work, beside the sketch)
    std::vector<std::vector<double>> pts(count);
    {
      if (!ctx->side) H2_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
      H2_HIP(hipStreamWaitEvent(ctx->side, ev.ready, 0));
      for (int i = 0; i < count; ++i) {
        pts[i].resize(static_cast<size_t>(problems[i].n) * problems[i].dim);
        H2_HIP(hipMemcpyAsync(pts[i].data(), problems[i].points, pts[i].size() * sizeof(double),
                              hipMemcpyDeviceToHost, ctx->side));
      }
      H2_HIP(hipStreamSynchronize(ctx->side));
    }

    // ---- host plans (threaded over problems)
    {
      // one problem per pool participant, largest first; each plan runs
      // serially inside its participant
      std::vector<std::string> errs(count);
      std::vector<int> order(count);
      for (int i = 0; i < count; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return problems[a].n > problems[b].n; });
      h2::parallel_for(count, 1, [&](int r) {
        const int i = order[r];
        try {
          P[i].plan = h2::make_plan(P[i].in.n, P[i].in.dim, pts[i].data(), P[i].in.leaf_size, P[i].in.eta);
        } catch (const std::exception& e) {
          errs[i] = e.what();
        }
      });
      for (int i = 0; i < count; ++i)
        if (!errs[i].empty()) throw Error(H2_ERR_ARG, "problem " + std::to_string(i) + ": " + errs[i]);
    }
    for (auto& p : P) {
      p.D = p.plan.depth;
      p.top = top_depth(p.plan);
      p.L = p.top > p.D ? 0 : p.D - p.top + 1;
    }
    const double t_plan = ms_since(t0);

    // ---- layout (problems ordered by processed levels, descending)
    t0 = Clock::now();
    std::stable_sort(P.begin(), P.end(), [](const Prob& a, const Prob& b) { return a.L > b.L; });
    const int np = count;
    int64_t nt = 0;
    int nleaf_total = 0;
    for (auto& p : P) {
      p.base = nt;
      nt += p.in.n;
      p.leafbase = nleaf_total;
      nleaf_total += 1 << p.D;
    }
    // global tree order: row p.base + r of the tree-ordered arrays is row
    // base0[orig] + perm[r] of the original-order ones
    std::vector<int32_t> perm_g(NT);
    h2::parallel_for(np, 1, [&](int q) {  // each problem fills its own rows
      const auto& p = P[q];
      for (int64_t r = 0; r < p.in.n; ++r) perm_g[p.base + r] = static_cast<int32_t>(base0[p.orig] + p.plan.perm[r]);
    });
    // leaves and near field
    std::vector<int32_t> leafoff(nleaf_total + 1), nptr(nleaf_total + 1, 0), nidx, leafprob(nleaf_total);
    std::vector<int64_t> dsz;
    int leaf_max = 0;
    for (int q = 0; q < np; ++q) {
      auto& p = P[q];
      const int nl = 1 << p.D, lb = p.plan.level_begin(p.D);
      for (int a = 0; a < nl; ++a) {
        leafoff[p.leafbase + a] = static_cast<int32_t>(p.base + p.plan.begin[lb + a]);
        leafprob[p.leafbase + a] = q;
        leaf_max = std::max(leaf_max, p.plan.end[lb + a] - p.plan.begin[lb + a]);
      }
    }
    leafoff[nleaf_total] = static_cast<int32_t>(NT);
    // near lists of problem q occupy entries [noff[q], noff[q+1]); filled per
    // problem in parallel, then the dense-block bases by a prefix over problems
    std::vector<int64_t> noff(np + 1, 0), dq(np, 0);
    for (int q = 0; q < np; ++q) noff[q + 1] = noff[q] + int64_t(P[q].plan.near_idx.size());
    nidx.assign(size_t(noff[np]), 0);
    dsz.assign(size_t(noff[np]), 0);
    h2::parallel_for(np, 1, [&](int q) {
      const auto& p = P[q];
      const int nl = 1 << p.D, lb = p.plan.level_begin(p.D);
      int64_t tot = 0;
      for (int a = 0; a < nl; ++a) {
        const int g = p.leafbase + a;
        const int ma = p.plan.end[lb + a] - p.plan.begin[lb + a];
        for (int j = p.plan.near_ptr[a]; j < p.plan.near_ptr[a + 1]; ++j) {
          const int b = p.plan.near_idx[j];
          nidx[noff[q] + j] = p.leafbase + b;
          const int64_t sz = int64_t(ma) * (p.plan.end[lb + b] - p.plan.begin[lb + b]);
          dsz[noff[q] + j] = sz;
          tot += sz;
        }
        nptr[g + 1] = static_cast<int32_t>(noff[q] + p.plan.near_ptr[a + 1]);
      }
      dq[q] = tot;
    });
    int64_t dtot = 0;
    for (int q = 0; q < np; ++q) {
      P[q].dbase = dtot;
      dtot += dq[q];
    }
    const std::vector<int64_t> doff = prefix(dsz);

    // levels
    int Lmax = 0;
    for (auto& p : P) Lmax = std::max(Lmax, p.L);
    B.lv.resize(Lmax);
    for (int l = 1; l <= Lmax; ++l) {
      LevelB& V = B.lv[l - 1];
      V.nodebase.assign(np, -1);
      for (int q = 0; q < np && P[q].L >= l; ++q) {
        const int t = P[q].D - l + 1;
        V.nodebase[q] = V.G;
        for (int a = 0; a < (1 << t); ++a) V.nodeprob.push_back(q);
        V.G += 1 << t;
      }
      V.mcap.resize(V.G);
      V.kcap.resize(V.G);
      if (l == 1) {
        V.rowoff_h.assign(leafoff.begin(), leafoff.begin() + V.G + 1);
        for (int g = 0; g < V.G; ++g) V.mcap[g] = V.rowoff_h[g + 1] - V.rowoff_h[g];
        V.rcap = NT;
      } else {
        const LevelB& C = B.lv[l - 2];
        V.childfirst.resize(V.G + 1);
        for (int q = 0; q < np && P[q].L >= l; ++q) {
          const int t = P[q].D - l + 1;
          for (int a = 0; a < (1 << t); ++a) {
            const int g = V.nodebase[q] + a, c = C.nodebase[q] + 2 * a;
            V.childfirst[g] = c;
            V.mcap[g] = C.kcap[c] + C.kcap[c + 1];
          }
        }
        // end of the last active cluster: the children of active problems are a prefix
        int cend = 0;
        for (int q = 0; q < np && P[q].L >= l; ++q) cend = C.nodebase[q] + (2 << (P[q].D - l + 1));
        V.childfirst[V.G] = cend;
        V.rcap = C.rcap_next;
      }
      for (int g = 0; g < V.G; ++g) {
        V.kcap[g] = std::min(V.mcap[g], dcap);
        V.max_m = std::max(V.max_m, V.mcap[g]);
        V.max_k = std::max(V.max_k, V.kcap[g]);
      }
      std::vector<int64_t> jsz(V.G), usz(V.G);
      for (int g = 0; g < V.G; ++g) {
        jsz[g] = V.kcap[g];
        usz[g] = int64_t(V.mcap[g]) * V.kcap[g];
      }
      V.joff = prefix(jsz);
      V.uoff = prefix(usz);
      V.rcap_next = V.joff.back();
      // far lists at this level, global cluster indices; capacity offsets
      V.fptr.assign(V.G + 1, 0);
      std::vector<int64_t> bsz;
      {
        size_t nf = 0;
        for (int q = 0; q < np && P[q].L >= l; ++q) nf += P[q].plan.far_idx[P[q].D - l + 1].size();
        V.fidx.reserve(nf);
        bsz.reserve(nf);
      }
      for (int q = 0; q < np && P[q].L >= l; ++q) {
        const int t = P[q].D - l + 1;
        const auto& fp = P[q].plan.far_ptr[t];
        const auto& fi = P[q].plan.far_idx[t];
        for (int a = 0; a < (1 << t); ++a) {
          const int g = V.nodebase[q] + a;
          for (int j = fp[a]; j < fp[a + 1]; ++j) {
            const int b = V.nodebase[q] + fi[j];
            V.fidx.push_back(b);
            bsz.push_back(int64_t(V.kcap[g]) * V.kcap[b]);
          }
          V.fptr[g + 1] = static_cast<int32_t>(V.fidx.size());
        }
      }
      V.boff = prefix(bsz);
    }

    // ---- device allocation and static uploads
    const double t_layout = ms_since(t0);
    const auto t_alloc0 = Clock::now();
    B.work.want(B.Xt, size_t(3) * NT);
    B.keep.want(B.Dblk, size_t(doff.back()));
    B.work.want(B.xr, h2dev::bsr_scratch_doubles(NT, dcap, tiles_shape.bsr_cols));
    B.work.want(B.perm_g, perm_g);
    B.work.want(B.leafoff, leafoff);
    B.work.want(B.nptr, nptr);
    B.work.want(B.nidx, nidx);
    B.work.want(B.doff, doff);
    B.work.want(B.leafprob, leafprob);
    std::vector<int32_t> kinds(np), incs(np), ovs(np);
    std::vector<double> c2s(np);
    std::vector<char> tj(h2dev::threshold_job_bytes() * np);
    for (int q = 0; q < np; ++q) {
      const auto& p = P[q];
      kinds[q] = p.in.kernel.kind;
      incs[q] = p.in.d_inc;
      ovs[q] = p.in.oversample;
      const h2dev::KernelFn kf = kernel_fn(p.in.kernel);
      c2s[q] = -kf.scale * 1.4426950408889634;
      h2dev::pack_threshold_job(tj.data() + q * h2dev::threshold_job_bytes(), p.base, p.in.n, p.in.d0, 1 << p.D,
                                p.in.norm_mode == H2_NORM_FRO_SCALED ? 0 : 1, p.in.tol);
    }
    B.work.want(B.kinds, kinds);
    B.work.want(B.incprob, incs);
    B.work.want(B.ovprob, ovs);
    B.work.want(B.c2s, c2s);
    B.work.want(B.tjobs, tj);
    B.work.want(B.nu, np);
    B.work.want(B.delta, np);
    B.work.want(B.dprob, np);
    B.work.want(B.exhausted, np);
    for (int l = 1; l <= Lmax; ++l) {
      LevelB& V = B.lv[l - 1];
      B.work.want(V.d_nodeprob, V.nodeprob);
      if (l == 1)
        B.work.want(V.rowoff, V.rowoff_h);
      else {
        B.work.want(V.d_childfirst, V.childfirst);
        B.work.want(V.rowoff, V.G + 1);
      }
      B.work.want(V.k, V.G);
      B.work.want(V.koff, V.G + 1);
      B.work.want(V.d_joff, V.joff);
      B.work.want(V.d_uoff, V.uoff);
      B.keep.want(V.J, size_t(V.joff.back()));
      B.keep.want(V.U, size_t(V.uoff.back()));
      B.work.want(V.pos, size_t(V.rcap_next));
      B.work.want(V.xs, size_t(3) * V.rcap_next);
      B.work.want(V.d_fptr, V.fptr);
      B.work.want(V.d_fidx, V.fidx);
      B.work.want(V.d_boff, V.boff);
      B.keep.want(V.B, size_t(V.boff.back()));
      if (l >= 2) {
        B.work.want(V.om, size_t(V.rcap) * dcap);
        B.work.want(V.y, size_t(V.rcap) * dcap);
      }
      const size_t cbytes = size_t(3) * V.max_m * 8 + size_t(dcap | 1) * V.max_m * 8;
      const size_t qbytes = size_t(V.max_m | 1) * dcap * 8;
      if (std::max(cbytes, qbytes) > ctx->lds_limit) {
        const int64_t per = int64_t((V.max_m | 1) + 1) * int64_t((dcap | 1) + 1);
        V.gws_off_h.resize(V.G);
        for (int g = 0; g < V.G; ++g) V.gws_off_h[g] = per * g;
        B.work.want(V.gws_off, V.gws_off_h);
        B.work.want(V.gws, size_t(per) * V.G);
      }
    }
    // level 1 works on the tree-ordered sketch itself
    DevArray<double> Om1, Y1;  // tree-ordered Omega and Y (level 1 row space)
    B.work.want(Om1, size_t(NT) * dcap);
    B.work.want(Y1, size_t(NT) * dcap);
    B.keep.commit(s);
    // uploads after the sketch was enqueued: pinned, so the host goes on
    thread_local PinnedStage stage;
    B.work.commit_staged(s, stage);
    bytes = static_cast<int64_t>(B.pre.total + B.keep.total + B.work.total);
    const double t_setup = ms_since(t0);
    const double t_alloc = ms_since(t_alloc0);

    // ---- the launch sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;  // capture stream
    if (use_graph) H2_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    auto enqueue = [&](hipStream_t s) {
      // points, Omega and the sketch (enqueued before planning) to tree order
      H2_HIP(h2dev::permute_rows(s, NT, B.perm_g.get(), false, B.Xo.get(), NT, B.Xt.get(), NT, 3));
      H2_HIP(h2dev::permute_rows(s, NT, B.perm_g.get(), false, B.Om0.get(), NT, Om1.get(), NT, dcap));
      H2_HIP(h2dev::permute_rows(s, NT, B.perm_g.get(), false, B.Y0.get(), NT, Y1.get(), NT, dcap));
      H2_HIP(h2dev::thresholds(s, np, B.tjobs.get(), Y1.get(), NT, B.nu.get(), B.delta.get(), B.dprob.get()));
      H2_HIP(h2dev::fill_i32(s, B.exhausted.get(), np, 0));
      // dense near field of every leaf, and its subtraction from the samples
      H2_HIP(h2dev::gen_blocks_batched(s, nleaf_total, B.nptr.get(), B.nidx.get(), B.leafoff.get(), B.doff.get(),
                                       B.Xt.get(), NT, B.leafprob.get(), B.kinds.get(), B.c2s.get(),
                                       B.Dblk.get()));
      H2_HIP(h2dev::bsr_gemm(s, nleaf_total, B.nptr.get(), B.nidx.get(), B.leafoff.get(), B.doff.get(),
                             B.Dblk.get(), Om1.get(), NT, Y1.get(), NT, dcap, -1.0, leaf_max, B.xr.get(),
                             B.xr.size(), tiles_shape.bsr_cols));
      for (int l = 1; l <= Lmax; ++l) {
        LevelB& V = B.lv[l - 1];
        double* om = l == 1 ? Om1.get() : V.om.get();
        double* y = l == 1 ? Y1.get() : V.y.get();
        const int64_t ld = V.rcap;
        if (l >= 2) {
          LevelB& C = B.lv[l - 2];
          H2_HIP(h2dev::gather_i32(s, V.G, V.d_childfirst.get(), C.koff.get(), V.rowoff.get()));
          H2_HIP(h2dev::bsr_gemm(s, C.G, C.d_fptr.get(), C.d_fidx.get(), C.koff.get(), C.d_boff.get(), C.B.get(),
                                 om, ld, y, ld, dcap, -1.0, std::max(C.max_k, 1), B.xr.get(), B.xr.size(),
                                 tiles_shape.bsr_cols));
        }
        H2_HIP(h2dev::qr_first_conv(s, V.G, V.rowoff.get(), y, ld, dcap, B.incprob.get(), B.ovprob.get(),
                                    V.d_nodeprob.get(), B.dprob.get(), B.delta.get(), B.exhausted.get(), V.max_m,
                                    ctx->lds_limit, V.gws.get(), V.gws_off.get()));
        H2_HIP(h2dev::cpqr_id(s, V.G, V.rowoff.get(), y, ld, dcap, 0.0, V.k.get(), V.J.get(), V.d_joff.get(),
                              V.U.get(), V.d_uoff.get(), V.max_m, ctx->lds_limit, V.gws.get(), V.gws_off.get(),
                              V.d_nodeprob.get(), B.dprob.get(), B.delta.get()));
        H2_HIP(h2dev::scan_i32(s, V.G, V.k.get(), V.koff.get()));
        if (l < Lmax) {
          LevelB& N = B.lv[l];
          H2_HIP(h2dev::shrink_up(s, V.G, V.rowoff.get(), V.koff.get(), V.J.get(), V.d_joff.get(), V.U.get(),
                                  V.d_uoff.get(), y, ld, om, ld, N.y.get(), N.rcap, N.om.get(), N.rcap, dcap,
                                  V.max_k));
        }
        const int32_t* pos_in = l == 1 ? nullptr : B.lv[l - 2].pos.get();
        H2_HIP(h2dev::skeleton(s, V.G, V.rowoff.get(), V.koff.get(), V.J.get(), V.d_joff.get(), pos_in,
                               V.pos.get(), 3, B.Xt.get(), NT, V.xs.get(), V.rcap_next));
        H2_HIP(h2dev::gen_blocks_batched(s, V.G, V.d_fptr.get(), V.d_fidx.get(), V.koff.get(), V.d_boff.get(),
                                         V.xs.get(), V.rcap_next, V.d_nodeprob.get(), B.kinds.get(), B.c2s.get(),
                                         V.B.get()));
      }
    };
    double t_capture = 0;
    size_t graph_nodes = 0;
    try {
      if (use_graph) {
        t0 = Clock::now();
        H2_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        try {
          enqueue(cs);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cs, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        H2_HIP(hipStreamEndCapture(cs, &graph));
        H2_HIP(hipGraphGetNodes(graph, nullptr, &graph_nodes));
        H2_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        t_capture = ms_since(t0);
        H2_HIP(hipGraphLaunch(exec, s));
      } else {
        enqueue(s);
      }
      H2_HIP(hipEventRecord(ev.e1, s));
      H2_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      if (cs) (void)hipStreamDestroy(cs);
      throw;
    }
    // from the sketch's start (before planning) to the end of the sequence
    float dev_ms = 0;
    H2_HIP(hipEventElapsedTime(&dev_ms, ev.e0, ev.e1));
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);

    // ---- results back to per-problem matrices (views into the batch storage)
    const auto t_res0 = Clock::now();
    const std::vector<int32_t> dprob = download(B.dprob.get(), np, s);
    const std::vector<int32_t> exh = download(B.exhausted.get(), np, s);
    const std::vector<double> nu = download(B.nu.get(), np, s);
    const std::vector<double> delta = download(B.delta.get(), np, s);
    for (int q = 0; q < np; ++q)
      if (exh[q] && P[q].L > 0) exhausted.push_back(P[q].orig);
    std::vector<std::vector<int32_t>> pos_h(Lmax);
    for (int l = 1; l <= Lmax; ++l) {
      LevelB& V = B.lv[l - 1];
      V.k_h = download(V.k.get(), V.G, s);
      V.koff_h = download(V.koff.get(), V.G + 1, s);
      if (l >= 2) V.rowoff_h = download(V.rowoff.get(), V.G + 1, s);
      pos_h[l - 1] = download(V.pos.get(), size_t(V.koff_h.back()), s);
    }
    std::vector<std::unique_ptr<h2_matrix>> mats(np);
    double sketch_flops = 0;
    for (int q = 0; q < np; ++q) {
      Prob& p = P[q];
      if (exh[q] && p.L > 0) continue;
      auto h = std::make_unique<h2_matrix>();
      h->device = ctx->device;
      h->stream = s;
      h->keep = store;
      h->kernel = p.in.kernel;
      h2_opts o{};
      o.tol = p.in.tol;
      o.leaf_size = p.in.leaf_size;
      o.eta = p.in.eta;
      o.d0 = p.in.d0;
      o.d_inc = p.in.d_inc;
      o.d_max = dcap;
      o.seed = p.in.seed;
      o.precision = prec;
      o.norm_mode = p.in.norm_mode;
      o.sketch_ahead = dcap - p.in.d0;
      o.oversample = p.in.oversample;
      h->opts = o;
      const int n = static_cast<int>(p.in.n);
      const int D = p.D;
      h->top = p.top;
      h->delta = p.L > 0 ? delta[q] : 0.0;
      h->nu = p.L > 0 ? nu[q] : 0.0;
      h->samples = p.L > 0 ? dprob[q] : 0;
      h->sketched = p.L > 0 ? dcap : 0;
      h->rounds = p.L > 0 ? (dprob[q] - p.in.d0) / p.in.d_inc : 0;
      B.meta.add(h->perm, p.plan.perm);
      const int nl = 1 << D;
      h->leafoff_h.resize(nl + 1);
      for (int a = 0; a <= nl; ++a) h->leafoff_h[a] = leafoff[p.leafbase + a] - static_cast<int32_t>(p.base);
      B.meta.add(h->leafoff, h->leafoff_h);
      B.meta.add(h->nptr, p.plan.near_ptr);
      B.meta.add(h->nidx, p.plan.near_idx);
      const int j0 = nptr[p.leafbase], j1 = nptr[p.leafbase + nl];
      h->doff_h.assign(doff.begin() + j0, doff.begin() + j1 + 1);
      for (auto& v : h->doff_h) v -= doff[j0];
      B.meta.add(h->doff, h->doff_h);
      h->Dblk.borrow(B.Dblk.get() + doff[j0], size_t(doff[j1] - doff[j0]));
      h->lv.resize(D + 1);
      for (int t = 0; t <= D; ++t) {
        h->lv[t].t = t;
        h->lv[t].nn = 1 << t;
      }
      for (int l = 1; l <= p.L; ++l) {
        LevelB& V = B.lv[l - 1];
        const int t = D - l + 1;
        Level& L = h->lv[t];
        const int g0 = V.nodebase[q], nn = 1 << t;
        L.processed = true;
        L.rowoff_h.resize(nn + 1);
        L.koff_h.resize(nn + 1);
        for (int a = 0; a <= nn; ++a) {
          L.rowoff_h[a] = V.rowoff_h[g0 + a] - V.rowoff_h[g0];
          L.koff_h[a] = V.koff_h[g0 + a] - V.koff_h[g0];
        }
        L.k_h.assign(V.k_h.begin() + g0, V.k_h.begin() + g0 + nn);
        L.joff_h.assign(V.joff.begin() + g0, V.joff.begin() + g0 + nn + 1);
        L.uoff_h.assign(V.uoff.begin() + g0, V.uoff.begin() + g0 + nn + 1);
        const int64_t jb = L.joff_h[0], ub = L.uoff_h[0];
        for (auto& v : L.joff_h) v -= jb;
        for (auto& v : L.uoff_h) v -= ub;
        L.max_m = 0;
        L.max_k = 0;
        for (int a = 0; a < nn; ++a) {
          L.max_m = std::max(L.max_m, L.rowoff_h[a + 1] - L.rowoff_h[a]);
          L.max_k = std::max(L.max_k, L.k_h[a]);
        }
        B.meta.add(L.rowoff, L.rowoff_h);
        B.meta.add(L.koff, L.koff_h);
        B.meta.add(L.joff, L.joff_h);
        B.meta.add(L.uoff, L.uoff_h);
        L.J.borrow(V.J.get() + jb, size_t(L.joff_h.back()));
        L.U.borrow(V.U.get() + ub, size_t(L.uoff_h.back()));
        // skeleton tree positions, local to the problem
        std::vector<int32_t> pos(pos_h[l - 1].begin() + V.koff_h[g0],
                                 pos_h[l - 1].begin() + V.koff_h[g0] + L.koff_h.back());
        for (auto& v : pos) v -= static_cast<int32_t>(p.base);
        B.meta.add(L.pos_out, pos);
        L.fptr_h = p.plan.far_ptr[t];
        L.fidx_h = p.plan.far_idx[t];
        const int f0 = V.fptr[g0], f1 = V.fptr[g0 + nn];
        L.boff_h.assign(V.boff.begin() + f0, V.boff.begin() + f1 + 1);
        const int64_t bb = L.boff_h[0];
        for (auto& v : L.boff_h) v -= bb;
        B.meta.add(L.fptr, L.fptr_h);
        B.meta.add(L.fidx, L.fidx_h);
        B.meta.add(L.boff, L.boff_h);
        L.B.borrow(V.B.get() + bb, size_t(L.boff_h.back()));
      }
      h->plan = std::move(p.plan);
      if (p.L > 0) {
        h->sketch_flops = 2.0 * double(n) * double(n) * dcap;
        h->sketch_entries = double(n) * double(n);
        sketch_flops += h->sketch_flops;
      }
      h->total_ms = dev_ms;
      mats[q] = std::move(h);
    }
    bytes += static_cast<int64_t>(B.meta.host.size());
    B.meta.commit(s);
    // only the factors stay: dense blocks, bases, skeleton indices, couplings
    H2_HIP(hipStreamSynchronize(s));
    B.meta.host.clear();
    B.work.block.release();
    for (int q = 0; q < np; ++q) out[P[q].orig] = mats[q].release();
    if (info) {
      h2_batch_info r{};
      r.t_total_ms = ms_since(t_start);
      r.t_plan_ms = t_plan;
      r.t_setup_ms = t_setup;
      r.t_layout_ms = t_layout;
      r.t_alloc_ms = t_alloc;
      r.t_results_ms = ms_since(t_res0);
      r.t_capture_ms = t_capture;
      r.t_device_ms = dev_ms;
      r.levels = Lmax;
      r.graph_nodes = static_cast<int32_t>(graph_nodes);
      r.device_bytes = bytes;
      r.sketch_flops = sketch_flops;
      *info = r;
    }
  }
}

}  // namespace

extern "C" h2_status h2_build_batched(h2_ctx* ctx, int32_t count, const h2_problem* problems,
                                      const h2_batch_opts* bopts, h2_matrix** out, h2_batch_info* info) {
  if (out && count > 0)
    for (int i = 0; i < count; ++i) out[i] = nullptr;
  return guarded([&] {
    const auto t_start = Clock::now();
    H2_REQUIRE(ctx && problems && bopts && out, "NULL argument");
    H2_REQUIRE(count >= 1, "count must be >= 1");
    const int prec = bopts->precision;
    if (prec == H2_FP64_SYM)
      throw Error(H2_ERR_UNSUPPORTED, "batched builds use the dense sketch (H2_FP64_SYM is for single builds)");
    H2_REQUIRE(prec == H2_FP64 || prec == H2_FP32 || prec == H2_BF16X3 || prec == H2_FP32E || prec == H2_BF16X6,
               "unknown precision");
    const int dcap = bopts->d_max;
    H2_REQUIRE(dcap >= 1 && dcap <= 96, "d_max must be in [1, 96]");
    H2_REQUIRE(bopts->first_pass >= 0, "first_pass must be >= 0");
    auto tile_ok = [](int c) { return c == 0 || c == 16 || c == 32 || c == 48 || c == 64; };
    H2_REQUIRE(tile_ok(bopts->sketch_cols), "sketch_cols must be 0, 16, 32, 48 or 64");
    H2_REQUIRE(tile_ok(bopts->bsr_cols), "bsr_cols must be 0, 16, 32, 48 or 64");
    Tiles shape;
    if (bopts->sketch_cols) shape.sketch_cols = bopts->sketch_cols;
    if (bopts->bsr_cols) shape.bsr_cols = bopts->bsr_cols;
    int d0max = 1;
    for (int i = 0; i < count; ++i) {
      check_problem(problems[i]);
      H2_REQUIRE(problems[i].d0 <= dcap, "problem d0 exceeds d_max");
      d0max = std::max(d0max, problems[i].d0);
    }
    H2_HIP(hipSetDevice(ctx->device));
    // first launch sequence: d0 plus the single build's default look-ahead
    // (32 columns) unless given; problems not converged within it are built
    // again, together, with d_max columns
    int first = bopts->first_pass > 0 ? bopts->first_pass : d0max + 32;
    first = std::max(d0max, std::min(first, dcap));
    const bool graph = bopts->use_graph != 0;
    std::vector<int> ex;
    h2_batch_info i1{}, i2{};
    int rerun = 0;
    auto drop = [&](h2_matrix** m, int k) {
      for (int i = 0; i < k; ++i)
        if (m[i]) {
          h2_free(m[i]);
          m[i] = nullptr;
        }
    };
    try {
      build_pass(ctx, count, problems, prec, first, graph, shape, out, ex, &i1);
      if (!ex.empty() && first < dcap) {
        std::vector<h2_problem> sub;
        for (int i : ex) sub.push_back(problems[i]);
        rerun = static_cast<int>(sub.size());
        std::vector<h2_matrix*> o2(sub.size(), nullptr);
        std::vector<int> ex2;
        try {
          build_pass(ctx, static_cast<int>(sub.size()), sub.data(), prec, dcap, graph, shape, o2.data(), ex2,
                     &i2);
        } catch (...) {
          drop(o2.data(), static_cast<int>(o2.size()));
          throw;
        }
        std::vector<int> still;
        for (int k : ex2) still.push_back(ex[k]);
        for (size_t k = 0; k < sub.size(); ++k) out[ex[k]] = o2[k];
        ex.swap(still);
      }
      if (!ex.empty())
        throw Error(H2_ERR_SAMPLES, "problem " + std::to_string(*std::min_element(ex.begin(), ex.end())) +
                                        " not converged within d_max = " + std::to_string(dcap) + " columns");
    } catch (...) {
      drop(out, count);
      throw;
    }
    if (info) {
      h2_batch_info r = i1;
      r.t_total_ms = ms_since(t_start);
      r.t_plan_ms += i2.t_plan_ms;
      r.t_setup_ms += i2.t_setup_ms;
      r.t_layout_ms += i2.t_layout_ms;
      r.t_alloc_ms += i2.t_alloc_ms;
      r.t_results_ms += i2.t_results_ms;
      r.t_capture_ms += i2.t_capture_ms;
      r.t_device_ms += i2.t_device_ms;
      r.levels = std::max(i1.levels, i2.levels);
      r.graph_nodes += i2.graph_nodes;
      r.device_bytes += i2.device_bytes;
      r.sketch_flops += i2.sketch_flops;
      r.first_pass = first;
      r.second_pass = rerun;
      r.sketch_cols = shape.sketch_cols;
      r.bsr_cols = shape.bsr_cols;
      *info = r;
    }
  });
}

// Leaf-size autotuner for batched builds.  Problems are grouped by (dim,
// kernel kind, floor(log2 n)); for each group the problem of median n is built
// alone (as a one-problem batch, graph launch) with every candidate leaf size,
// twice, and the candidate with the smallest device time of the second build
// is assigned to every problem of the group.  Candidates whose build fails
// (e.g. the sample cap is reached) are skipped.
extern "C" h2_status h2_autotune_leaf(h2_ctx* ctx, int32_t count, const h2_problem* problems,
                                      const h2_batch_opts* opts, const int32_t* candidates, int32_t ncand,
                                      int32_t* best) {
  return guarded([&] {
    H2_REQUIRE(ctx && problems && opts && candidates && best, "NULL argument");
    H2_REQUIRE(count >= 1 && ncand >= 1, "count and ncand must be >= 1");
    for (int c = 0; c < ncand; ++c)
      H2_REQUIRE(candidates[c] >= 2 && candidates[c] <= 256, "candidate leaf sizes must be in [2, 256]");
    for (int i = 0; i < count; ++i) check_problem(problems[i]);
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
      const auto& p = problems[i];
      const int lg = static_cast<int>(std::floor(std::log2(double(p.n))));
      groups[{p.dim, p.kernel.kind, lg}].push_back(i);
    }
    for (auto& [key, members] : groups) {
      std::vector<int> ord = members;
      std::sort(ord.begin(), ord.end(), [&](int a, int b) { return problems[a].n < problems[b].n; });
      h2_problem rep = problems[ord[ord.size() / 2]];
      int choice = -1;
      double tbest = 0;
      for (int c = 0; c < ncand; ++c) {
        rep.leaf_size = candidates[c];
        double t = -1;
        for (int rep_i = 0; rep_i < 2; ++rep_i) {
          h2_matrix* m = nullptr;
          h2_batch_info info{};
          const h2_status st = h2_build_batched(ctx, 1, &rep, opts, &m, &info);
          if (st != H2_OK) {
            if (st != H2_ERR_SAMPLES) throw Error(st, std::string("autotune build: ") + h2_last_error());
            t = -1;
            break;
          }
          h2_free(m);
          t = info.t_device_ms;
        }
        if (t >= 0 && (choice < 0 || t < tbest)) {
          choice = candidates[c];
          tbest = t;
        }
      }
      if (choice < 0) throw Error(H2_ERR_SAMPLES, "autotune: no candidate leaf size converged within d_max");
      for (int i : members) best[i] = choice;
    }
  });
}

// Tile-shape autotuner: coordinate search over the columns per sketch launch,
// then the column-tile width of the block-sparse products, on the batch
// itself (graph launches; the smaller device time of two builds counts).
extern "C" h2_status h2_autotune_tiles(h2_ctx* ctx, int32_t count, const h2_problem* problems,
                                       const h2_batch_opts* opts, h2_batch_opts* tuned, double* times_ms) {
  return guarded([&] {
    H2_REQUIRE(ctx && problems && opts && tuned, "NULL argument");
    H2_REQUIRE(count >= 1, "count must be >= 1");
    for (int i = 0; i < count; ++i) check_problem(problems[i]);
    std::vector<h2_matrix*> mats(count, nullptr);
    auto timed = [&](int sketch_cols, int bsr_cols, int reps) {
      h2_batch_opts o = *opts;
      o.use_graph = 1;
      o.sketch_cols = sketch_cols;
      o.bsr_cols = bsr_cols;
      double best = -1;
      for (int r = 0; r < reps; ++r) {
        h2_batch_info info{};
        const h2_status st = h2_build_batched(ctx, count, problems, &o, mats.data(), &info);
        if (st != H2_OK) throw Error(st, std::string("autotune build: ") + h2_last_error());
        for (auto& m : mats) {
          h2_free(m);
          m = nullptr;
        }
        if (best < 0 || info.t_device_ms < best) best = info.t_device_ms;
      }
      return best;
    };
    (void)timed(64, 64, 1);  // warm-up: allocations and code objects
    static const int kSketch[3] = {64, 48, 32};
    static const int kBsr[4] = {64, 48, 32, 16};
    double t[7];
    int sk = 64;
    double tbest = 0;
    for (int c = 0; c < 3; ++c) {
      t[c] = timed(kSketch[c], 64, 2);
      if (c == 0 || t[c] < tbest) {
        tbest = t[c];
        sk = kSketch[c];
      }
    }
    int bc = 64;
    for (int c = 0; c < 4; ++c) {
      // (sk, 64) was timed by the first search when sk is 64
      t[3 + c] = (c == 0 && sk == 64) ? t[0] : timed(sk, kBsr[c], 2);
      if (c == 0 || t[3 + c] < tbest) {
        tbest = t[3 + c];
        bc = kBsr[c];
      }
    }
    *tuned = *opts;
    tuned->sketch_cols = sk;
    tuned->bsr_cols = bc;
    if (times_ms)
      for (int c = 0; c < 7; ++c) times_ms[c] = t[c];
  });
}
