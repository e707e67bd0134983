// Low-rank update of an H^2 matrix, A = H + U V^T, re-compressed on H's
// partition with the two-sided form of Algorithm 1 (adaptive sampling of
// Sec. III-B).  The black box is the H^2 product of H plus the low-rank
// product (Sec. V uses an H^2 matrix as the sampler); entries come from the
// format of H itself.
//
// Two-sided reading (the paper treats symmetric matrices and states that the
// non-symmetric case follows the same steps):
//   row side    Y = A Omega,    subtract D_{s,b} Omega_b / B_{s,b} (V_b^T Omega_b)
//   column side Z = A^T Omega', subtract D_{b,s}^T Omega'_b / B_{b,s}^T (U_b^T Omega'_b)
// Each side's random vectors are carried up by the other side's IDs; one
// sample count d serves both sides (a level is converged when every cluster
// of both sides is); Omega' uses seed + 1; delta comes from the row sketch.
//
// The leaf samples Alg. 1 works on are Y_loc = Y - sum_{b near s} A(s, b)
// Omega_b.  With H's own product as the sampler, the part D_H(s, b) Omega_b
// of Y is exactly what the subtraction removes, so neither is formed: the
// sampler runs H's product without its near field and the subtraction
// removes only the low-rank part U_s V_b^T Omega_b of the near blocks (the
// same Y_loc up to rounding, without reading the dense blocks twice per
// pass).  The norm estimate needs the full first d0 columns of Y: their near
// field is added once, to a copy.
//
// Entries of A at the new skeletons:
//   D_new(s, b) = D_H(s, b) + U_s V_b^T      kept as D_H plus the factors
//   B_new(s, b) = R_r_s B_H(s, b) R_c_b^T + U(I~r_s) V(I~c_b)^T
// where R_r_s = (nested basis of H at s)(I~r_s, :) is built level by level
// from the new skeleton selections (basis_rows) -- every admissible pair of
// the shared partition is an admissible pair of H, so H's entries there are
// exactly row_i(U_s) B_H(s, b) row_j(U_b)^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "h2_internal.hpp"

using namespace h2i;

namespace {

class UpdateBuilder {
 public:
  UpdateBuilder(h2_ctx* ctx, const h2_matrix& old, h2_matrix* h, int rank)
      : ctx_(ctx), old_(old), h_(h), s_(ctx->stream), timer_(ctx->stream), r_(rank) {}

  void run(const double* U, int64_t ldu, const double* V, int64_t ldv) {
    hipEvent_t t0, t1;
    H2_HIP(hipEventCreate(&t0));
    H2_HIP(hipEventCreate(&t1));
    H2_HIP(hipEventRecord(t0, s_));
    try {
      run_inner(U, ldu, V, ldv);
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
    for (auto* side : {&h_->lv, &h_->lvc})
      for (auto& L : *side) {
        L.om.release();
        L.y.release();
      }
  }

 private:
  h2_ctx* ctx_;
  const h2_matrix& old_;
  h2_matrix* h_;
  hipStream_t s_;
  PhaseTimer timer_;
  int r_;
  int dcap_ = 0, d_ = 0, dsk_ = 0, ahead_ = 0;
  DevArray<int32_t> perm_dev_;
  std::vector<DevArray<double>> Rr_, Rc_;  // per depth: rows of H's basis at the new skeletons
  std::vector<int> maxko_;
  DevArray<double> lrW_, lrPart_, lrSum_;
  PanelWorkspace ws_;
  PrefixConvTest conv_;
  BsrScratch xr_;


  void run_inner(const double* U, int64_t ldu, const double* V, int64_t ldv) {
    h2_matrix& h = *h_;
    const h2_opts& o = h.opts;
    dcap_ = o.d_max;
    ahead_ = o.sketch_ahead;
    const h2::Plan& p = h.plan;
    const int64_t n = p.n;
    const int D = p.depth;
    const int nleaves = 1 << D;

    // ---- structure shared with H: partition, dense blocks; U, V in tree order
    int ph = timer_.begin(kNearGen);
    h.perm.upload(p.perm, s_);
    perm_dev_.upload(p.perm, s_);
    h.leafoff_h = old_.leafoff_h;
    h.doff_h = old_.doff_h;
    h.leafoff.upload(h.leafoff_h, s_);
    h.doff.upload(h.doff_h, s_);
    h.nptr.upload(p.near_ptr, s_);
    h.norder.upload(bsr_order(p.near_ptr), s_);
    h.nidx.upload(p.near_idx, s_);
    h.lr_rank = r_;
    if (r_ > 0) {
      h.lrU.alloc(size_t(n) * r_, s_);
      h.lrV.alloc(size_t(n) * r_, s_);
      H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, U, ldu, h.lrU.get(), n, r_));
      H2_HIP(h2dev::permute_rows(s_, n, h.perm.get(), false, V, ldv, h.lrV.get(), n, r_));
    }
    timer_.end(ph);

    h.lv.clear();
    h.lv.resize(D + 1);
    h.lvc.clear();
    h.lvc.resize(D + 1);
    for (int t = 0; t <= D; ++t) {
      h.lv[t].t = h.lvc[t].t = t;
      h.lv[t].nn = h.lvc[t].nn = 1 << t;
    }
    h.top = old_.top;
    if (h.top > D) return;  // no admissible block: the dense blocks are the whole matrix

    // transposed positions of the far lists (column-side subtraction uses B_{b,s}^T)
    h.tpos.resize(D + 1);
    for (int t = h.top; t <= D; ++t) {
      const auto& fp = p.far_ptr[t];
      const auto& fi = p.far_idx[t];
      std::vector<int64_t> tp(fi.size());
      for (int a = 0; a < (1 << t); ++a)
        for (int j = fp[a]; j < fp[a + 1]; ++j) {
          const int b = fi[j];
          const auto* lo = fi.data() + fp[b];
          const auto* hi = fi.data() + fp[b + 1];
          const auto* it = std::lower_bound(lo, hi, a);
          if (it == hi || *it != a) throw Error(H2_ERR_STATE, "far lists are not symmetric");
          tp[j] = it - fi.data();
        }
      h.tpos[t].upload(tp, s_);
    }

    // ---- first sketch of both sides (tree order), threshold from the row sketch
    ph = timer_.begin(kSample);
    for (auto* side : {&h.lv, &h.lvc}) {
      Level& L = (*side)[D];
      L.M = n;
      L.om.alloc(size_t(n) * dcap_, s_);
      L.y.alloc(size_t(n) * dcap_, s_);
    }
    const int first = std::min(o.d0 + ahead_, dcap_);
    draw(0, first);
    const int nb = 512;
    DevArray<double> part;
    part.alloc(nb, s_);
    {
      // Y(:, 0:d0) = (far field + low rank, as drawn) + D_H Omega(:, 0:d0)
      Level& Lr = h.lv[D];
      DevArray<double> full;
      full.alloc(size_t(n) * o.d0, s_);
      H2_HIP(hipMemcpyAsync(full.get(), Lr.y.get(), size_t(n) * o.d0 * sizeof(double), hipMemcpyDeviceToDevice,
                            s_));
      int leaf_max = 0;
      for (int i = 0; i < nleaves; ++i) leaf_max = std::max(leaf_max, h.leafoff_h[i + 1] - h.leafoff_h[i]);
      for (int q0 = 0; q0 < o.d0; q0 += 64) {
        const int w = std::min(64, o.d0 - q0);
        double* xr = xr_.get(n, w, s_);
        H2_HIP(h2dev::bsr_gemm(s_, nleaves, h.nptr.get(), h.nidx.get(), h.leafoff.get(), h.doff.get(),
                               old_.Dblk.get(), Lr.om.get() + int64_t(q0) * n, n, full.get() + int64_t(q0) * n, n,
                               w, 1.0, leaf_max, xr, xr_.cap()));
      }
      H2_HIP(h2dev::sumsq_partial(s_, n, o.d0, full.get(), n, part.get(), nb));
    }
    std::vector<double> part_h = download(part.get(), nb, s_);
    double ss = 0;
    for (double v : part_h) ss += v;
    h.nu = std::sqrt(ss) / std::sqrt(double(o.d0));
    h.delta = o.norm_mode == H2_NORM_FRO_SCALED ? o.tol * h.nu / std::sqrt(double(nleaves)) : o.tol * h.nu;
    dsk_ = first;
    d_ = o.d0;
    timer_.end(ph);

    conv_.init(s_, nleaves, o.d_inc, o.oversample, h.delta, ctx_->lds_limit);
    Rr_.resize(D + 2);
    Rc_.resize(D + 2);
    maxko_.assign(D + 2, 0);
    for (int t = D; t >= h.top; --t) level(t);
    h.samples = d_;
    h.sketched = dsk_;
  }

  // Omega, Y = A Omega, Omega', Z = A^T Omega' for columns [c0, c0+nc), tree order.
  void draw(int c0, int nc) {
    h2_matrix& h = *h_;
    const int D = h.plan.depth;
    const int64_t n = h.plan.n;
    const int nleaves = 1 << D;
    Level& Lr = h.lv[D];
    Level& Lc = h.lvc[D];
    H2_HIP(h2dev::gaussian(s_, h.opts.seed, n, perm_dev_.get(), c0, nc, Lr.om.get() + int64_t(c0) * n, n));
    H2_HIP(h2dev::gaussian(s_, h.opts.seed + 1, n, perm_dev_.get(), c0, nc, Lc.om.get() + int64_t(c0) * n, n));
    const int chunk = 64;
    if (r_ > 0 && lrW_.size() < size_t(nleaves) * r_ * chunk) {
      lrW_.alloc(size_t(nleaves) * r_ * chunk, s_);
      lrPart_.alloc(h2dev::lr_sum_scratch(nleaves, r_ * chunk), s_);
      lrSum_.alloc(size_t(r_) * chunk, s_);
    }
    for (int a = 0; a < 2; ++a) {
      // row side: H Omega + U (V^T Omega); column side: H Omega' + V (U^T Omega')  (H symmetric)
      Level& L = a == 0 ? Lr : Lc;
      const double* left = a == 0 ? h.lrU.get() : h.lrV.get();
      const double* right = a == 0 ? h.lrV.get() : h.lrU.get();
      for (int q0 = 0; q0 < nc; q0 += chunk) {
        const int w = std::min(chunk, nc - q0);
        const double* x = L.om.get() + int64_t(c0 + q0) * n;
        double* y = L.y.get() + int64_t(c0 + q0) * n;
        H2_HIP(h2dev::fill_zero(s_, y, n * w));
        matvec_tree(old_, s_, x, n, y, n, w, false, nullptr, false);  // far field of H (its near field cancels)
        if (r_ > 0) {
          H2_HIP(h2dev::lr_leaf_project(s_, nleaves, h.leafoff.get(), right, n, r_, x, n, w, lrW_.get()));
          H2_HIP(h2dev::lr_sum(s_, nleaves, r_ * w, lrW_.get(), lrPart_.get(), lrSum_.get()));
          H2_HIP(h2dev::lr_apply(s_, nleaves, nullptr, nullptr, nullptr, n, left, n, r_, lrSum_.get(), w, y, n, 1.0));
        }
      }
    }
  }

  // Y_loc and Z_loc on columns [c0, c0+nc) at depth t.
  void subtract(int t, int c0, int nc) {
    h2_matrix& h = *h_;
    const int D = h.plan.depth;
    Level& Lr = h.lv[t];
    Level& Lc = h.lvc[t];
    const int64_t Mr = Lr.M, Mc = Lc.M;
    if (t == D) {
      const int64_t n = h.plan.n;
      const int nleaves = 1 << D;
      for (int a = 0; a < 2; ++a) {
        Level& L = a == 0 ? Lr : Lc;
        const double* left = a == 0 ? h.lrU.get() : h.lrV.get();
        const double* right = a == 0 ? h.lrV.get() : h.lrU.get();
        // the drawn samples hold no D_H part (see the top of this file): only
        // the low-rank part of the near blocks is subtracted
        if (r_ > 0) {
          for (int q0 = 0; q0 < nc; q0 += 64) {
            const int w = std::min(64, nc - q0);
            const double* x = L.om.get() + int64_t(c0 + q0) * n;
            H2_HIP(h2dev::lr_leaf_project(s_, nleaves, h.leafoff.get(), right, n, r_, x, n, w, lrW_.get()));
            H2_HIP(h2dev::lr_apply(s_, nleaves, h.nptr.get(), h.nidx.get(), h.leafoff.get(), n, left, n, r_,
                                   lrW_.get(), w, L.y.get() + int64_t(c0 + q0) * n, n, -1.0));
          }
        }
      }
      return;
    }
    const Level& Cr = h.lv[t + 1];
    const Level& Cc = h.lvc[t + 1];
    const int mk = std::max({Cr.max_k, Cc.max_k, 1});
    // row side: Y -= B_{s,b} (V_b^T Omega_b); Omega of the row side lives in column rows
    double* xr = xr_.get(std::max(Mr, Mc), nc, s_);
    H2_HIP(h2dev::bsr_gemm2(s_, Cr.nn, Cr.fptr.get(), Cr.fidx.get(), Cr.koff.get(), Cc.koff.get(), nullptr,
                            Cr.boff.get(), Cr.B.get(), Lr.om.get() + int64_t(c0) * Mc, Mc,
                            Lr.y.get() + int64_t(c0) * Mr, Mr, nc, -1.0, mk, xr, xr_.cap(), 64, Cr.forder.get()));
    // column side: Z -= B_{b,s}^T (U_b^T Omega'_b)
    H2_HIP(h2dev::bsr_gemm2(s_, Cr.nn, Cr.fptr.get(), Cr.fidx.get(), Cc.koff.get(), Cr.koff.get(),
                            h.tpos[t + 1].get(), Cr.boff.get(), Cr.B.get(), Lc.om.get() + int64_t(c0) * Mr, Mr,
                            Lc.y.get() + int64_t(c0) * Mc, Mc, nc, -1.0, mk, xr, xr_.cap(), 64, Cr.forder.get()));
  }

  // Shrink with each side's own ID; random vectors carried up by the other side's ID.
  void upsweep(int t, int c0, int nc) {
    h2_matrix& h = *h_;
    Level& Lr = h.lv[t];
    Level& Lc = h.lvc[t];
    Level& Pr = h.lv[t - 1];
    Level& Pc = h.lvc[t - 1];
    const int64_t Mr = Lr.M, Mc = Lc.M, PMr = Pr.M, PMc = Pc.M;
    // row side: Y_next = Y_loc(J_r); Omega_next = V^T Omega (column-side ID, column rows)
    H2_HIP(h2dev::shrink_up(s_, Lr.nn, Lr.rowoff.get(), Lr.koff.get(), Lr.J.get(), Lr.joff.get(), Lr.U.get(),
                            Lr.uoff.get(), Lr.y.get() + int64_t(c0) * Mr, Mr, nullptr, 0,
                            Pr.y.get() + int64_t(c0) * PMr, PMr, nullptr, 0, nc));
    H2_HIP(h2dev::shrink_up(s_, Lc.nn, Lc.rowoff.get(), Lc.koff.get(), Lc.J.get(), Lc.joff.get(), Lc.U.get(),
                            Lc.uoff.get(), nullptr, 0, Lr.om.get() + int64_t(c0) * Mc, Mc, nullptr, 0,
                            Pr.om.get() + int64_t(c0) * PMc, PMc, nc, Lc.max_k));
    // column side: Z_next = Z_loc(J_c); Omega'_next = U^T Omega' (row-side ID, row rows)
    H2_HIP(h2dev::shrink_up(s_, Lc.nn, Lc.rowoff.get(), Lc.koff.get(), Lc.J.get(), Lc.joff.get(), Lc.U.get(),
                            Lc.uoff.get(), Lc.y.get() + int64_t(c0) * Mc, Mc, nullptr, 0,
                            Pc.y.get() + int64_t(c0) * PMc, PMc, nullptr, 0, nc));
    H2_HIP(h2dev::shrink_up(s_, Lr.nn, Lr.rowoff.get(), Lr.koff.get(), Lr.J.get(), Lr.joff.get(), Lr.U.get(),
                            Lr.uoff.get(), nullptr, 0, Lc.om.get() + int64_t(c0) * Mr, Mr, nullptr, 0,
                            Pc.om.get() + int64_t(c0) * PMr, PMr, nc, Lr.max_k));
  }

  void in_rows(Level& L, const Level* C, int t, int D) {
    h2_matrix& h = *h_;
    L.processed = true;
    if (t == D) {
      L.rowoff_h = h.leafoff_h;
    } else {
      L.rowoff_h.resize(L.nn + 1);
      for (int i = 0; i <= L.nn; ++i) L.rowoff_h[i] = C->koff_h[2 * i];
      L.M = C->koff_h.back();
    }
    L.max_m = 0;
    for (int i = 0; i < L.nn; ++i) L.max_m = std::max(L.max_m, L.rowoff_h[i + 1] - L.rowoff_h[i]);
    L.rowoff.upload(L.rowoff_h, s_);
  }

  void identify(Level& L) {
    h2_matrix& h = *h_;
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
    L.J.alloc(size_t(L.joff_h.back()), s_);
    L.U.alloc(size_t(L.uoff_h.back()), s_);
    DevArray<int32_t> kdev;
    kdev.alloc(L.nn, s_);
    const size_t cbytes = size_t(3) * L.max_m * sizeof(double) + size_t(d_ | 1) * L.max_m * sizeof(double);
    if (cbytes > ctx_->lds_limit) ws_.ensure(L.nn, L.max_m, d_, s_);
    H2_HIP(h2dev::cpqr_id(s_, L.nn, L.rowoff.get(), L.y.get(), L.M, d_, h.delta, kdev.get(), L.J.get(),
                          L.joff.get(), L.U.get(), L.uoff.get(), L.max_m, ctx_->lds_limit, ws_.buf.get(),
                          ws_.off.get()));
    L.k_h = download(kdev.get(), L.nn, s_);
    L.koff_h = prefix(L.k_h);
    L.koff.upload(L.koff_h, s_);
    L.max_k = 0;
    for (int k : L.k_h) L.max_k = std::max(L.max_k, k);
  }

  void level(int t) {
    h2_matrix& h = *h_;
    const h2::Plan& p = h.plan;
    const int D = p.depth;
    Level& Lr = h.lv[t];
    Level& Lc = h.lvc[t];
    in_rows(Lr, t < D ? &h.lv[t + 1] : nullptr, t, D);
    in_rows(Lc, t < D ? &h.lvc[t + 1] : nullptr, t, D);

    int ph = timer_.begin(kSubtract);
    subtract(t, 0, dsk_);
    timer_.end(ph);

    // adaptive sampling: both sides share d; the counts d_, d_ + d_inc, ...
    // are tested together on every sketched column (prefix test)
    const int inc = h.opts.d_inc;
    while (true) {
      ph = timer_.begin(kConv);
      const int dconv = conv_.first_converged(s_, {&Lr, &Lc}, d_, dsk_, ws_);
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

    // IDs of both sides
    ph = timer_.begin(kId);
    identify(Lr);
    identify(Lc);
    timer_.end(ph);

    ph = timer_.begin(kUpsweep);
    if (t > h.top) {
      Level& Pr = h.lv[t - 1];
      Level& Pc = h.lvc[t - 1];
      Pr.M = Lr.koff_h.back();
      Pc.M = Lc.koff_h.back();
      Pr.y.alloc(size_t(Pr.M) * dcap_, s_);
      Pr.om.alloc(size_t(Pc.M) * dcap_, s_);
      Pc.y.alloc(size_t(Pc.M) * dcap_, s_);
      Pc.om.alloc(size_t(Pr.M) * dcap_, s_);
      upsweep(t, 0, dsk_);
    }
    // skeleton tree positions and rows of H's bases at them
    const Level& Ho = old_.lv[t];
    maxko_[t] = Ho.max_k;
    for (int a = 0; a < 2; ++a) {
      Level& L = a == 0 ? Lr : Lc;
      std::vector<DevArray<double>>& R = a == 0 ? Rr_ : Rc_;
      const int64_t Mn = L.koff_h.back();
      L.pos_out.alloc(size_t(Mn), s_);
      const int32_t* pos_in = t == D ? nullptr : (a == 0 ? h.lv : h.lvc)[t + 1].pos_out.get();
      H2_HIP(h2dev::skeleton(s_, L.nn, L.rowoff.get(), L.koff.get(), L.J.get(), L.joff.get(), pos_in,
                             L.pos_out.get(), 0, nullptr, 0, nullptr, 0));
      R[t].alloc(size_t(std::max<int64_t>(Mn, 1)) * std::max(Ho.max_k, 1), s_);
      const Level* Ct = t == D ? nullptr : &(a == 0 ? h.lv : h.lvc)[t + 1];
      H2_HIP(h2dev::basis_rows(s_, L.nn, t == D, L.koff.get(), L.J.get(), L.joff.get(), Ho.koff.get(),
                               t == D ? nullptr : old_.lv[t + 1].koff.get(), h.leafoff.get(), Ho.U.get(),
                               Ho.uoff.get(), Ct ? Ct->koff.get() : nullptr, t == D ? nullptr : R[t + 1].get(),
                               t == D ? 0 : std::max<int64_t>(Ct->koff_h.back(), 1), R[t].get(),
                               std::max<int64_t>(Mn, 1)));
    }
    if (t < D) {
      Rr_[t + 1].release();
      Rc_[t + 1].release();
    }
    timer_.end(ph);

    // couplings B_new(s, b) = A(I~r_s, I~c_b) from H's format plus U V^T
    ph = timer_.begin(kCoupling);
    Lr.fptr_h = p.far_ptr[t];
    Lr.fidx_h = p.far_idx[t];
    std::vector<int64_t> bsz(Lr.fidx_h.size());
    for (int a = 0; a < Lr.nn; ++a)
      for (int j = Lr.fptr_h[a]; j < Lr.fptr_h[a + 1]; ++j) bsz[j] = int64_t(Lr.k_h[a]) * Lc.k_h[Lr.fidx_h[j]];
    Lr.boff_h = prefix(bsz);
    Lr.fptr.upload(Lr.fptr_h, s_);
    Lr.forder.upload(bsr_order(Lr.fptr_h), s_);
    Lr.fidx.upload(Lr.fidx_h, s_);
    Lr.boff.upload(Lr.boff_h, s_);
    Lr.B.alloc(size_t(Lr.boff_h.back()), s_);
    // the column-side level carries the same lists (export and matvec read the row side's)
    Lc.fptr_h = Lr.fptr_h;
    Lc.fidx_h = Lr.fidx_h;
    std::vector<int32_t> frow(Lr.fidx_h.size());
    for (int a = 0; a < Lr.nn; ++a)
      for (int j = Lr.fptr_h[a]; j < Lr.fptr_h[a + 1]; ++j) frow[j] = a;
    DevArray<int32_t> frow_d;
    frow_d.upload(frow, s_);
    // rows of U and V at the new skeletons, gathered once for every pair of the level
    const int64_t Mr = std::max<int64_t>(Lr.koff_h.back(), 1), Mc = std::max<int64_t>(Lc.koff_h.back(), 1);
    DevArray<double> Ug, Vg;
    if (r_ > 0) {
      Ug.alloc(size_t(Mr) * r_, s_);
      Vg.alloc(size_t(Mc) * r_, s_);
      H2_HIP(h2dev::permute_rows(s_, Lr.koff_h.back(), Lr.pos_out.get(), false, h.lrU.get(), h.plan.n, Ug.get(), Mr,
                                 r_));
      H2_HIP(h2dev::permute_rows(s_, Lc.koff_h.back(), Lc.pos_out.get(), false, h.lrV.get(), h.plan.n, Vg.get(), Mc,
                                 r_));
    }
    H2_HIP(h2dev::coupling_update(s_, static_cast<int>(frow.size()), frow_d.get(), Lr.fidx.get(), Lr.koff.get(),
                                  Lc.koff.get(), Ho.koff.get(), Ho.max_k, Ho.B.get(), Ho.boff.get(), Rr_[t].get(), Mr,
                                  Rc_[t].get(), Mc, Ug.get(), Mr, Vg.get(), Mc, r_, Lr.B.get(), Lr.boff.get()));
    timer_.end(ph);
    if (t == h.top) {
      Rr_[t].release();
      Rc_[t].release();
    }
  }
};

void check_update_opts(const h2_opts* o) {
  H2_REQUIRE(o != nullptr, "opts is NULL");
  H2_REQUIRE(o->tol > 0.0 && std::isfinite(o->tol), "tol must be finite and > 0");
  H2_REQUIRE(o->d0 >= 1 && o->d0 <= 256, "d0 must be in [1, 256]");
  H2_REQUIRE(o->d_inc >= 1 && o->d_inc <= 128, "d_inc must be in [1, 128]");
  H2_REQUIRE(o->d_max >= o->d0 && o->d_max <= 256, "d_max must be in [d0, 256]");
  H2_REQUIRE(o->norm_mode == H2_NORM_FRO_SCALED || o->norm_mode == H2_NORM_LITERAL, "unknown norm_mode");
  H2_REQUIRE(o->sketch_ahead >= 0 && o->sketch_ahead <= 256, "sketch_ahead must be in [0, 256]");
  H2_REQUIRE(o->oversample >= 0 && o->oversample <= 64, "oversample must be in [0, 64]");
  if (o->precision != H2_FP64) throw Error(H2_ERR_UNSUPPORTED, "updates are built in FP64 only");
}

}  // namespace

extern "C" h2_status h2_build_update(h2_ctx* ctx, h2_matrix* old, int32_t rank, const double* U, int64_t ldu,
                                     const double* V, int64_t ldv, const h2_opts* opts, h2_matrix** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    H2_REQUIRE(ctx != nullptr && old != nullptr && out != nullptr, "NULL argument");
    check_update_opts(opts);
    H2_REQUIRE(rank >= 0 && rank <= 128, "rank must be in [0, 128]");
    const int64_t n = old->plan.n;
    H2_REQUIRE(rank == 0 || (U != nullptr && V != nullptr), "U or V is NULL");
    H2_REQUIRE(rank == 0 || (ldu >= n && ldv >= n), "ld < n");
    if (old->two_sided() || old->lr_rank > 0)
      throw Error(H2_ERR_UNSUPPORTED, "the matrix to update must be a symmetric build (h2_build or h2_build_batched)");
    for (const Level& L : old->lv)
      if (L.processed && L.max_k > 128) throw Error(H2_ERR_UNSUPPORTED, "ranks of the matrix to update exceed 128");
    H2_HIP(hipSetDevice(ctx->device));
    // the dense blocks become shared between the two matrices
    if (!old->keep_d && !old->keep) {
      auto holder = std::make_shared<DevArray<double>>(std::move(old->Dblk));
      old->Dblk.borrow(holder->get(), holder->size());
      old->keep_d = holder;
    }
    auto h = std::make_unique<h2_matrix>();
    h->device = ctx->device;
    h->stream = ctx->stream;
    h->plan = old->plan;
    h->kernel = old->kernel;
    h->opts = *opts;
    h->opts.leaf_size = old->opts.leaf_size;
    h->opts.eta = old->opts.eta;
    h->keep = old->keep;
    h->keep_d = old->keep_d;
    h->keep_small = old->small ? old->small : old->keep_small;
    h->Dblk.borrow(old->Dblk.get(), old->Dblk.size());
    UpdateBuilder b(ctx, *old, h.get(), rank);
    b.run(U, ldu, V, ldv);
    *out = h.release();
  });
}
