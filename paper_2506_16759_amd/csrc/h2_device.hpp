// Launchers of the gfx950 kernels behind the C ABI.  All sizes are element
// counts; all matrices are column-major float64 with explicit leading
// dimensions; every launcher enqueues on `s` and returns hipSuccess or the
// launch error.
//
// Row spaces.  The construction works level by level (Alg. 1).  The rows of
// the sample matrices at depth t form a "row space" R_t: at the leaf depth it
// is the n points in tree order; at an inner depth it is the concatenation of
// the skeleton rows of the depth t+1 clusters, cluster by cluster.  A cluster
// i at depth t owns rows [rowoff[i], rowoff[i+1]) of R_t, and its skeleton
// (after its ID) owns rows [koff[i], koff[i+1]) of R_{t-1}.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2dev {

enum KernelKind : int { kExp = 1, kGauss = 2, kHelm = 3 };

struct KernelFn {
  int kind;      // KernelKind
  double scale;  // exp: 1/l (kappa = exp(-r*scale)); gauss: 1/(2 l^2) (kappa = exp(-r^2*scale));
                 // helm: the wavenumber k (kappa = cos(k r)/r, 0 at r = 0)
};

// Omega(rows[p], col0 + c) -> out[p + c*ldo]; counter-based Philox4x64-10 + Box-Muller.
// rows == nullptr means row p is original index p.
hipError_t gaussian(hipStream_t s, uint64_t seed, int64_t nrows, const int32_t* rows, int64_t col0, int ncols,
                    double* out, int64_t ldo);

// Dense on-the-fly sketch y = K(X,X) omega, X = (dim x n) SoA with leading
// dimension ldx; precision is an h2_precision value (0 FP64, 1 FP32, 2
// BF16X3, 3 FP32E, 4 BF16X6, 5 FP64 with symmetric-tile reuse).  Mixed modes
// fold FP32 partial sums into FP64 every 64 points; y is always FP64.  The
// split-bf16 modes take stream-ordered scratch (hipMallocAsync); mode 5 uses
// sym_scratch (sketch_sym_scratch_bytes(n) bytes, stream-ordered on s) when
// given, else allocates it likewise.
hipError_t sketch(hipStream_t s, int precision, int64_t n, int dim, const double* X, int64_t ldx, KernelFn k,
                  int ncols, const double* omega, int64_t ldo, double* y, int64_t ldy,
                  double* sym_scratch = nullptr);

// Device scratch of one symmetric-tile sketch call (precision 5):
// 512 * sum over tiles a of max(0, n - 128 (a + 1)) bytes, about 2 n^2.
size_t sketch_sym_scratch_bytes(int64_t n);

// Kernel blocks of a CSR block pattern: for block row i and entry j in [ptr[i], ptr[i+1]) with
// b = idx[j], writes kappa(X[rowoff[i] + r], X[rowoff[b] + c]) to out[blkoff[j] + r + c*m_i].
hipError_t gen_blocks(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                      const int64_t* blkoff, int dim, const double* X, int64_t ldx, KernelFn k, double* out);

// Block-sparse product Y[rows_i, :] += alpha * sum_j Blk_j X[rows_b, :] over nc
// columns, on the FP64 matrix cores.  max_m bounds every block-row height.
// X (ldx rows, column-major) is first copied row-major into `scratch`, which
// must hold bsr_scratch_doubles(ldx, nc, tile_cols) doubles (else
// hipErrorInvalidValue).  tile_cols (16, 32, 48 or 64) is the column-tile width
// of one workgroup: the columns are covered by ceil(nc / tile_cols) tiles, each
// reading the blocks once; the sums are the same bit for bit for every width.
// order (optional, device): the block rows in launch order, a permutation of
// [0, nrows) (bsr_order: longest rows first); results do not depend on it.
size_t bsr_scratch_doubles(int64_t ldx, int nc, int tile_cols = 64);
hipError_t bsr_gemm(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                    const int64_t* blkoff, const double* blocks, const double* X, int64_t ldx, double* Y,
                    int64_t ldy, int nc, double alpha, int max_m, double* scratch, size_t scratch_doubles,
                    int tile_cols = 64, const int32_t* order = nullptr);

// Two-sided form: block row i has rows [rowoff[i], rowoff[i+1]) of Y, block
// column b rows [coloff[b], coloff[b+1]) of X; with tpos != nullptr the block of
// entry j is the transpose of stored block tpos[j] (which is stored
// (coloff height) x (rowoff height), column-major).  max_m bounds the row heights.
hipError_t bsr_gemm2(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                     const int32_t* coloff, const int64_t* tpos, const int64_t* blkoff, const double* blocks,
                     const double* X, int64_t ldx, double* Y, int64_t ldy, int nc, double alpha, int max_m,
                     double* scratch, size_t scratch_doubles, int tile_cols = 64, const int32_t* order = nullptr);

// Row ID per cluster via column-pivoted QR of A = Y_loc^T (d x m): k[i], J (pivot order, local
// row numbers, at joff[i]), U (m x k column-major at uoff[i], identity on rows J).
// Batched use: nodeprob[i] names cluster i's problem, whose column count and
// threshold are dprob[.] and deltaprob[.] (then d and delta are ignored).
hipError_t cpqr_id(hipStream_t s, int nnodes, const int32_t* rowoff, const double* Y, int64_t ldy, int d,
                   double delta, int32_t* kout, int32_t* J, const int64_t* joff, double* U, const int64_t* uoff,
                   int max_m, size_t lds_limit, double* gws, const int64_t* gws_off,
                   const int32_t* nodeprob = nullptr, const int32_t* dprob = nullptr,
                   const double* deltaprob = nullptr);

// Shrink and upsweep (Alg. 1 batchedShrink + batchedGemm) on nc columns:
//   Yout[koff[i] + r, :] = Yloc[rowoff[i] + J[r], :]           (skipped when Yloc == nullptr)
//   Wout[koff[i] + r, :] = sum_q U[q, r] Win[rowoff[i] + q, :]    (skipped when Win == nullptr)
// kmax bounds every node's k (at most 256, else hipErrorInvalidValue).
hipError_t shrink_up(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const int32_t* J,
                     const int64_t* joff, const double* U, const int64_t* uoff, const double* Yloc, int64_t ldyl,
                     const double* Win, int64_t ldwi, double* Yout, int64_t ldyo, double* Wout, int64_t ldwo,
                     int nc, int kmax = 256);

// Downsweep of the matvec: Yt[rowoff[i] + q, :] += sum_r U[q, r] Yh[koff[i] + r, :].
hipError_t expand(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const double* U,
                  const int64_t* uoff, const double* Yh, int64_t ldh, double* Yt, int64_t ldt, int nc);

// Skeleton rows: pos_out[koff[i] + r] = pos_in[rowoff[i] + J[r]] (or rowoff[i] + J[r] when
// pos_in == nullptr); Xs[a*ldxs + q] = X[a*ldx + pos_out[q]].
hipError_t skeleton(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const int32_t* J,
                    const int64_t* joff, const int32_t* pos_in, int32_t* pos_out, int dim, const double* X,
                    int64_t ldx, double* Xs, int64_t ldxs);

// dst[p + c*ldd] = src[idx[p] + c*lds] (gather, scatter = false) or dst[idx[p] + c*ldd] = src[p + c*lds];
// nc <= 65535 (else hipErrorInvalidValue).
hipError_t permute_rows(hipStream_t s, int64_t n, const int32_t* idx, bool scatter, const double* src, int64_t lds,
                        double* dst, int64_t ldd, int nc);

// Partial sums of squares of an (n x nc) block: partial[b] for b < nblocks (fixed, deterministic).
hipError_t sumsq_partial(hipStream_t s, int64_t n, int nc, const double* A, int64_t lda, double* partial,
                         int nblocks);

// Sets the dynamic-LDS limit of every kernel that can use more than 64 KB
// (call once per device before launching or capturing).
hipError_t prepare_kernels(size_t lds_limit);

// Fill n doubles with zero (used instead of memset so the call is graph-capturable).
hipError_t fill_zero(hipStream_t s, double* p, int64_t n);
hipError_t fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);

// ------------------------------------------------------------------ batched
// Several independent problems share concatenated arrays: problem p owns
// global rows [base_p, base_p + n_p) of the points (3 coordinates, unused
// ones zero), of Omega and of Y; its clusters of a level are contiguous in
// that level's node list.

// Omega(rows[p], col0 + c) with the seed of problem rowprob[p].
hipError_t gaussian_batched(hipStream_t s, int64_t nrows, const int32_t* rows, const int32_t* rowprob,
                            const uint64_t* seeds, int64_t col0, int ncols, double* out, int64_t ldo);

// y = K_p omega for every problem: workgroup b computes row tile tiles[2b+1]
// (a multiple of 128) of problem tiles[2b].  jobs: device array of packed jobs.
// The columns go through launches of at most chunk_cols (16, 32, 48 or 64)
// columns each; every launch evaluates all kernel entries once, and each
// column's sum is the same bit for bit for every chunk width.
hipError_t sketch_batched(hipStream_t s, int precision, int ntiles, const void* jobs, const int32_t* tiles,
                          const double* X, int64_t ldx, int ncols, const double* omega, int64_t ldo, double* y,
                          int64_t ldy, int chunk_cols = 64);
size_t sketch_job_bytes();
void pack_sketch_job(void* dst, int64_t n, int64_t base, int kind, double scale);

// gen_blocks with per-block-row problem: kind kinds[rowprob[i]], exponent c2s[rowprob[i]]
// (c2 = -scale * log2 e); X has 3 coordinate rows.
hipError_t gen_blocks_batched(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                              const int64_t* blkoff, const double* X, int64_t ldx, const int32_t* rowprob,
                              const int32_t* kinds, const double* c2s, double* out);

// Adaptive convergence test (Sec. III-B) over all dsk sketched columns, with
// an oversampling margin: a cluster of m rows is converged at count d if
// m + ovprob[p] <= d or min |R_jj| < delta over j < d - ovprob[p] (unpivoted
// Householder QR of its samples).  Raises dprob[p] to the first count on the
// grid dprob[p] + j*incprob[p] at which every cluster of problem p is
// converged; sets exhausted[p] if some cluster is not converged within dsk.
// Panels larger than lds_limit bytes use gws.
hipError_t qr_first_conv(hipStream_t s, int nnodes, const int32_t* rowoff, const double* Y, int64_t ldy, int dsk,
                         const int32_t* incprob, const int32_t* ovprob, const int32_t* nodeprob, int32_t* dprob,
                         const double* deltaprob, int32_t* exhausted, int max_m, size_t lds_limit, double* gws,
                         const int64_t* gws_off);

// dst[i] = src[map[i]] for i < n (index gather, e.g. original indices of skeleton positions).
hipError_t gather_idx(hipStream_t s, int64_t n, const int32_t* map, const int32_t* src, int32_t* dst);

// Exclusive scan: out[i] = sum_{j<i} in[j], out[n] = total.
hipError_t scan_i32(hipStream_t s, int n, const int32_t* in, int32_t* out);
// dst[i] = src[map[i]], i = 0..n.
hipError_t gather_i32(hipStream_t s, int n, const int32_t* map, const int32_t* src, int32_t* dst);

// Per problem: nu = ||Y_p(:, 0:d0)||_F / sqrt(d0), delta from tol and mode, d = d0.
size_t threshold_job_bytes();
void pack_threshold_job(void* dst, int64_t base, int64_t n, int d0, int nleaves, int mode, double tol);
hipError_t thresholds(hipStream_t s, int nprob, const void* jobs, const double* Y, int64_t ldy, double* nu,
                      double* delta, int32_t* d);

// ------------------------------------------------------- low-rank update
// A = H + U V^T with U, V (n x r, column-major, tree order).

// W_b = V(leaf b rows, :)^T X(leaf b rows, :) for every leaf b: r x nc blocks,
// column-major with ld r, block b at W + b*r*nc; nc <= 64 (else hipErrorInvalidValue).
hipError_t lr_leaf_project(hipStream_t s, int nleaves, const int32_t* leafoff, const double* V, int64_t ldv, int r,
                           const double* X, int64_t ldx, int nc, double* W);
// out (len) = sum_b W_b in a fixed order; partial holds lr_sum_scratch doubles.
size_t lr_sum_scratch(int nleaves, int len);
hipError_t lr_sum(hipStream_t s, int nleaves, int len, const double* W, double* partial, double* out);
// Y(leaf s rows, :) += alpha U(leaf s rows, :) sum_{b in ptr/idx row s} W_b   (ptr != nullptr), or
// Y(0..n, :) += alpha U W                                                 (ptr == nullptr).
// Requires r * nc <= 8192.
hipError_t lr_apply(hipStream_t s, int nleaves, const int32_t* ptr, const int32_t* idx, const int32_t* leafoff,
                    int64_t n, const double* U, int64_t ldu, int r, const double* W, int nc, double* Y, int64_t ldy,
                    double alpha);
// Rows of the old nested basis at the new skeletons (see the kernel's comment).
hipError_t basis_rows(hipStream_t s, int nnodes, bool leaf, const int32_t* koff, const int32_t* J,
                      const int64_t* joff, const int32_t* kold_off, const int32_t* kold_child_off,
                      const int32_t* leafoff, const double* Uold, const int64_t* uoff_old, const int32_t* koff_child,
                      const double* Rc, int64_t ldrc, double* R, int64_t ldr);
// B_new(s, b) = R_r_s B_old(s, b) R_c_b^T + Ug_s Vg_b^T for every far pair j (row
// frow[j], column cluster fidx[j]), where Ug (ld ldug) and Vg (ld ldvg) hold the rows
// of U and V at the level's row and column skeletons, in skeleton order (rows koff_r
// and koff_c).  Old ranks must be <= 128.
hipError_t coupling_update(hipStream_t s, int npairs, const int32_t* frow, const int32_t* fidx,
                           const int32_t* koff_r, const int32_t* koff_c, const int32_t* kold_off, int max_kold,
                           const double* Bold, const int64_t* boff_old, const double* Rr, int64_t ldrr,
                           const double* Rc, int64_t ldrc, const double* Ug, int64_t ldug, const double* Vg,
                           int64_t ldvg, int r, double* Bnew, const int64_t* boff_new);
// out_j = D_j + U(rows s) V(rows b)^T for the near blocks (explicit dense blocks of an update).
hipError_t dense_lowrank(hipStream_t s, int nleaves, const int32_t* ptr, const int32_t* idx,
                         const int32_t* leafoff, const int64_t* blkoff, const double* Din, const double* U,
                         int64_t ldu, const double* V, int64_t ldv, int r, double* out);

}  // namespace h2dev
