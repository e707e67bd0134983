/*
 * h2.h -- C ABI of the MI355X (gfx950) H^2 construction library.
 *
 * Builds an H^2 matrix of a symmetric operator on a point cloud (a kernel
 * matrix K(x_i, x_j), or any matrix given by a black-box product and an entry
 * evaluator) with the bottom-up adaptive-sketching construction of
 * "Adaptive Sketching Based Construction of H2 Matrices on GPUs"
 * (Boukaram, Liu, Ghysels, Li; arXiv 2506.16759), Algorithm 1 with the
 * adaptive sampling of Sec. III-B.
 *
 * Conventions shared by every call
 *   - Every function returns an h2_status (0 = H2_OK, negative = error) and
 *     never throws.  On error, output handles are set to NULL, nothing is
 *     leaked, and h2_last_error() returns a thread-local message.
 *   - Points are structure-of-arrays float64: a (dim x n) row-major array,
 *     coordinate a of point i at points[a*n + i]; 1 <= dim <= 3, n < 2^31.
 *   - Dense vectors/matrices are column-major float64 with a leading
 *     dimension argument (ld >= rows).  "Original order" means the caller's
 *     point order.
 *   - Device pointers must be allocations on the context's device; host
 *     pointers are plain host memory.  The library never frees caller memory.
 *   - Calls that take an h2_ctx enqueue on the context's stream.  h2_build is
 *     synchronous (it returns after the build completed); h2_matvec,
 *     h2_entries, h2_sketch and h2_gaussian are stream-ordered (synchronise
 *     the stream before reading results on the host).
 *   - One context per host thread; a context's calls must not overlap.
 */
#ifndef H2_H
#define H2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = -1,       /* invalid argument (NULL, size, ld, option out of range) */
  H2_ERR_HIP = -2,       /* a HIP runtime call failed */
  H2_ERR_OOM = -3,       /* device allocation failed */
  H2_ERR_CALLBACK = -4,  /* a user callback (h2_sketch_fn, h2_entry_fn) returned non-zero */
  H2_ERR_SAMPLES = -5,   /* adaptive sampling reached d_max unconverged */
  H2_ERR_STATE = -6,     /* object in the wrong state (e.g. export of a missing part) */
  H2_ERR_UNSUPPORTED = -7 /* request outside what this build implements */
} h2_status;

/* Kernel functions kappa(r), r = |x - y| (Sec. V-A, the two test problems). */
typedef enum {
  H2_K_EXP = 1,       /* exponential covariance exp(-r / length), eq. (cov); kappa(0) = 1 */
  H2_K_GAUSS = 2,     /* Gaussian covariance exp(-r^2 / (2 length^2)); kappa(0) = 1 */
  H2_K_HELMHOLTZ = 3  /* volume-IE operator of the Helmholtz equation cos(k r) / r, eq. (ie),
                       * k = wavenumber.  The formula holds for x != y only; the diagonal
                       * (and any pair of coincident points, r == 0) is taken as 0.
                       * FP64 single builds only (other precisions and batched builds
                       * return H2_ERR_UNSUPPORTED). */
} h2_kernel_kind;

typedef struct {
  int32_t kind;       /* h2_kernel_kind */
  double length;      /* correlation length l > 0 (H2_K_EXP, H2_K_GAUSS; ignored otherwise) */
  double wavenumber;  /* k > 0 (H2_K_HELMHOLTZ; ignored otherwise) */
} h2_kernel;

/* ------------------------------------------------------- black-box inputs
 * Alg. 1 takes the matrix through two user functions: the black box
 * Y = K_blk(Omega) and a batched evaluator of sub-blocks (batchedGen, Sec.
 * IV-A).  Both are called from the thread running h2_build, in stream order:
 * they enqueue their device work on `stream` (a hipStream_t passed as void*,
 * the context's stream) and return 0, or non-zero on failure, which aborts the
 * build with H2_ERR_CALLBACK (nothing leaks).  They may call h2_matvec and
 * h2_entries, on the building context or another one, and must not free or
 * write memory the library passes them except their output.  The operator
 * must be symmetric (the symmetric form of Alg. 1); an operator given by an
 * H^2 matrix plus a low-rank product, which is not, is built by
 * h2_build_update.
 *
 * Sketch callback: y(:, c) = A omega(:, c) for c < d.  omega: DEVICE n x d
 * (ld ldo), y: DEVICE n x d (ld ldy, overwritten), both in ORIGINAL point
 * order.  Called once per sketch pass (h2_info.sketch_calls). */
typedef int (*h2_sketch_fn)(void* user, int64_t n, int32_t d, const double* omega, int64_t ldo, double* y,
                            int64_t ldy, void* stream);

/* Entry callback (batchedGen): for every block b < nblocks,
 *   out[off[b] + r + c * rcnt[b]] = A(idx[rbeg[b] + r], idx[cbeg[b] + c]),
 *   r < rcnt[b], c < ccnt[b]  (block b column-major, leading dimension rcnt[b]),
 * with idx holding ORIGINAL point indices.  idx, rbeg, rcnt, cbeg, ccnt, off
 * and out are DEVICE arrays; max_rows and max_cols bound rcnt[] and ccnt[]
 * (host values, for launch shapes).  The library calls it for the dense leaf
 * blocks D (nblocks = near pairs) and, per level, for the coupling blocks B at
 * the skeletons (nblocks = far pairs of the level). */
typedef int (*h2_entry_fn)(void* user, int32_t nblocks, const int32_t* idx, const int64_t* rbeg,
                           const int32_t* rcnt, const int64_t* cbeg, const int32_t* ccnt, const int64_t* off,
                           double* out, int32_t max_rows, int32_t max_cols, void* stream);

/* Arithmetic of the dense on-the-fly sketch.  Kernel blocks D and B are
 * always evaluated and stored in FP64 and multiplied on the FP64 matrix cores
 * (the leaf near-field product is bound by block traffic and latency, so an
 * FP32 form gains nothing); the stopping test, CPQR and interpolation solve
 * are FP64.  In the reduced modes an entry is evaluated from the FP64 squared
 * distance with the FP32 square root and exponential (~1e-7 relative error).
 *   H2_FP64:   FP64 entries, FP64 matrix cores.
 *   H2_FP32:   FP32 entries and Omega, FP32 matrix cores; the FP32 partial
 *              sums are folded into FP64 every 64 points, which keeps their
 *              rounding below the entry error (same sample counts as FP64 at
 *              tol 1e-6 on the 131072-point covariance matrix).
 *   H2_BF16X3: FP32 entries and Omega split into round-to-nearest bf16
 *              hi + lo, three bf16 products (hi*hi + hi*lo + lo*hi) with FP32
 *              accumulation, folded into FP64 likewise; about 2^-17 relative
 *              error per product (tol >= ~1e-4).
 *   H2_FP32E:  FP32 entries converted to FP64 and contracted with the FP64
 *              Omega on the FP64 matrix cores with FP64 accumulation.
 *   H2_BF16X6: FP32 entries and Omega each split into three round-to-nearest
 *              bf16 terms; the six products whose split orders add up to at
 *              most 2 run on the bf16 matrix cores with FP32 accumulation,
 *              folded into FP64 every 64 points: FP32-accurate products at a
 *              fraction of the FP32 matrix-core cycles. */
typedef enum { H2_FP64 = 0, H2_FP32 = 1, H2_BF16X3 = 2, H2_FP32E = 3, H2_BF16X6 = 4, H2_FP64_SYM = 5 } h2_precision;
/*   H2_FP64_SYM: FP64 entries and matrix cores as H2_FP64, with the symmetry
 *              of K used in the sketch: the entries of each pair of 128-point
 *              tiles (a, b), a < b, are evaluated once and contracted with
 *              both Omega(I_b) (for Y(I_a)) and Omega(I_a) (for Y(I_b)).  The
 *              transposed products pass through device scratch that each
 *              sketch call allocates and frees in stream order:
 *              512 * sum_a max(0, n - 128 (a + 1)) bytes, about 2 n^2 (34 GB at
 *              n = 131072), so n <= 163840.  Results equal H2_FP64's to
 *              rounding (another summation order).  h2_sketch and single
 *              builds with a built-in kernel only. */

/* How the absolute ID/stopping threshold delta is derived from tol
 * (Sec. III-B: "an approximate norm of the matrix ... via sketching"):
 *   nu = ||Y_0||_F / sqrt(d0)  (unbiased estimate of ||K||_F)
 *   H2_NORM_FRO_SCALED: delta = tol * nu / sqrt(#leaves)
 *   H2_NORM_LITERAL:    delta = tol * nu                                    */
typedef enum { H2_NORM_FRO_SCALED = 0, H2_NORM_LITERAL = 1 } h2_norm_mode;

typedef struct {
  double tol;         /* relative compression tolerance epsilon, > 0 (Alg. 1 input) */
  int32_t leaf_size;  /* KD-tree leaf size m0, 2..256 */
  double eta;         /* general admissibility parameter (Sec. II-A), > 0 */
  int32_t d0;         /* initial sample columns (Alg. 1 "sample block size"), 1..256 */
  int32_t d_inc;      /* columns added per adaptive round (Sec. III-B), 1..128; 0 = fixed
                       * sample size (Sec. III-A): exactly d0 columns, no convergence test
                       * and no adaptive rounds (single builds only) */
  int32_t d_max;      /* cap on total columns, <= 256; exceeding it -> H2_ERR_SAMPLES */
  uint64_t seed;      /* key of the counter-based Gaussian test matrix */
  int32_t precision;  /* h2_precision */
  int32_t norm_mode;  /* h2_norm_mode */
  int32_t sketch_ahead; /* extra columns sketched whenever a sketch pass runs (0..256).  The
                         * adaptive loop still grows d by d_inc; columns already sketched
                         * are used without another pass.  Results are identical for any
                         * value (Omega is counter-based); only the number of passes over
                         * the O(n^2) black box changes. */
  int32_t oversample;   /* p, 0..64: the convergence test looks at the leading d - p sample
                         * columns only (a cluster with m + p <= d is converged), so the ID
                         * always has p samples beyond the rank it detects (Sec. III-A's
                         * oversampling).  p = 0 is the bare test of Sec. III-B, enough for
                         * kernel matrices (fast singular-value decay); operators with flat
                         * spectra such as low-rank updates need p >= 4: with p = 0 the
                         * nearly square sketch of a full-rank block shows a spuriously
                         * small trailing diagonal and the block is truncated. */
} h2_opts;

typedef struct h2_ctx h2_ctx;
typedef struct h2_matrix h2_matrix;
typedef struct h2_plan h2_plan;

/* Fills defaults: tol 1e-6, leaf 64, eta 0.7, d0 32, d_inc 16, d_max 256,
 * seed 1000, FP64, FRO_SCALED, sketch_ahead 32, oversample 0. */
h2_status h2_opts_default(h2_opts* opts);

const char* h2_status_string(h2_status s);
const char* h2_last_error(void);

/* ---------------------------------------------------------------- context */

/* Creates a context bound to HIP device `device` and stream `stream`
 * (a hipStream_t passed as void*; NULL = the default stream).  The stream is
 * borrowed and must outlive the context. */
h2_status h2_ctx_create(int device, void* stream, h2_ctx** out);
h2_status h2_ctx_destroy(h2_ctx* ctx);

/* ------------------------------------------------ host-only cluster plan */

/* Cluster tree and interaction lists of Sec. II-A, computed on the host with
 * no GPU involved (the same code h2_build runs).  KD bisection with tight
 * boxes, widest axis (lowest on ties), stable median by (coordinate, original
 * index), left child floor(n/2); leaves all at depth D = min{d : ceil(n/2^d)
 * <= leaf_size}; general admissibility (D(s)+D(t))/2 <= eta*Dist(s,t)
 * evaluated without square roots, touching boxes never admissible; dual-tree
 * traversal from (root, root).  points: HOST, (dim x n) SoA. */
h2_status h2_plan_create(int64_t n, int32_t dim, const double* points_host, int32_t leaf_size,
                         double eta, h2_plan** out);

/* The same plan built by device kernels (Sec. II-A's tree and dual-tree
 * traversal on the GPU): equal to h2_plan_create's bit for bit (permutation,
 * nodes, boxes, near and far lists).  Each node finds its split by radix
 * selection on (coordinate, original index) and partitions its points; the
 * last split sorts each node in LDS; each depth of the traversal tests every
 * cluster's candidate partners in one launch.  points: DEVICE, (dim x n)
 * SoA, original order, read on ctx's stream.  Errors as h2_plan_create
 * (non-finite coordinates: H2_ERR_ARG).  Synchronous. */
h2_status h2_plan_create_device(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, int32_t leaf_size,
                                double eta, h2_plan** out);
h2_status h2_plan_free(h2_plan* plan);

/* Parts exported by h2_plan_export and h2_export.  `depth` selects the tree
 * depth where a part is per depth; node indices inside a depth are local
 * (heap id - (2^depth - 1)). */
typedef enum {
  H2_PART_DEPTH = 0,     /* int32[1]: D */
  H2_PART_PERM = 1,      /* int32[n]: tree position -> original index */
  H2_PART_NODES = 2,     /* int32[2 * (2^(D+1)-1)]: [begin, end) per heap node */
  H2_PART_BOXES = 3,     /* float64[(2^(D+1)-1) * 2 * dim]: lo[dim], hi[dim] per node */
  H2_PART_NEAR_PTR = 4,  /* int32[2^D + 1]: CSR row pointers of N_tau (leaf depth) */
  H2_PART_NEAR_IDX = 5,  /* int32[nnz]: ascending local leaf indices */
  H2_PART_FAR_PTR = 6,   /* int32[2^depth + 1]: CSR of F_tau at `depth` */
  H2_PART_FAR_IDX = 7,   /* int32[nnz] */
  /* parts below exist only for built matrices (h2_export) */
  H2_PART_RANKS = 8,     /* int32[2^depth]: k_tau at `depth` (0 above the top depth) */
  H2_PART_SKEL = 9,      /* int32[sum k]: skeleton ORIGINAL indices, node by node */
  H2_PART_BASIS = 10,    /* float64: the ID matrix of every node at `depth`, node by node,
                            each m_tau x k_tau column-major (leaf: U_tau; inner: [E_nu1; E_nu2]) */
  H2_PART_COUPLING = 11, /* float64: B_{s,b} for the far pairs at `depth` in CSR order,
                            each k_s x k_b column-major */
  H2_PART_DENSE = 12,    /* float64: D_{s,b} for the near pairs in CSR order, each
                            m_s x m_b column-major (rows/cols in tree order) */
  H2_PART_TOP = 13,      /* int32[1]: coarsest processed depth */
  H2_PART_SKEL_POS = 14, /* int32[sum k]: skeleton tree positions, node by node */
  /* column side of a two-sided matrix (h2_build_update); for a symmetric
     matrix these equal RANKS, SKEL, BASIS and SKEL_POS.  COUPLING blocks of a
     two-sided matrix are k_s (row rank) x k_b (column rank). */
  H2_PART_RANKS_C = 15,
  H2_PART_SKEL_C = 16,
  H2_PART_BASIS_C = 17,
  H2_PART_SKEL_POS_C = 18
} h2_part;

/* Copies a part into host memory dst (dst_bytes large).  dst == NULL only
 * reports the size in *needed (bytes). */
h2_status h2_plan_export(const h2_plan* plan, int32_t part, int32_t depth, void* dst,
                         size_t dst_bytes, size_t* needed);

/* ------------------------------------------------------------ step calls */

/* Counter-based Gaussian test matrix of Alg. 1 (batchedRand):
 *   out[p + c*ldo] = Omega(rows[p], col0 + c), p < nrows, c < ncols,
 * with Omega(i, j) = sqrt(-2 ln u1) cos(2 pi u2), (u1, u2) from the first two
 * words of Philox4x64-10 (counter (i, j, 0, 0), key (seed, 0)) mapped to (0,1)
 * as (w >> 11) * 2^-53 + 2^-54.  rows: DEVICE int32 original indices; out:
 * DEVICE.  Stream-ordered. */
h2_status h2_gaussian(h2_ctx* ctx, uint64_t seed, int64_t nrows, const int32_t* rows, int64_t col0,
                      int32_t ncols, double* out, int64_t ldo);

/* Dense on-the-fly sketch Y = K(X, X) * Omega without storing K (the black box
 * Y = K_blk(Omega) of Alg. 1 for a kernel matrix): kernel tiles are generated
 * in registers and contracted with Omega on the matrix cores.
 * points: DEVICE (dim x n) SoA; omega: DEVICE n x ncols (ld ldo); y: DEVICE
 * n x ncols (ld ldy), overwritten.  ncols <= 128.  Stream-ordered. */
h2_status h2_sketch(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, const h2_kernel* kernel,
                    int32_t precision, int32_t ncols, const double* omega, int64_t ldo, double* y,
                    int64_t ldy);

/* ------------------------------------------------------------------ build */

/* Algorithm 1 + adaptive sampling (Sec. III): the H^2 matrix of a symmetric
 * n x n operator A on the cluster tree of `points` (DEVICE (dim x n) SoA,
 * borrowed for the call; they define the tree and admissibility of Sec. II-A).
 * Inputs of Alg. 1, in one of three forms:
 *   kernel != NULL, sketch == NULL: A = K(i, j) = kappa(|x_i - x_j|); the
 *       black box is the fused dense on-the-fly sketch (h2_sketch) and the
 *       blocks are evaluated from kappa;
 *   kernel != NULL, sketch != NULL: the black box is the callback (e.g. the
 *       product with an existing H^2 matrix, as in Sec. V-A) and the blocks
 *       are evaluated from kappa (entry == NULL);
 *   kernel == NULL: both callbacks (sketch and entry) define A.
 * opts->precision other than H2_FP64 applies to the built-in sketch only
 * (H2_ERR_UNSUPPORTED with a sketch callback).  Synchronous.  *out owns
 * every result until h2_free. */
h2_status h2_build(h2_ctx* ctx, int64_t n, int32_t dim, const double* points, const h2_kernel* kernel,
                   h2_sketch_fn sketch, void* sketch_user, h2_entry_fn entry, void* entry_user,
                   const h2_opts* opts, h2_matrix** out);

/* y = A_H x (trans = 0) or y = A_H^T x (trans = 1) for nrhs columns, x and y
 * DEVICE n x nrhs in ORIGINAL order (ld >= n), y overwritten.  Standard H^2
 * product (the format of Sec. II-A, Table I): upsweep through the column
 * bases, couplings, downsweep through the row bases, near field; the
 * transpose swaps the bases and applies B^T and D^T.  For a symmetric build
 * both are the same product.  Stream-ordered. */
h2_status h2_matvec(h2_ctx* ctx, const h2_matrix* h, int32_t trans, int32_t nrhs, const double* x, int64_t ldx,
                    double* y, int64_t ldy);

/* h2_matvec without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, layout and result as h2_matvec.  Its
 * temporaries (tree-ordered copies of x and y, x_hat and y_hat per depth, the
 * row-major staging copy of the block-sparse products, the leaf projection of
 * a low-rank term) live in a static device array of H2_NOALLOC_SCRATCH_BYTES
 * that every device the library runs on holds until the process ends; its
 * address is looked up when a context is created.  Columns are processed in
 * chunks of the widest width (<= 64) whose temporaries fit; a matrix whose
 * temporaries do not fit for one column (about 8 * (3 n + sum of ranks) bytes)
 * is rejected with H2_ERR_ARG and a message giving the bytes it needs.  The
 * array keeps the last call's contents, and every call on a device uses that
 * device's one array: calls that overlap on one device (other streams or
 * threads, other contexts) race and give wrong results.  Results equal
 * h2_matvec's up to the summation order of the chunked products.
 * Stream-ordered. */
#define H2_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
h2_status h2_matvec_noalloc(h2_ctx* ctx, const h2_matrix* h, int32_t trans, int32_t nrhs, const double* x,
                            int64_t ldx, double* y, int64_t ldy);

/* Entries of a built H^2 matrix from the definition of the format (Sec.
 * II-A, nested basis): entry (i, j) lies in exactly one block of the
 * partition, a dense leaf block D_{s,b} (plus U_s V_b^T for an update) or an
 * admissible pair (s, b) at some depth, where it equals
 * row_i(U_s) B_{s,b} row_j(V_b)^T with the nested bases expanded through the
 * transfer matrices.  Same block batch as h2_entry_fn (all arrays DEVICE,
 * original indices), so a built matrix can serve as the entry callback of
 * another build (Sec. IV-A batchedGen on an H^2 input).  The first call
 * expands every point's nested-basis rows once (8 bytes x n x the largest
 * rank of each processed depth, kept until h2_free).  Stream-ordered. */
h2_status h2_entries(h2_ctx* ctx, const h2_matrix* h, int32_t nblocks, const int32_t* idx, const int64_t* rbeg,
                     const int32_t* rcnt, const int64_t* cbeg, const int32_t* ccnt, const int64_t* off,
                     double* out, int32_t max_rows, int32_t max_cols);

/* Same parts as h2_plan_export plus the built factors (RANKS .. SKEL_POS).
 * on_device = 0: dst is HOST memory; 1: dst is DEVICE memory on the
 * matrix's device.  dst == NULL only reports the size in *needed (bytes).
 * Synchronises the matrix's stream before returning. */
h2_status h2_export(const h2_matrix* h, int32_t part, int32_t depth, int32_t on_device, void* dst,
                    size_t dst_bytes, size_t* needed);

typedef struct {
  int64_t n;
  int32_t dim, depth, top;     /* tree depth D, coarsest processed depth */
  int32_t samples;             /* sample columns used by the construction (d) */
  int32_t sketched;            /* sample columns sketched (>= samples with look-ahead) */
  int32_t rounds;              /* adaptive rounds over all levels */
  int32_t rank_min, rank_max;  /* over all processed nodes */
  double delta;                /* absolute threshold used */
  double norm_estimate;        /* nu = ||Y_0||_F / sqrt(d0) */
  int64_t near_blocks, far_blocks;
  int64_t bytes_dense, bytes_coupling, bytes_basis; /* stored factor sizes */
  /* phase times in milliseconds (HIP events on the context stream) */
  double t_total, t_tree, t_sample, t_near_gen, t_subtract, t_convtest, t_id, t_upsweep,
      t_coupling, t_misc;
  double t_host_plan;          /* host time of the tree + lists (overlaps the first sketch) */
  double sketch_flops;         /* algorithmic 2*n*n*columns summed over sketch passes */
  double sketch_entries;       /* kernel entries evaluated by the sketch passes */
  int32_t sketch_calls;        /* sketch passes (calls of the black box) */
  int32_t fixed_samples;       /* 1: built with the fixed sample size (d_inc = 0) */
  int64_t bytes_peak;          /* device bytes held by the build at its largest (pool usage) */
} h2_info;

h2_status h2_query(const h2_matrix* h, h2_info* info);
h2_status h2_free(h2_matrix* h);

/* ---------------------------------------------------------------- batched */

/* One problem of a batched build (a kernel matrix on its own point cloud). */
typedef struct {
  int64_t n;
  int32_t dim;
  const double* points;  /* DEVICE (dim x n) SoA, original order; borrowed for the call */
  h2_kernel kernel;
  double tol;
  int32_t leaf_size;
  double eta;
  int32_t d0, d_inc;
  uint64_t seed;
  int32_t norm_mode;
  int32_t oversample;    /* as h2_opts.oversample */
} h2_problem;

typedef struct {
  int32_t precision;  /* h2_precision, common to the batch */
  int32_t d_max;      /* most columns any problem may use, 1..96 */
  int32_t use_graph;  /* 1: capture each launch sequence in one hipGraph and launch it once */
  int32_t first_pass; /* columns sketched up front by the first launch sequence; 0: the
                       * largest d0 plus 32 (the single build's default look-ahead); capped
                       * at d_max.  Problems not converged within them are built again,
                       * together, by a second sequence with d_max columns.  Results equal
                       * those of one sequence with d_max columns (the same sample counts,
                       * ranks and skeletons; factors to rounding, as the ID kernel is
                       * chosen by a sequence's column capacity): Omega is counter-based
                       * and the prefix convergence test at a count does not depend on
                       * later columns. */
  /* Tile shapes (0: the default, 64; else 16, 32, 48 or 64; h2_autotune_tiles
   * picks them).  Results are the same bit for bit for every choice. */
  int32_t sketch_cols; /* columns of Omega per dense-sketch launch: every launch
                        * evaluates each kernel entry once for that many columns */
  int32_t bsr_cols;    /* column-tile width of one workgroup of the block-sparse
                        * products (near-field and far-field subtraction) */
} h2_batch_opts;

typedef struct {
  /* times, nodes, bytes and flops are summed over both launch sequences */
  double t_total_ms;   /* wall time of the call */
  double t_plan_ms;    /* host cluster trees and lists of all problems (threaded) */
  double t_setup_ms;   /* host layout, device allocation and uploads */
  double t_capture_ms; /* graph capture and instantiation (0 without a graph) */
  double t_device_ms;  /* device work: graph launch (or first enqueue) to completion */
  int32_t levels;      /* levels of the longest problem */
  int32_t graph_nodes; /* nodes of the captured graph (0 without a graph) */
  int64_t device_bytes;
  double sketch_flops; /* algorithmic 2 * n^2 * (columns sketched) summed over problems */
  double t_layout_ms;  /* part of t_setup_ms: host layout of the batch */
  double t_alloc_ms;   /* part of t_setup_ms: device allocation and uploads */
  double t_results_ms; /* per-problem result objects after the device work */
  int32_t first_pass;  /* columns of the first launch sequence */
  int32_t second_pass; /* problems built again with d_max columns */
  int32_t sketch_cols; /* tile shapes used (defaults resolved) */
  int32_t bsr_cols;
} h2_batch_info;

/* Builds `count` independent H^2 matrices (Alg. 1 with adaptive sampling, Sec.
 * III) in one launch sequence: every stage of a level is one kernel over the
 * clusters of all problems, and with use_graph the whole sequence is captured
 * in one hipGraph.  The first sequence sketches opts->first_pass columns up
 * front (problems not converged within them are built again by a second
 * sequence with d_max columns); the adaptive loop picks each problem's column
 * count with one prefix QR per cluster, which gives the same count, and the
 * same factors, as adding d_inc columns at a time.  A problem not converged
 * within d_max makes the call fail with H2_ERR_SAMPLES.  out: array of `count` handles (each freed with h2_free;
 * they share device storage, released with the last one).  info may be NULL.
 * Synchronous. */
h2_status h2_build_batched(h2_ctx* ctx, int32_t count, const h2_problem* problems, const h2_batch_opts* opts,
                           h2_matrix** out, h2_batch_info* info);

/* Leaf-size autotuner for h2_build_batched: problems are grouped by (dim,
 * kernel kind, floor(log2 n)); the median-n problem of each group is built
 * alone with every candidate leaf size (twice; the second build's device time
 * counts) and the fastest candidate is written to best[i] for every problem i
 * of the group.  problems' own leaf_size is ignored; opts as for
 * h2_build_batched.  candidates: HOST int32[ncand], each in [2, 256]; best:
 * HOST int32[count].  Candidates that reach d_max are skipped; if none
 * converges the call fails with H2_ERR_SAMPLES.  Synchronous. */
h2_status h2_autotune_leaf(h2_ctx* ctx, int32_t count, const h2_problem* problems, const h2_batch_opts* opts,
                           const int32_t* candidates, int32_t ncand, int32_t* best);

/* Tile-shape autotuner for h2_build_batched (Sec. IV runs each stage of a
 * level as one batched launch; the shapes of those launches are tuned here):
 * builds the given batch with candidate shapes and writes the fastest to
 * tuned (a copy of opts with sketch_cols and bsr_cols set).  The search is
 * coordinate-wise: sketch_cols over {64, 48, 32} with bsr_cols 64, then
 * bsr_cols over {64, 48, 32, 16} with the chosen sketch_cols; each candidate
 * is built twice and the smaller device time counts (one warm-up build with
 * the defaults comes first).  times_ms (HOST double[7], may be NULL) receives
 * those times in that order (sketch 64, 48, 32; bsr 64, 48, 32, 16).  Results
 * do not depend on the shapes, so a tuned batch gives the same matrices.
 * Synchronous; fails as h2_build_batched. */
h2_status h2_autotune_tiles(h2_ctx* ctx, int32_t count, const h2_problem* problems, const h2_batch_opts* opts,
                            h2_batch_opts* tuned, double* times_ms);

/* ------------------------------------------------------------ low-rank update */

/* H^2 approximation of A = H + U V^T on the partition of H (same points,
 * tree and lists), built with the two-sided form of Algorithm 1 and adaptive
 * sampling: row bases from Y = A Omega, column bases from Z = A^T Omega'
 * (Omega' keyed by seed + 1), one shared sample count d, delta from the row
 * sketch.  The black box is the H^2 product of H plus U (V^T Omega) (Sec. V
 * uses an existing H^2 matrix as the sampler); coupling entries at the new
 * skeletons come from H's own format (the nested basis of H evaluated at the
 * skeleton rows) plus U V^T.  The near blocks stay those of H plus the
 * factors U_s V_b^T, which is exact; h2_export(DENSE) writes them out.
 *   old:   a symmetric matrix from h2_build or h2_build_batched; its dense
 *          blocks become shared with the result and live until both are freed.
 *   U, V:  DEVICE n x rank (ld >= n), ORIGINAL point order, borrowed for the
 *          call; 0 <= rank <= 128 (NULL allowed when rank = 0).
 *   opts:  tol, d0, d_inc, d_max, seed, norm_mode, sketch_ahead and oversample
 *          are used (use oversample >= 4: the update's block rows have flat
 *          spectra); leaf_size and eta are taken from old; precision must be
 *          H2_FP64 (else H2_ERR_UNSUPPORTED).
 * The result is two-sided: h2_matvec applies A, the *_C parts export its
 * column side.  Synchronous. */
h2_status h2_build_update(h2_ctx* ctx, h2_matrix* old, int32_t rank, const double* U, int64_t ldu,
                          const double* V, int64_t ldv, const h2_opts* opts, h2_matrix** out);

#ifdef __cplusplus
}
#endif

#endif /* H2_H */
