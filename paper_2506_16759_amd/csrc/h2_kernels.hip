// gfx950 kernels of the adaptive-sketching H^2 construction (Alg. 1, Sec. III-IV).
//
// Wave64 throughout.  The only dense contraction with real arithmetic
// intensity -- the on-the-fly sketch Y = K Omega -- runs on the FP64 matrix
// cores (v_mfma_f64_16x16x4); kernel entries are produced straight into the
// MFMA A-operand lane layout, so no kernel tile ever touches LDS or HBM.  The
// per-cluster QR / column-pivoted QR keep a cluster's sample panel in LDS with
// one thread per panel column and wave shuffles for norms and the pivot argmax.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include <cmath>
#include <cstdint>

#include "h2_device.hpp"
#include "h2_devmath.hpp"

namespace h2dev {
namespace {

constexpr int kWave = 64;

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// kappa as a function of the squared distance.  Covariance kernels: c2 =
// -scale * log2(e) so that exp(-scale * x) = 2^(c2 * x).  Helmholtz IE
// kernel: c2 is the wavenumber k and kappa = cos(k r) / r for r > 0, 0 at
// r == 0 (the diagonal, where the formula is undefined).
template <int KIND>
__device__ __forceinline__ double kernel_of_r2(double r2, double c2) {
  if constexpr (KIND == kExp) {
    return exp2_nonpos(c2 * sqrt_nonneg(r2));
  } else if constexpr (KIND == kGauss) {
    return exp2_nonpos(c2 * r2);
  } else {
    const double r = sqrt(r2);
    return r2 > 0.0 ? cos(c2 * r) / r : 0.0;
  }
}

// Argument of kernel_of_r2 for a kernel function.
__host__ __device__ inline double kernel_c2(KernelFn k) {
  return k.kind == kHelm ? k.scale : -k.scale * kLog2e;
}

// ---------------------------------------------------------- Philox4x64-10

constexpr uint64_t kPhM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox_block(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3, uint64_t k0,
                                             uint64_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    const uint64_t hi0 = __umul64hi(kPhM0, c0), lo0 = kPhM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhM1, c2), lo1 = kPhM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, int64_t nrows, const int32_t* __restrict__ rows,
                                                       int64_t col0, int ncols, double* __restrict__ out, int64_t ldo,
                                                       const int32_t* __restrict__ rowprob,
                                                       const uint64_t* __restrict__ seeds) {
  const int64_t total = nrows * ncols;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t p = e % nrows, c = e / nrows;
    uint64_t c0 = static_cast<uint64_t>(rows ? rows[p] : p), c1 = static_cast<uint64_t>(col0 + c), c2 = 0, c3 = 0;
    philox_block(c0, c1, c2, c3, rowprob ? seeds[rowprob[p]] : seed, 0);
    const double u1 = (static_cast<double>(c0 >> 11) + 0.5) * 0x1p-53;
    const double u2 = (static_cast<double>(c1 >> 11) + 0.5) * 0x1p-53;
    out[p + c * ldo] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// ------------------------------------------------ dense on-the-fly sketch

// One workgroup = 4 waves = 128 consecutive rows; each wave owns 32 rows as two
// 16-row MFMA tiles and all NC output columns.  Columns of K (points j) are
// streamed through LDS 64 at a time together with the matching Omega rows.
// For v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// holds D[l/16 + 4q][l%16] in accumulator element q (rows interleaved by 4).
constexpr int kSkRows = 128;
constexpr int kSkK = 64;
// Points per LDS stage of the FP64 sketch: 32 keeps its registers within
// three waves per SIMD (the contraction runs over the same points in the
// same order whatever the stage size).
constexpr int kSkF64 = 32;

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int DIM, int NC>
struct SkF64Smem {
  double xs[DIM][kSkF64];
  double om[kSkF64][NC + 2];
};

// Rows [tile0, tile0 + 128) of y = K omega for one point set of n points.
template <int DIM, int KIND, int NC>
__device__ __forceinline__ void sketch_f64_body(SkF64Smem<DIM, NC>& sm, int64_t tile0, int64_t n,
                                                const double* __restrict__ X, int64_t ldx, double c2, int ncr,
                                                const double* __restrict__ omega, int64_t ldo,
                                                double* __restrict__ y, int64_t ldy) {
  constexpr int NB = NC / 16;
  auto& xs = sm.xs;
  auto& om = sm.om;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = tile0 + wave * 32;
  const int li = lane & 15, lk = lane >> 4;

  double xa[DIM], xb[DIM];
  {
    const int64_t ia = row0 + li, ib = row0 + 16 + li;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      xa[a] = ia < n ? X[a * ldx + ia] : 0.0;
      xb[a] = ib < n ? X[a * ldx + ib] : 0.0;
    }
  }
  dbl4 acc0[NB], acc1[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    acc0[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    acc1[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  }

  // The next stage's points and Omega rows are fetched into registers while
  // the current stage computes, then written to LDS between two barriers.
  constexpr int PX = (DIM * kSkF64 + 255) / 256, PO = NC * kSkF64 / 256;
  double rx[PX], ro[PO];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u, a = e / kSkF64, jj = e % kSkF64;
      rx[u] = (e < DIM * kSkF64 && j0 + jj < n) ? X[a * ldx + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u, c = e / kSkF64, jj = e % kSkF64;
      ro[u] = (j0 + jj < n && c < ncr) ? omega[c * ldo + j0 + jj] : 0.0;
    }
  };
  fetch(0);
  for (int64_t j0 = 0; j0 < n; j0 += kSkF64) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u;
      if (e < DIM * kSkF64) xs[e / kSkF64][e % kSkF64] = rx[u];
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u;
      om[e % kSkF64][e / kSkF64] = ro[u];
    }
    __syncthreads();
    if (j0 + kSkF64 < n) fetch(j0 + kSkF64);
    // the whole stage unrolled (160 registers, still three waves per SIMD;
    // measured 1.4 % faster than four steps at a time)
#pragma unroll
    for (int kk = 0; kk < kSkF64 / 4; ++kk) {
      const int jj = kk * 4 + lk;
      double ra = 0.0, rb = 0.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double xj = xs[a][jj];
        const double da = xa[a] - xj, db = xb[a] - xj;
        ra += da * da;
        rb += db * db;
      }
      const double ka = kernel_of_r2<KIND>(ra, c2);
      const double kb = kernel_of_r2<KIND>(rb, c2);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double bv = om[jj][c * 16 + li];
        acc0[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ka, bv, acc0[c], 0, 0, 0);
        acc1[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(kb, bv, acc1[c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = c * 16 + li;
    if (col >= ncr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ra = row0 + lk + 4 * q, rb = row0 + 16 + lk + 4 * q;
      if (ra < n) y[col * ldy + ra] = acc0[c][q];
      if (rb < n) y[col * ldy + rb] = acc1[c][q];
    }
  }
}

// One problem of a batched sketch: its n points start at global row `base`
// of the shared (point, Omega, y) arrays.
struct SketchJob {
  int64_t n;
  int64_t base;
  double c2;
  int kind;
  int pad;
};

template <int DIM, int KIND, int NC>
__global__ __launch_bounds__(256, KIND == kHelm ? 2 : 3) void sketch_f64_kernel(int64_t n, const double* __restrict__ X,
                                                                                int64_t ldx,
                                                         double c2, int ncr, const double* __restrict__ omega,
                                                         int64_t ldo, double* __restrict__ y, int64_t ldy) {
  __shared__ SkF64Smem<DIM, NC> sm;
  sketch_f64_body<DIM, KIND, NC>(sm, int64_t(blockIdx.x) * kSkRows, n, X, ldx, c2, ncr, omega, ldo, y, ldy);
}

// Batched: workgroup b handles row tile tiles[2b+1] of job tiles[2b] (3-D
// coordinates; lower-dimensional point sets carry zero coordinates).
template <int NC>
__global__ __launch_bounds__(256, 3) void sketch_f64_batched(const SketchJob* __restrict__ jobs,
                                                          const int32_t* __restrict__ tiles,
                                                          const double* __restrict__ X, int64_t ldx, int ncr,
                                                          const double* __restrict__ omega, int64_t ldo,
                                                          double* __restrict__ y, int64_t ldy) {
  __shared__ SkF64Smem<3, NC> sm;
  const SketchJob J = jobs[tiles[2 * blockIdx.x]];
  const int64_t t0 = tiles[2 * blockIdx.x + 1];
  if (J.kind == kExp)
    sketch_f64_body<3, kExp, NC>(sm, t0, J.n, X + J.base, ldx, J.c2, ncr, omega + J.base, ldo, y + J.base, ldy);
  else
    sketch_f64_body<3, kGauss, NC>(sm, t0, J.n, X + J.base, ldx, J.c2, ncr, omega + J.base, ldo, y + J.base, ldy);
}

// --------------------------------------------- symmetric-tile FP64 sketch
//
// K is symmetric, so the entries of a pair of 128-row tiles (a, b), a < b,
// serve both Y(I_a) += K(I_a, I_b) Omega(I_b) and Y(I_b) += K(I_a, I_b)^T
// Omega(I_a): every entry of the upper block triangle is evaluated once.
// Workgroup a keeps rows I_a stationary and streams the points from the start
// of I_a to n, 32 per stage:
//  * the row side accumulates in registers as in sketch_f64_body (the
//    diagonal tile in full, then every later point);
//  * in stages past the diagonal tile the entries also go to LDS, and the
//    four waves form P = K(I_a, stage)^T Omega(I_a) (32 points x 64 columns)
//    on the matrix cores: wave w takes points 16 (w / 2) .. + 15 of the stage
//    and column tiles 2 (w % 2), 2 (w % 2) + 1, the contraction running over
//    all 128 rows of the tile, with its Omega(I_a) operands (64 per lane)
//    held in registers for the whole workgroup (one workgroup per CU, so a
//    wave has the register file of its SIMD to itself).  The entries of
//    consecutive stages alternate between two LDS buffers, and the transposed
//    product of a stage runs in the next stage, after the row side's entries,
//    so that a stage has two barriers.  P goes to the scratch slot of tile a,
//    which holds points 128 (a + 1) .. n - 1, 64 doubles per point, from
//    sym_slot(a, n) points on.
// sketch_sym_reduce_kernel then adds to each point's row-side result the
// slots of the tiles before its own, in increasing a (a fixed order, so the
// result does not depend on scheduling).
constexpr int kSymLdE = kSkF64 + 2;

template <int DIM>
struct SkSymSmem {
  double xs[DIM][kSkF64];
  double om[kSkF64][64 + 2];
  double e[2][kSkRows][kSymLdE];  // K(I_a, stage points), stages alternating
};

// First scratch row of tile a's slot: sum over a' < a of (n - 128 (a' + 1)).
__host__ __device__ inline int64_t sym_slot(int64_t a, int64_t n) { return a * n - kSkRows * a * (a + 1) / 2; }

template <int DIM, int KIND>
__global__ __launch_bounds__(256, 1) void sketch_sym_f64_kernel(int64_t n, const double* __restrict__ X,
                                                                int64_t ldx, double c2, int ncr,
                                                                const double* __restrict__ omega, int64_t ldo,
                                                                double* __restrict__ y, int64_t ldy,
                                                                double* __restrict__ z) {
  constexpr int NC = 64, NB = 4;
  __shared__ SkSymSmem<DIM> sm;
  auto& xs = sm.xs;
  auto& om = sm.om;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t a = blockIdx.x;
  const int64_t tile0 = a * kSkRows;
  const int64_t row0 = tile0 + wave * 32;

  double xa[DIM], xb[DIM];
  {
    const int64_t ia = row0 + li, ib = row0 + 16 + li;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      xa[d] = ia < n ? X[d * ldx + ia] : 0.0;
      xb[d] = ib < n ? X[d * ldx + ib] : 0.0;
    }
  }
  dbl4 acc0[NB], acc1[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    acc0[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    acc1[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  const int pb = wave >> 1, ct = 2 * (wave & 1);  // this wave's block of the transposed product
  // B operands of the transposed product: Omega(tile0 + 4s + l/16, 16 (ct + h) + l%16)
  double ob[2][kSkRows / 4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = 16 * (ct + h) + li;
#pragma unroll
    for (int s2 = 0; s2 < kSkRows / 4; ++s2) {
      const int64_t r = tile0 + 4 * s2 + lk;
      ob[h][s2] = (r < n && c < ncr) ? omega[c * ldo + r] : 0.0;
    }
  }
  double* const zs = z + NC * sym_slot(a, n);

  constexpr int PX = (DIM * kSkF64 + 255) / 256, PO = NC * kSkF64 / 256;
  double rx[PX], ro[PO];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u, d = e / kSkF64, jj = e % kSkF64;
      rx[u] = (e < DIM * kSkF64 && j0 + jj < n) ? X[d * ldx + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u, c = e / kSkF64, jj = e % kSkF64;
      ro[u] = (j0 + jj < n && c < ncr) ? omega[c * ldo + j0 + jj] : 0.0;
    }
  };
  // D[point][column] = sum over the 128 rows r of K(r, point) Omega(r, column)
  // for the 32 points of stage jp (entries in buffer eb): lane l supplies
  // A[l%16][l/16] = K(4s + l/16, point) and B[l/16][l%16] = Omega(4s + l/16, column).
  // The result stays in registers until the next stage has passed its
  // barriers and is stored before that stage's prefetch is issued, so the
  // wait for the prefetch does not include fresh stores (one counter covers
  // both).
  dbl4 t0{0.0, 0.0, 0.0, 0.0}, t1{0.0, 0.0, 0.0, 0.0};
  int64_t tst = -1;  // stage of the unstored result
  // (even and odd row steps accumulate separately: four independent chains)
  auto transposed = [&](int64_t jp, int eb) {
    dbl4 u0{0.0, 0.0, 0.0, 0.0}, u1{0.0, 0.0, 0.0, 0.0};
    t0 = dbl4{0.0, 0.0, 0.0, 0.0};
    t1 = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kSkRows / 4; s += 2) {
      const double av = sm.e[eb][4 * s + lk][16 * pb + li];
      const double aw = sm.e[eb][4 * s + 4 + lk][16 * pb + li];
      t0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ob[0][s], t0, 0, 0, 0);
      t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ob[1][s], t1, 0, 0, 0);
      u0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aw, ob[0][s + 1], u0, 0, 0, 0);
      u1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aw, ob[1][s + 1], u1, 0, 0, 0);
    }
    t0 += u0;
    t1 += u1;
    tst = jp;
  };
  auto store_transposed = [&] {
    if (tst < 0) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p = tst + 16 * pb + lk + 4 * q;
      if (p < n) {
        double* zr = zs + (p - tile0 - kSkRows) * NC;
        zr[16 * ct + li] = t0[q];
        zr[16 * ct + 16 + li] = t1[q];
      }
    }
    tst = -1;
  };
  fetch(tile0);
  int64_t pending = -1;  // stage whose transposed product is still to do
  for (int64_t j0 = tile0; j0 < n; j0 += kSkF64) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u;
      if (e < DIM * kSkF64) xs[e / kSkF64][e % kSkF64] = rx[u];
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u;
      om[e % kSkF64][e / kSkF64] = ro[u];
    }
    __syncthreads();
    store_transposed();
    if (j0 + kSkF64 < n) fetch(j0 + kSkF64);
    const bool cross = j0 >= tile0 + kSkRows;  // the same for the whole workgroup
    const int cur = int((j0 - tile0) / kSkF64) & 1;
    // the whole stage unrolled (measured 1.3 % faster than four steps at a time)
#pragma unroll
    for (int kk = 0; kk < kSkF64 / 4; ++kk) {
      const int jj = kk * 4 + lk;
      double ra = 0.0, rb = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double xj = xs[d][jj];
        const double da = xa[d] - xj, db = xb[d] - xj;
        ra += da * da;
        rb += db * db;
      }
      const double ka = kernel_of_r2<KIND>(ra, c2);
      const double kb = kernel_of_r2<KIND>(rb, c2);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double bv = om[jj][c * 16 + li];
        acc0[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ka, bv, acc0[c], 0, 0, 0);
        acc1[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(kb, bv, acc1[c], 0, 0, 0);
      }
      if (cross) {
        sm.e[cur][wave * 32 + li][jj] = ka;
        sm.e[cur][wave * 32 + 16 + li][jj] = kb;
      }
    }
    // the previous stage's entries were written before this stage's barriers
    if (pending >= 0) transposed(pending, cur ^ 1);
    pending = cross ? j0 : -1;
  }
  store_transposed();
  if (pending >= 0) {
    __syncthreads();
    transposed(pending, int((pending - tile0) / kSkF64) & 1);
    store_transposed();
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = c * 16 + li;
    if (col >= ncr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ra = row0 + lk + 4 * q, rb = row0 + 16 + lk + 4 * q;
      if (ra < n) y[col * ldy + ra] = acc0[c][q];
      if (rb < n) y[col * ldy + rb] = acc1[c][q];
    }
  }
}

// y(p, c) += slot a of z at point p for every tile a before p's own, in
// increasing a.  One workgroup per 64 points (all in one 128-point tile); y is
// read and written down its columns through an LDS transpose, z along its
// 64-double rows.
__global__ __launch_bounds__(256) void sketch_sym_reduce_kernel(int64_t n, int ncr, const double* __restrict__ z,
                                                                double* __restrict__ y, int64_t ldy) {
  __shared__ double t[64][65];  // [column][point]
  // the last points (the most slots to add) first
  const int64_t p0 = int64_t(gridDim.x - 1 - blockIdx.x) * 64;
  const int64_t b = p0 / kSkRows;
  if (b == 0) return;  // tile 0 receives nothing (uniform over the workgroup)
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k, c = e >> 6, pp = e & 63;
    t[c][pp] = (c < ncr && p0 + pp < n) ? y[c * ldy + p0 + pp] : 0.0;
  }
  __syncthreads();
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k;
    v[k] = t[e & 63][e >> 6];
  }
  // two slots' loads in flight before their sums (same order of additions)
  int64_t a = 0;
  for (; a + 1 < b; a += 2) {
    const double* z0 = z + 64 * (sym_slot(a, n) + p0 - (a + 1) * kSkRows);
    const double* z1 = z + 64 * (sym_slot(a + 1, n) + p0 - (a + 2) * kSkRows);
    double w0[16], w1[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      const bool in = p0 + (e >> 6) < n;
      w0[k] = in ? z0[e] : 0.0;
      w1[k] = in ? z1[e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (v[k] + w0[k]) + w1[k];
  }
  if (a < b) {
    const double* z0 = z + 64 * (sym_slot(a, n) + p0 - (a + 1) * kSkRows);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      if (p0 + (e >> 6) < n) v[k] += z0[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k;
    t[e & 63][e >> 6] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k, c = e >> 6, pp = e & 63;
    if (c < ncr && p0 + pp < n) y[c * ldy + p0 + pp] = t[c][pp];
  }
}

// --------------------------------------------- mixed-precision sketches

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// kappa in FP32 from the hardware square root and base-2 exponential.
template <int KIND>
__device__ __forceinline__ float kernel_of_r2_f32(float r2, float c2) {
  if constexpr (KIND == kExp) {
    return __builtin_amdgcn_exp2f(c2 * __builtin_amdgcn_sqrtf(r2));
  } else {
    return __builtin_amdgcn_exp2f(c2 * r2);
  }
}

// FP32 partial sums are folded into FP64 accumulators every kFlush stages of
// kSkK points.  Over 256 points the FP32 rounding of the running sums already
// lifts the noise of the samples above the adaptive threshold at tol 1e-6 (16
// extra samples on the 131072-point covariance matrix); every 64 points it does
// not.
constexpr int kFlush = 1;

// FP32 entries, v_mfma_f32_16x16x4_f32.  Same tiling as the FP64 kernel:
// lane l supplies A[l%16][l/16], B[l/16][l%16] and holds D[4*(l/16)+q][l%16].
// Squared distances are formed in FP64 (without packed FP32 arithmetic an FP64
// add or FMA issues at the FP32 rate) and rounded once to FP32; the square
// root and exponential are the hardware FP32 ones.  Omega is staged in LDS as
// FP32; the next stage's points and Omega rows are fetched into registers
// while the current one computes.  Waves of one SIMD overlap their entry
// generation (VALU) with each other's FP32 MFMAs.
template <int DIM, int NC>
struct SkF32Smem {
  double xs[DIM][kSkK];
  float om[kSkK][NC + 4];
};

template <int DIM, int KIND, int NC>
__device__ __forceinline__ void sketch_f32_body(SkF32Smem<DIM, NC>& sm, int64_t tile0, int64_t n,
                                                const double* __restrict__ X, int64_t ldx, float c2, int ncr,
                                                const double* __restrict__ omega, int64_t ldo,
                                                double* __restrict__ y, int64_t ldy) {
  constexpr int NB = NC / 16;
  auto& xs = sm.xs;
  auto& om = sm.om;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = tile0 + wave * 32;
  const int li = lane & 15, lk = lane >> 4;
  double xa[DIM], xb[DIM];
  {
    const int64_t ia = row0 + li, ib = row0 + 16 + li;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      xa[a] = ia < n ? X[a * ldx + ia] : 0.0;
      xb[a] = ib < n ? X[a * ldx + ib] : 0.0;
    }
  }
  flt4 acc0[NB], acc1[NB];
  double ya[NB][4], yb[NB][4];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    acc0[c] = flt4{0.f, 0.f, 0.f, 0.f};
    acc1[c] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) ya[c][q] = yb[c][q] = 0.0;
  }
  constexpr int PX = (DIM * kSkK + 255) / 256, PO = NC * kSkK / 256;
  double rx[PX];
  float ro[PO];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u, a = e / kSkK, jj = e % kSkK;
      rx[u] = (e < DIM * kSkK && j0 + jj < n) ? X[a * ldx + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u, c = e / kSkK, jj = e % kSkK;
      ro[u] = (j0 + jj < n && c < ncr) ? float(omega[c * ldo + j0 + jj]) : 0.0f;
    }
  };
  fetch(0);
  int stage = 0;
  for (int64_t j0 = 0; j0 < n; j0 += kSkK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u;
      if (e < DIM * kSkK) xs[e / kSkK][e % kSkK] = rx[u];
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u;
      om[e % kSkK][e / kSkK] = ro[u];
    }
    __syncthreads();
    if (j0 + kSkK < n) fetch(j0 + kSkK);
#pragma unroll
    for (int kk = 0; kk < kSkK / 4; ++kk) {
      const int jj = kk * 4 + lk;
      double ra = 0.0, rb = 0.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double xj = xs[a][jj];
        const double da = xa[a] - xj, db = xb[a] - xj;
        ra += da * da;
        rb += db * db;
      }
      const float ka = kernel_of_r2_f32<KIND>(float(ra), c2);
      const float kb = kernel_of_r2_f32<KIND>(float(rb), c2);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const float bv = om[jj][c * 16 + li];
        acc0[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ka, bv, acc0[c], 0, 0, 0);
        acc1[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(kb, bv, acc1[c], 0, 0, 0);
      }
    }
    if (++stage == kFlush || j0 + kSkK >= n) {
      stage = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ya[c][q] += double(acc0[c][q]);
          yb[c][q] += double(acc1[c][q]);
        }
        acc0[c] = flt4{0.f, 0.f, 0.f, 0.f};
        acc1[c] = flt4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = c * 16 + li;
    if (col >= ncr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ra = row0 + 4 * lk + q, rb = row0 + 16 + 4 * lk + q;
      if (ra < n) y[col * ldy + ra] = ya[c][q];
      if (rb < n) y[col * ldy + rb] = yb[c][q];
    }
  }
}

template <int DIM, int KIND, int NC>
__global__ __launch_bounds__(256) void sketch_f32_kernel(int64_t n, const double* __restrict__ X, int64_t ldx,
                                                         float c2, int ncr, const double* __restrict__ omega,
                                                         int64_t ldo, double* __restrict__ y, int64_t ldy) {
  __shared__ SkF32Smem<DIM, NC> sm;
  sketch_f32_body<DIM, KIND, NC>(sm, int64_t(blockIdx.x) * kSkRows, n, X, ldx, c2, ncr, omega, ldo, y, ldy);
}

template <int NC>
__global__ __launch_bounds__(256) void sketch_f32_batched(const SketchJob* __restrict__ jobs,
                                                          const int32_t* __restrict__ tiles,
                                                          const double* __restrict__ X, int64_t ldx, int ncr,
                                                          const double* __restrict__ omega, int64_t ldo,
                                                          double* __restrict__ y, int64_t ldy) {
  __shared__ SkF32Smem<3, NC> sm;
  const SketchJob J = jobs[tiles[2 * blockIdx.x]];
  const int64_t t0 = tiles[2 * blockIdx.x + 1];
  const float c2 = float(J.c2);
  if (J.kind == kExp)
    sketch_f32_body<3, kExp, NC>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, y + J.base, ldy);
  else
    sketch_f32_body<3, kGauss, NC>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, y + J.base, ldy);
}

// Split bf16 products.  A pair of FP32 values (a, b) is split into S packed
// bf16x2 words, each the round-to-nearest bf16 of what the earlier words left
// (the remainders are exact in FP32).  With S = 2 the products
// hi*hi + hi*lo + lo*hi keep about 2^-17 relative accuracy; with S = 3 the six
// products whose split orders add up to at most 2 (hh, hm, mh, hl, lh, mm)
// keep about 2^-24, the accuracy of FP32 products, on the bf16 matrix cores.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <int S>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t (&w)[S]) {
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const bf16x2 p = {__bf16(a), __bf16(b)};
    const uint32_t u = __builtin_bit_cast(uint32_t, p);
    w[t] = u;
    if (t + 1 < S) {
      a -= __uint_as_float(u << 16);
      b -= __uint_as_float(u & 0xffff0000u);
    }
  }
}

// Entries in FP32 split into S bf16 terms, v_mfma_f32_16x16x32_bf16.  Lane l
// supplies A[l%16][8*(l/16)+e] and B[8*(l/16)+e][l%16], e = 0..7, and holds
// D[4*(l/16)+q][l%16].  Entries as in the FP32 kernel (FP64 squared distance,
// FP32 exp2/sqrt).  The Omega tile is staged pre-split as [term][column][point]
// bf16 so each lane reads its 8 points of a term with one 16-byte LDS load.
// FP32 partial sums are folded into FP64 every kFlush stages.
constexpr int kBfK = 64;  // points per stage (two MFMA k-steps of 32)

constexpr int kBfLdp = kBfK / 2 + 4;  // dwords per staged column (2 bf16 per dword)

template <int DIM, int NC, int S>
struct SkBfSmem {
  double xs[DIM][kBfK];
  uint32_t om[S][NC * kBfLdp];
};

// PRE: Omega arrives pre-split (split_omega_kernel): word (t, c, p) at
// wsplit[(t * ncr + c) * npairs + p] holds term t of points 2p, 2p+1 of column c.
template <int DIM, int KIND, int NC, int S, bool PRE>
__device__ __forceinline__ void sketch_bf16_body(SkBfSmem<DIM, NC, S>& sm, int64_t tile0, int64_t n,
                                                 const double* __restrict__ X, int64_t ldx, float c2, int ncr,
                                                 const double* __restrict__ omega, int64_t ldo,
                                                 const uint32_t* __restrict__ wsplit, int64_t npairs,
                                                 double* __restrict__ y, int64_t ldy) {
  static_assert(S == 2 || S == 3, "two or three bf16 terms");
  constexpr int NB = NC / 16;
  constexpr int LDP = kBfLdp;
  // products (term of K, term of Omega) with split orders adding up to < S
  constexpr int NP = S == 2 ? 3 : 6;
  constexpr int PI[6] = {0, 0, 1, 0, 2, 1};
  constexpr int PJ[6] = {0, 1, 0, 2, 0, 1};
  auto& xs = sm.xs;
  auto& om = sm.om;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = tile0 + wave * 32;
  const int li = lane & 15, lk = lane >> 4;
  double xa[DIM], xb[DIM];
  {
    const int64_t ia = row0 + li, ib = row0 + 16 + li;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      xa[a] = ia < n ? X[a * ldx + ia] : 0.0;
      xb[a] = ib < n ? X[a * ldx + ib] : 0.0;
    }
  }
  flt4 acc0[NB], acc1[NB];
  double ya[NB][4], yb[NB][4];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    acc0[c] = flt4{0.f, 0.f, 0.f, 0.f};
    acc1[c] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) ya[c][q] = yb[c][q] = 0.0;
  }
  // The next stage's points and Omega rows are fetched into registers while
  // the current stage computes; a thread stages pairs of points (2p, 2p+1) of
  // one column, which form one dword of each split Omega term.
  constexpr int PX = (DIM * kBfK + 255) / 256, PP = NC * (kBfK / 2) / 256;
  double rx[PX];
  float ro0[PRE ? 1 : PP], ro1[PRE ? 1 : PP];
  uint32_t rw[PRE ? S : 1][PRE ? PP : 1];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u, a = e / kBfK, jj = e % kBfK;
      rx[u] = (e < DIM * kBfK && j0 + jj < n) ? X[a * ldx + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int e = tid + 256 * u, c = e / (kBfK / 2), pp = e % (kBfK / 2);
      if constexpr (PRE) {
        const int64_t pw = j0 / 2 + pp;
#pragma unroll
        for (int t = 0; t < S; ++t)
          rw[t][u] = (c < ncr && pw < npairs) ? wsplit[(int64_t(t) * ncr + c) * npairs + pw] : 0u;
      } else {
        const int64_t j = j0 + 2 * pp;
        ro0[u] = (c < ncr && j < n) ? float(omega[c * ldo + j]) : 0.0f;
        ro1[u] = (c < ncr && j + 1 < n) ? float(omega[c * ldo + j + 1]) : 0.0f;
      }
    }
  };
  fetch(0);
  int stage = 0;
  for (int64_t j0 = 0; j0 < n; j0 += kBfK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u;
      if (e < DIM * kBfK) xs[e / kBfK][e % kBfK] = rx[u];
    }
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int e = tid + 256 * u, c = e / (kBfK / 2), pp = e % (kBfK / 2);
      uint32_t w[S];
      if constexpr (PRE) {
#pragma unroll
        for (int t = 0; t < S; ++t) w[t] = rw[t][u];
      } else {
        split_pair<S>(ro0[u], ro1[u], w);
      }
#pragma unroll
      for (int t = 0; t < S; ++t) om[t][c * LDP + pp] = w[t];
    }
    __syncthreads();
    if (j0 + kBfK < n) fetch(j0 + kBfK);
#pragma unroll
    for (int ks = 0; ks < kBfK; ks += 32) {
      const int jb = ks + 8 * lk;  // first of this lane's 8 points
      u32x4 a0[S], a1[S];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        float kv[2][2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int jj = jb + 2 * w + e;
          double ra = 0.0, rb = 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            const double xj = xs[a][jj];
            const double da = xa[a] - xj, db = xb[a] - xj;
            ra += da * da;
            rb += db * db;
          }
          kv[0][e] = kernel_of_r2_f32<KIND>(float(ra), c2);
          kv[1][e] = kernel_of_r2_f32<KIND>(float(rb), c2);
        }
        uint32_t w0[S], w1[S];
        split_pair<S>(kv[0][0], kv[0][1], w0);
        split_pair<S>(kv[1][0], kv[1][1], w1);
#pragma unroll
        for (int t = 0; t < S; ++t) {
          a0[t][w] = w0[t];
          a1[t][w] = w1[t];
        }
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const int col = c * 16 + li;
        bf16x8 B[S];
#pragma unroll
        for (int t = 0; t < S; ++t)
          B[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&om[t][col * LDP + jb / 2]));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const bf16x8 A0 = __builtin_bit_cast(bf16x8, a0[PI[p]]), A1 = __builtin_bit_cast(bf16x8, a1[PI[p]]);
          acc0[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B[PJ[p]], acc0[c], 0, 0, 0);
          acc1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B[PJ[p]], acc1[c], 0, 0, 0);
        }
      }
    }
    if (++stage == kFlush || j0 + kBfK >= n) {
      stage = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ya[c][q] += double(acc0[c][q]);
          yb[c][q] += double(acc1[c][q]);
        }
        acc0[c] = flt4{0.f, 0.f, 0.f, 0.f};
        acc1[c] = flt4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = c * 16 + li;
    if (col >= ncr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ra = row0 + 4 * lk + q, rb = row0 + 16 + 4 * lk + q;
      if (ra < n) y[col * ldy + ra] = ya[c][q];
      if (rb < n) y[col * ldy + rb] = yb[c][q];
    }
  }
}

template <int DIM, int KIND, int NC, int S>
__global__ __launch_bounds__(256) void sketch_bf16_kernel(int64_t n, const double* __restrict__ X, int64_t ldx,
                                                          float c2, int ncr, const uint32_t* __restrict__ wsplit,
                                                          int64_t npairs, double* __restrict__ y, int64_t ldy) {
  __shared__ SkBfSmem<DIM, NC, S> sm;
  sketch_bf16_body<DIM, KIND, NC, S, true>(sm, int64_t(blockIdx.x) * kSkRows, n, X, ldx, c2, ncr, nullptr, 0,
                                           wsplit, npairs, y, ldy);
}

// Omega columns split once for every workgroup of a sketch launch: word
// (t, c, p) = term t of the pair (Omega[2p, c], Omega[2p+1, c]) (FP32 values,
// the second zero past n), npairs = ceil(n / 2).
template <int S>
__global__ __launch_bounds__(256) void split_omega_kernel(int64_t n, int ncols, const double* __restrict__ omega,
                                                          int64_t ldo, int64_t npairs, uint32_t* __restrict__ w) {
  const int64_t total = int64_t(ncols) * npairs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(e / npairs);
    const int64_t pw = e % npairs, j = 2 * pw;
    float a = float(omega[c * ldo + j]);
    float b = j + 1 < n ? float(omega[c * ldo + j + 1]) : 0.0f;
    // Omega is rounded to FP32 first and the FP32 value is split, as in the
    // in-kernel split of the batched sketch: without this barrier the compiler
    // fuses the two roundings of the first value into one double -> bf16
    // rounding, which differs at FP32 values halfway between two bf16 values
    asm volatile("" : "+v"(a), "+v"(b));
    uint32_t v[S];
    split_pair<S>(a, b, v);
#pragma unroll
    for (int t = 0; t < S; ++t) w[(int64_t(t) * ncols + c) * npairs + pw] = v[t];
  }
}

template <int NC, int S>
__global__ __launch_bounds__(256) void sketch_bf16_batched(const SketchJob* __restrict__ jobs,
                                                           const int32_t* __restrict__ tiles,
                                                           const double* __restrict__ X, int64_t ldx, int ncr,
                                                           const double* __restrict__ omega, int64_t ldo,
                                                           double* __restrict__ y, int64_t ldy) {
  __shared__ SkBfSmem<3, NC, S> sm;
  const SketchJob J = jobs[tiles[2 * blockIdx.x]];
  const int64_t t0 = tiles[2 * blockIdx.x + 1];
  const float c2 = float(J.c2);
  if (J.kind == kExp)
    sketch_bf16_body<3, kExp, NC, S, false>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, nullptr, 0,
                                            y + J.base, ldy);
  else
    sketch_bf16_body<3, kGauss, NC, S, false>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, nullptr, 0,
                                              y + J.base, ldy);
}

// FP32 kernel entries, FP64 contraction: entries are evaluated in FP32 (FP64
// squared distance, hardware exp2/sqrt), converted to FP64 and contracted with the
// FP64 Omega on the FP64 matrix cores with FP64 accumulation.  The entry error
// (~1e-7 relative) enters the samples as independent noise, not accumulated
// rounding, so the samples stay within ~1e-7 of K Omega at about a third of
// the FP64 entry cost.  Same tiling and lane layout as the FP64 kernel.
template <int DIM, int NC>
struct SkE32Smem {
  double xs[DIM][kSkK];
  double om[kSkK][NC + 2];
};

template <int DIM, int KIND, int NC>
__device__ __forceinline__ void sketch_e32_body(SkE32Smem<DIM, NC>& sm, int64_t tile0, int64_t n,
                                                const double* __restrict__ X, int64_t ldx, float c2, int ncr,
                                                const double* __restrict__ omega, int64_t ldo,
                                                double* __restrict__ y, int64_t ldy) {
  constexpr int NB = NC / 16;
  auto& xs = sm.xs;
  auto& om = sm.om;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = tile0 + wave * 32;
  const int li = lane & 15, lk = lane >> 4;
  double xa[DIM], xb[DIM];
  {
    const int64_t ia = row0 + li, ib = row0 + 16 + li;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      xa[a] = ia < n ? X[a * ldx + ia] : 0.0;
      xb[a] = ib < n ? X[a * ldx + ib] : 0.0;
    }
  }
  dbl4 acc0[NB], acc1[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    acc0[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    acc1[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  constexpr int PX = (DIM * kSkK + 255) / 256, PO = NC * kSkK / 256;
  double rx[PX], ro[PO];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u, a = e / kSkK, jj = e % kSkK;
      rx[u] = (e < DIM * kSkK && j0 + jj < n) ? X[a * ldx + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u, c = e / kSkK, jj = e % kSkK;
      ro[u] = (j0 + jj < n && c < ncr) ? omega[c * ldo + j0 + jj] : 0.0;
    }
  };
  fetch(0);
  for (int64_t j0 = 0; j0 < n; j0 += kSkK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + 256 * u;
      if (e < DIM * kSkK) xs[e / kSkK][e % kSkK] = rx[u];
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int e = tid + 256 * u;
      om[e % kSkK][e / kSkK] = ro[u];
    }
    __syncthreads();
    if (j0 + kSkK < n) fetch(j0 + kSkK);
    // the whole stage unrolled (measured 2 % faster than four steps at a time)
#pragma unroll
    for (int kk = 0; kk < kSkK / 4; ++kk) {
      const int jj = kk * 4 + lk;
      double ra = 0.0, rb = 0.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double xj = xs[a][jj];
        const double da = xa[a] - xj, db = xb[a] - xj;
        ra += da * da;
        rb += db * db;
      }
      const double ka = double(kernel_of_r2_f32<KIND>(float(ra), c2));
      const double kb = double(kernel_of_r2_f32<KIND>(float(rb), c2));
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double bv = om[jj][c * 16 + li];
        acc0[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ka, bv, acc0[c], 0, 0, 0);
        acc1[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(kb, bv, acc1[c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = c * 16 + li;
    if (col >= ncr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ra = row0 + lk + 4 * q, rb = row0 + 16 + lk + 4 * q;
      if (ra < n) y[col * ldy + ra] = acc0[c][q];
      if (rb < n) y[col * ldy + rb] = acc1[c][q];
    }
  }
}

template <int DIM, int KIND, int NC>
__global__ __launch_bounds__(256) void sketch_e32_kernel(int64_t n, const double* __restrict__ X, int64_t ldx,
                                                         float c2, int ncr, const double* __restrict__ omega,
                                                         int64_t ldo, double* __restrict__ y, int64_t ldy) {
  __shared__ SkE32Smem<DIM, NC> sm;
  sketch_e32_body<DIM, KIND, NC>(sm, int64_t(blockIdx.x) * kSkRows, n, X, ldx, c2, ncr, omega, ldo, y, ldy);
}

template <int NC>
__global__ __launch_bounds__(256) void sketch_e32_batched(const SketchJob* __restrict__ jobs,
                                                          const int32_t* __restrict__ tiles,
                                                          const double* __restrict__ X, int64_t ldx, int ncr,
                                                          const double* __restrict__ omega, int64_t ldo,
                                                          double* __restrict__ y, int64_t ldy) {
  __shared__ SkE32Smem<3, NC> sm;
  const SketchJob J = jobs[tiles[2 * blockIdx.x]];
  const int64_t t0 = tiles[2 * blockIdx.x + 1];
  const float c2 = float(J.c2);
  if (J.kind == kExp)
    sketch_e32_body<3, kExp, NC>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, y + J.base, ldy);
  else
    sketch_e32_body<3, kGauss, NC>(sm, t0, J.n, X + J.base, ldx, c2, ncr, omega + J.base, ldo, y + J.base, ldy);
}

template <int P, int DIM, int KIND, int NC>
void launch_sketch_one(dim3 grid, hipStream_t s, int64_t n, const double* X, int64_t ldx, double c2, int ncr,
                       const double* omega, int64_t ldo, const uint32_t* wsplit, int64_t npairs, double* y,
                       int64_t ldy) {
  if constexpr (P == 0)
    sketch_f64_kernel<DIM, KIND, NC><<<grid, 256, 0, s>>>(n, X, ldx, c2, ncr, omega, ldo, y, ldy);
  else if constexpr (P == 1)
    sketch_f32_kernel<DIM, KIND, NC><<<grid, 256, 0, s>>>(n, X, ldx, float(c2), ncr, omega, ldo, y, ldy);
  else if constexpr (P == 2)
    sketch_bf16_kernel<DIM, KIND, NC, 2><<<grid, 256, 0, s>>>(n, X, ldx, float(c2), ncr, wsplit, npairs, y, ldy);
  else if constexpr (P == 3)
    sketch_e32_kernel<DIM, KIND, NC><<<grid, 256, 0, s>>>(n, X, ldx, float(c2), ncr, omega, ldo, y, ldy);
  else
    sketch_bf16_kernel<DIM, KIND, NC, 3><<<grid, 256, 0, s>>>(n, X, ldx, float(c2), ncr, wsplit, npairs, y, ldy);
}

template <int P, int DIM, int KIND>
hipError_t launch_sketch_nc(hipStream_t s, int64_t n, const double* X, int64_t ldx, double c2, int ncr,
                            const double* omega, int64_t ldo, const uint32_t* wsplit, int64_t npairs, double* y,
                            int64_t ldy) {
  const dim3 grid(static_cast<unsigned>((n + kSkRows - 1) / kSkRows));
  if (ncr <= 16)
    launch_sketch_one<P, DIM, KIND, 16>(grid, s, n, X, ldx, c2, ncr, omega, ldo, wsplit, npairs, y, ldy);
  else if (ncr <= 32)
    launch_sketch_one<P, DIM, KIND, 32>(grid, s, n, X, ldx, c2, ncr, omega, ldo, wsplit, npairs, y, ldy);
  else if (ncr <= 48)
    launch_sketch_one<P, DIM, KIND, 48>(grid, s, n, X, ldx, c2, ncr, omega, ldo, wsplit, npairs, y, ldy);
  else if (ncr <= 64)
    launch_sketch_one<P, DIM, KIND, 64>(grid, s, n, X, ldx, c2, ncr, omega, ldo, wsplit, npairs, y, ldy);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int P>
hipError_t launch_sketch_p(hipStream_t s, int64_t n, int dim, int kind, const double* X, int64_t ldx, double c2,
                           int nc, const double* om, int64_t ldo, const uint32_t* w, int64_t npairs, double* yy,
                           int64_t ldy) {
  if (kind == kHelm) {  // FP64 only
    if constexpr (P == 0) {
      if (dim == 1) return launch_sketch_nc<P, 1, kHelm>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
      if (dim == 2) return launch_sketch_nc<P, 2, kHelm>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
      return launch_sketch_nc<P, 3, kHelm>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    }
    return hipErrorInvalidValue;
  }
  if (kind == kExp) {
    if (dim == 1) return launch_sketch_nc<P, 1, kExp>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    if (dim == 2) return launch_sketch_nc<P, 2, kExp>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    return launch_sketch_nc<P, 3, kExp>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
  }
  if (dim == 1) return launch_sketch_nc<P, 1, kGauss>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
  if (dim == 2) return launch_sketch_nc<P, 2, kGauss>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
  return launch_sketch_nc<P, 3, kGauss>(s, n, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
}

// ------------------------------------------------------ kernel block gen

// One workgroup per run of consecutive blocks of a block row (gen_part).  The
// row cluster's coordinates stay in LDS for the whole run.  The run's blocks
// are taken in stages of consecutive blocks
// with at most kGenMax columns together (several small coupling blocks per
// stage, one barrier per stage): thread t fetches the coordinates and output
// offset of stage column t into registers while the current stage is
// evaluated and stashes them into the other of two LDS buffers.  Entry
// (r, column cc of the stage) goes to out[off[cc] + r] (column-major blocks):
// when the threads can be laid out as fixed rows (m * (256/m) of them, at
// least three quarters of the workgroup), thread t keeps row t % m in
// registers and walks stage columns t/m, t/m + 256/m, ..; otherwise the
// threads walk the entries in order.  Consecutive threads write consecutive
// entries; the blocks are written once and read later, so the stores are
// non-temporal.
constexpr int kGenMax = 256;

struct GenStage {
  double v[3];  // this thread's stage column: coordinates
  int64_t off;  // and output offset of its first row
  int jend;     // the stage covers blocks [j, jend)
  int total;    // columns in the stage
};

// The stage that starts at block j: blocks while their columns fit kGenMax;
// thread tid fetches stage column tid.
template <int DIM>
__device__ __forceinline__ void gen_fetch(GenStage& st, const int32_t* __restrict__ idx,
                                          const int32_t* __restrict__ rowoff, const int64_t* __restrict__ blkoff,
                                          const double* __restrict__ X, int64_t ldx, int m, int j, int je, int tid) {
  int total = 0, jj = j;
  int myb = -1, mycol = 0;
  while (jj < je) {
    const int b = idx[jj];
    const int mb = rowoff[b + 1] - rowoff[b];
    if (total + mb > kGenMax && jj > j) break;
    if (tid >= total && tid < total + mb) {
      myb = jj;
      mycol = tid - total;
    }
    total += mb;
    ++jj;
  }
  st.jend = jj;
  st.total = total;
  st.off = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) st.v[a] = 0.0;
  if (myb >= 0) {
    const int c0 = rowoff[idx[myb]] + mycol;
#pragma unroll
    for (int a = 0; a < DIM; ++a) st.v[a] = X[int64_t(a) * ldx + c0];
    st.off = blkoff[myb] + int64_t(mycol) * m;
  }
}

template <int DIM>
__device__ __forceinline__ void gen_stash(const GenStage& st, double (*xc)[kGenMax], int64_t* off, int tid) {
  if (tid < st.total) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) xc[a][tid] = st.v[a];
    off[tid] = st.off;
  }
}

// The block row's blocks [jb, je); f(r2) gives the entry of squared distance r2.
template <int DIM, typename F>
__device__ __forceinline__ void gen_row(const int32_t* __restrict__ idx, const int32_t* __restrict__ rowoff,
                                        const int64_t* __restrict__ blkoff, const double* __restrict__ X,
                                        int64_t ldx, double* __restrict__ out, int jb, int je, int r0, int m,
                                        double (*xr)[kGenMax], double (*xc)[DIM][kGenMax], int64_t (*off)[kGenMax],
                                        F f) {
  const int tid = threadIdx.x;
  for (int e = tid; e < DIM * m; e += 256) xr[e / m][e % m] = X[int64_t(e / m) * ldx + r0 + e % m];
  GenStage st;
  gen_fetch<DIM>(st, idx, rowoff, blkoff, X, ldx, m, jb, je, tid);
  gen_stash<DIM>(st, xc[0], off[0], tid);
  int total = st.total, jn = st.jend;
  __syncthreads();
  const int dc = 256 / m, act = m * dc;
  const bool rows_fixed = act >= 192;
  double rx[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) rx[a] = xr[a][tid % m];
  int cur = 0;
  for (int j = jb; j < je;) {
    const bool more = jn < je;
    if (more) gen_fetch<DIM>(st, idx, rowoff, blkoff, X, ldx, m, jn, je, tid);
    const double(*xcc)[kGenMax] = xc[cur];
    const int64_t* oc = off[cur];
    if (rows_fixed) {
      if (tid < act) {
        const int r = tid % m;
#pragma unroll 4
        for (int c = tid / m; c < total; c += dc) {
          double r2 = 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            const double d = rx[a] - xcc[a][c];
            r2 += d * d;
          }
          __builtin_nontemporal_store(f(r2), out + oc[c] + r);
        }
      }
    } else {
      const int dr = 256 % m;
      int r = tid % m, c = tid / m;
      for (int e = tid; e < m * total; e += 256) {
        double r2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const double d = xr[a][r] - xcc[a][c];
          r2 += d * d;
        }
        __builtin_nontemporal_store(f(r2), out + oc[c] + r);
        r += dr;
        c += dc;
        if (r >= m) {
          r -= m;
          ++c;
        }
      }
    }
    j = jn;
    if (more) {
      gen_stash<DIM>(st, xc[cur ^ 1], off[cur ^ 1], tid);
      total = st.total;
      jn = st.jend;
    }
    __syncthreads();
    cur ^= 1;
  }
}

// A block row's blocks split into `parts` consecutive runs, one workgroup
// each (workgroup b: row b / parts, run b % parts), so that a launch has
// enough workgroups of similar size to fill the chip evenly.
__device__ __forceinline__ void gen_part(const int32_t* __restrict__ ptr, int parts, int& i, int& jb, int& je) {
  i = blockIdx.x / parts;
  const int part = blockIdx.x % parts;
  const int b0 = ptr[i], len = ptr[i + 1] - b0;
  jb = b0 + (len * part) / parts;
  je = b0 + (len * (part + 1)) / parts;
}

// Workgroups per block row of a block generation: about 16384 workgroups in
// all (several per CU at its occupancy), at most 16 per row (measured on the
// 131072-point cube: the leaf near field 3.54 ms with one workgroup per row,
// 3.01 with 4, 2.80 with 8, 2.94 with 16).
int gen_parts(int nrows) { return std::max(1, std::min(16, (16384 + nrows - 1) / std::max(nrows, 1))); }

template <int DIM, int KIND>
__global__ __launch_bounds__(256) void gen_blocks_kernel(const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const int32_t* __restrict__ rowoff,
                                                         const int64_t* __restrict__ blkoff,
                                                         const double* __restrict__ X, int64_t ldx, double c2,
                                                         double* __restrict__ out, int parts) {
  __shared__ double xr[DIM][kGenMax];
  __shared__ double xc[2][DIM][kGenMax];
  __shared__ int64_t off[2][kGenMax];
  int i, jb, je;
  gen_part(ptr, parts, i, jb, je);
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  if (jb == je || m == 0) return;  // uniform over the workgroup
  gen_row<DIM>(idx, rowoff, blkoff, X, ldx, out, jb, je, r0, m, xr, xc, off,
               [c2](double r2) { return kernel_of_r2<KIND>(r2, c2); });
}

// Batched form: block row i belongs to problem rowprob[i] with its own kernel
// kind and exponent scale (points carry 3 coordinates, unused ones zero).
__global__ __launch_bounds__(256) void gen_blocks_batched_kernel(const int32_t* __restrict__ ptr,
                                                                 const int32_t* __restrict__ idx,
                                                                 const int32_t* __restrict__ rowoff,
                                                                 const int64_t* __restrict__ blkoff,
                                                                 const double* __restrict__ X, int64_t ldx,
                                                                 const int32_t* __restrict__ rowprob,
                                                                 const int32_t* __restrict__ kinds,
                                                                 const double* __restrict__ c2s,
                                                                 double* __restrict__ out, int parts) {
  __shared__ double xr[3][kGenMax];
  __shared__ double xc[2][3][kGenMax];
  __shared__ int64_t off[2][kGenMax];
  int i, jb, je;
  gen_part(ptr, parts, i, jb, je);
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  if (jb == je || m == 0) return;  // uniform over the workgroup
  const int pr = rowprob[i];
  const double c2 = c2s[pr];
  if (kinds[pr] == kExp)
    gen_row<3>(idx, rowoff, blkoff, X, ldx, out, jb, je, r0, m, xr, xc, off,
               [c2](double r2) { return kernel_of_r2<kExp>(r2, c2); });
  else
    gen_row<3>(idx, rowoff, blkoff, X, ldx, out, jb, je, r0, m, xr, xc, off,
               [c2](double r2) { return kernel_of_r2<kGauss>(r2, c2); });
}

// ------------------------------------------------------- block-sparse GEMM

// Block-sparse product on the FP64 matrix cores:
//   Y[rows_i, c0:c0+16NB] += alpha * sum_j Blk_j X[rows_b, c0:c0+16NB].
// X is read from a row-major copy Xr (row q at Xr + q*ldr, zero-padded to ldr
// columns), so that one MFMA B operand (4 rows x 16 columns) is four 128-byte
// runs; the blocks (column-major) stream into the A operand (16 rows x 4
// columns, also four 128-byte runs).  One workgroup of four waves per block
// row and 64-row slice of it (blockIdx.z); wave w takes the row's blocks
// w, w+4, .., covering all of the slice's row tiles itself, so the main loop
// has no LDS traffic and no barrier.  The four partial sums are added through
// LDS at the end, one column tile at a time (wave c keeps column tile c).
constexpr int kBsrKu = 4;  // k-steps (4 rows each) per batch of operand loads

// Rows [rz, rz + m) of the block row, m <= 16 L.
template <int NB, bool TR, int L>
__device__ __forceinline__ void bsr_rows(const int32_t* __restrict__ idx, const int32_t* __restrict__ coloff,
                                         const int64_t* __restrict__ tpos, const int64_t* __restrict__ blkoff,
                                         const double* __restrict__ blocks, const double* __restrict__ Xr, int ldr,
                                         double* __restrict__ Y, int64_t ldy, double alpha, int jb, int je, int r0,
                                         int mfull, int rz, int m, int c0, int ncl, dbl4* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  dbl4 acc[L][NB];
#pragma unroll
  for (int t = 0; t < L; ++t)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[t][c] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int j = jb + wave; j < je; j += 4) {
    const int b = idx[j];
    const int q0 = coloff[b], mb = coloff[b + 1] - q0;
    // without TR the block is mfull x mb column-major; with TR it is the
    // transpose of a stored mb x mfull column-major block
    const double* blk = blocks + blkoff[TR ? tpos[j] : j];
    const double* xb = Xr + int64_t(q0) * ldr + c0 + li;
    for (int k0 = 0; k0 < mb; k0 += 4 * kBsrKu) {
      double a[kBsrKu][L], x[kBsrKu][NB];
#pragma unroll
      for (int kc = 0; kc < kBsrKu; ++kc) {
        const int q = k0 + 4 * kc + lk;
        const bool ok = q < mb;
#pragma unroll
        for (int t = 0; t < L; ++t) {
          const int row = rz + t * 16 + li;
          a[kc][t] = (ok && t * 16 + li < m) ? (TR ? blk[int64_t(row) * mb + q] : blk[int64_t(q) * mfull + row]) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) x[kc][c] = ok ? xb[int64_t(q) * ldr + c * 16] : 0.0;
      }
#pragma unroll
      for (int kc = 0; kc < kBsrKu; ++kc)
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
          for (int t = 0; t < L; ++t)
            acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kc][t], x[kc][c], acc[t][c], 0, 0, 0);
    }
  }
  dbl4 fin[L];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
#pragma unroll
    for (int t = 0; t < L; ++t) red[(wave * L + t) * 64 + lane] = acc[t][c];
    __syncthreads();
    if (wave == c) {
#pragma unroll
      for (int t = 0; t < L; ++t) {
        dbl4 sum = red[t * 64 + lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) sum += red[(w * L + t) * 64 + lane];
        fin[t] = sum;
      }
    }
    __syncthreads();
  }
  if (wave < NB) {
    const int col = wave * 16 + li;
    if (col < ncl) {
#pragma unroll
      for (int t = 0; t < L; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = t * 16 + lk + 4 * q;  // MFMA C layout: lane (li, lk) holds rows lk + 4q of column li
          if (row < m) {
            double* yp = Y + int64_t(c0 + col) * ldy + r0 + row;
            *yp += alpha * fin[t][q];
          }
        }
    }
  }
}

// grid (nrows, ceil(nc / 16NB), ceil(max height / 64)); Xr has at least
// gridDim.y * 16NB columns.  Two workgroups per CU by registers.  order
// (optional): workgroup b takes block row order[b], a permutation of the rows
// (longest first balances the launch).
template <int NB, bool TR>
__global__ __launch_bounds__(256, 2) void bsr_gemm_kernel(const int32_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ idx,
                                                          const int32_t* __restrict__ rowoff,
                                                          const int32_t* __restrict__ coloff,
                                                          const int64_t* __restrict__ tpos,
                                                          const int64_t* __restrict__ blkoff,
                                                          const double* __restrict__ blocks,
                                                          const double* __restrict__ Xr, int ldr,
                                                          double* __restrict__ Y, int64_t ldy, int nc, double alpha,
                                                          const int32_t* __restrict__ order) {
  constexpr int LDB = NB * 16;
  __shared__ dbl4 red[4 * 4 * 64];
  const int i = order ? order[blockIdx.x] : blockIdx.x;
  const int mfull = rowoff[i + 1] - rowoff[i];
  const int rz = blockIdx.z * 64;
  const int jb = ptr[i], je = ptr[i + 1];
  if (rz >= mfull || jb == je) return;  // uniform over the workgroup
  const int m = min(64, mfull - rz);
  const int r0 = rowoff[i] + rz;
  const int c0 = blockIdx.y * LDB;
  const int ncl = min(LDB, nc - c0);
#define H2_BSR_ROWS(L) \
  bsr_rows<NB, TR, L>(idx, coloff, tpos, blkoff, blocks, Xr, ldr, Y, ldy, alpha, jb, je, r0, mfull, rz, m, c0, ncl, red)
  switch ((m + 15) >> 4) {
    case 1: H2_BSR_ROWS(1); break;
    case 2: H2_BSR_ROWS(2); break;
    case 3: H2_BSR_ROWS(3); break;
    default: H2_BSR_ROWS(4); break;
  }
#undef H2_BSR_ROWS
}

// Xr[q * ldr + c] = X[c * ldx + q] for q < M, c < nc; zero for nc <= c < ldr.
__global__ __launch_bounds__(256) void to_rows_kernel(int64_t M, int nc, int ldr, const double* __restrict__ X,
                                                      int64_t ldx, double* __restrict__ Xr) {
  __shared__ double tile[64][65];
  const int64_t q0 = int64_t(blockIdx.x) * 64;
  const int c0 = blockIdx.y * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int cc = w; cc < 64; cc += 4) {
    const int c = c0 + cc;
    const int64_t q = q0 + lane;
    tile[cc][lane] = (c < nc && q < M) ? X[int64_t(c) * ldx + q] : 0.0;
  }
  __syncthreads();
  for (int qq = w; qq < 64; qq += 4) {
    const int64_t q = q0 + qq;
    const int c = c0 + lane;
    if (q < M && c < ldr) Xr[q * ldr + c] = tile[lane][qq];
  }
}

// ------------------------------------------------- adaptive convergence test

// Prefix form of the convergence test.  The leading R_ii of a Householder QR
// do not depend on later columns, so one QR over all dsk sketched columns
// gives, for each cluster, the first column count d' = d + j*inc (d = its
// problem's current count) at which it is converged: m <= d' or
// min_{i < d'} |R_ii| < delta.  The problem's count is raised to the largest
// d' over its clusters (atomic max).  A cluster that is not converged at any
// admissible d' <= dsk sets *exhausted.
template <bool kLds>
__global__ void qr_first_conv_kernel(const int32_t* __restrict__ rowoff, const double* __restrict__ Y, int64_t ldy,
                                     int dsk, const int32_t* __restrict__ incprob, const int32_t* __restrict__ ovprob,
                                     const int32_t* __restrict__ nodeprob, int32_t* __restrict__ dprob,
                                     const double* __restrict__ deltaprob, int32_t* __restrict__ exhausted,
                                     double* __restrict__ gws, const int64_t* __restrict__ gws_off) {
  extern __shared__ double smem[];
  __shared__ double s_tau, s_beta;
  const int i = blockIdx.x;
  const int pr = nodeprob[i];
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int dcur = dprob[pr];
  const int inc = incprob[pr];
  const int p = ovprob[pr];
  const double delta = deltaprob[pr];
  // smallest admissible count d' >= x (grid dcur + j*inc), or -1 beyond dsk
  auto grid_at_least = [&](int x) {
    if (x <= dcur) return dcur;
    const int g = dcur + ((x - dcur + inc - 1) / inc) * inc;
    return g <= dsk ? g : -1;
  };
  // first admissible count with every row resolved (m + p <= d')
  const int dfirst = grid_at_least(m + p);
  const int ncols = min(m, dsk - p);  // R_ii tested for i < d' - p <= dsk - p
  if (dfirst == dcur || ncols <= 0) {
    if (tid == 0) {
      if (dfirst < 0) atomicOr(&exhausted[pr], 1);
      else atomicMax(&dprob[pr], dfirst);
    }
    return;
  }
  const int ldp = m | 1;
  double* P = kLds ? smem : gws + gws_off[i];
  // element (r, c) of the panel: column-major with the odd stride ldp in LDS,
  // row-major in the global workspace (threads of consecutive columns touch
  // consecutive addresses)
  const int cs = kLds ? ldp : 1, rs = kLds ? 1 : ncols;
  auto at = [&](int r, int c) -> double& { return P[c * cs + r * rs]; };
  for (int e = tid; e < m * ncols; e += nt) {
    const int r = e % m, c = e / m;
    at(r, c) = Y[int64_t(c) * ldy + r0 + r];
  }
  __syncthreads();
  double mn = INFINITY;
  int found = -1;
  for (int j = 0; j < ncols; ++j) {
    auto pj = [&](int r) -> double& { return at(r, j); };
    if (tid < kWave) {
      double sg = 0.0;
      for (int r = j + 1 + tid; r < m; r += kWave) sg += pj(r) * pj(r);
      sg = wave_sum(sg);
      const double alpha = pj(j);
      double beta, tau, scal;
      if (sg == 0.0) {
        beta = alpha;
        tau = 0.0;
        scal = 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + sg);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      for (int r = j + 1 + tid; r < m; r += kWave) pj(r) *= scal;
      if (tid == 0) {
        s_tau = tau;
        s_beta = beta;
      }
    }
    __syncthreads();
    mn = fmin(mn, fabs(s_beta));
    // a diagonal below delta among the first j+1: converged at the first grid count >= j + 1 + p
    if (mn < delta) {
      found = grid_at_least(j + 1 + p);
      break;
    }
    if (dfirst > 0 && j + 1 + p >= dfirst) break;  // m + p <= d' reached first
    const double tau = s_tau;
    for (int c = j + 1 + tid; c < ncols; c += nt) {
      auto pc = [&](int r) -> double& { return at(r, c); };
      double w0 = pc(j), w1 = 0.0;
      int r = j + 1;
      for (; r + 1 < m; r += 2) {
        w0 += pj(r) * pc(r);
        w1 += pj(r + 1) * pc(r + 1);
      }
      if (r < m) w0 += pj(r) * pc(r);
      const double w = (w0 + w1) * tau;
      pc(j) -= w;
      for (int rr = j + 1; rr < m; ++rr) pc(rr) -= w * pj(rr);
    }
    __syncthreads();
  }
  if (tid == 0) {
    int d = found;
    if (d < 0 || (dfirst > 0 && dfirst < d)) d = dfirst;
    if (d < 0) atomicOr(&exhausted[pr], 1);
    else atomicMax(&dprob[pr], d);
  }
}

// Register-resident form of the same test for panels of m <= 4R rows and at
// most 64 tested columns: thread t of 256 holds rows [qR, qR + R) (q = t & 3)
// of column c = t >> 2 in registers.  Each step's Householder vector goes
// through LDS with zeros above the diagonal, so every thread runs the same
// unrolled loops over its R rows; the four threads of a column (one quad of
// a wave) combine their partial sums by shuffles.  Same reflectors as
// qr_first_conv_kernel (sums of squares in another order).
template <int R>
__global__ __launch_bounds__(256) void qr_conv_reg_kernel(const int32_t* __restrict__ rowoff,
                                                          const double* __restrict__ Y, int64_t ldy, int dsk,
                                                          const int32_t* __restrict__ incprob,
                                                          const int32_t* __restrict__ ovprob,
                                                          const int32_t* __restrict__ nodeprob,
                                                          int32_t* __restrict__ dprob,
                                                          const double* __restrict__ deltaprob,
                                                          int32_t* __restrict__ exhausted) {
  __shared__ double vbuf[4 * R];
  __shared__ double s_tau, s_beta;
  const int i = blockIdx.x;
  const int pr = nodeprob[i];
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int tid = threadIdx.x;
  const int dcur = dprob[pr];
  const int inc = incprob[pr];
  const int p = ovprob[pr];
  const double delta = deltaprob[pr];
  auto grid_at_least = [&](int x) {
    if (x <= dcur) return dcur;
    const int g = dcur + ((x - dcur + inc - 1) / inc) * inc;
    return g <= dsk ? g : -1;
  };
  const int dfirst = grid_at_least(m + p);
  const int ncols = min(m, dsk - p);
  if (dfirst == dcur || ncols <= 0 || m > 4 * R || ncols > 64) {  // uniform; the launcher keeps the bounds
    if (tid == 0 && m <= 4 * R && ncols <= 64) {
      if (dfirst < 0) atomicOr(&exhausted[pr], 1);
      else atomicMax(&dprob[pr], dfirst);
    }
    return;
  }
  const int c = tid >> 2, q = tid & 3, rb = q * R;
  double a[R];
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = (c < ncols && rb + r < m) ? Y[int64_t(c) * ldy + r0 + rb + r] : 0.0;
  double mn = INFINITY;
  int found = -1;
  for (int j = 0; j < ncols; ++j) {
    if (c == j) {
      double sg = 0.0, al = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = rb + r;
        if (row > j) sg += a[r] * a[r];
        if (row == j) al = a[r];
      }
      sg += __shfl_xor(sg, 1);
      sg += __shfl_xor(sg, 2);
      al += __shfl_xor(al, 1);
      al += __shfl_xor(al, 2);
      double beta, tau, scal;
      if (sg == 0.0) {
        beta = al;
        tau = 0.0;
        scal = 0.0;
      } else {
        const double nrm = sqrt(al * al + sg);
        beta = al >= 0.0 ? -nrm : nrm;
        tau = (beta - al) / beta;
        scal = 1.0 / (al - beta);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = rb + r;
        vbuf[row] = row > j ? a[r] * scal : (row == j ? 1.0 : 0.0);
      }
      if (q == 0) {
        s_tau = tau;
        s_beta = beta;
      }
    }
    __syncthreads();
    mn = fmin(mn, fabs(s_beta));
    if (mn < delta) {
      found = grid_at_least(j + 1 + p);
      break;
    }
    if (dfirst > 0 && j + 1 + p >= dfirst) break;  // m + p <= d' reached first
    const double tau = s_tau;
    if (c > j && c < ncols) {
      double v[R];
      double w = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v[r] = vbuf[rb + r];
        w += v[r] * a[r];
      }
      w += __shfl_xor(w, 1);
      w += __shfl_xor(w, 2);
      w *= tau;
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] -= w * v[r];
    }
    __syncthreads();
  }
  if (tid == 0) {
    int d = found;
    if (d < 0 || (dfirst > 0 && dfirst < d)) d = dfirst;
    if (d < 0) atomicOr(&exhausted[pr], 1);
    else atomicMax(&dprob[pr], d);
  }
}

// Blocked form of the same test for panels beyond LDS.  The panel lives
// row-major in the global workspace; kQrNb columns at a time are copied to
// LDS (rows jb.. only) and factored there with the same Householder steps,
// their reflectors are accumulated as H_1..H_nb = I - V T V^T (T upper
// triangular) and applied to the trailing columns as A -= V (T^T (V^T A)):
// two passes over global memory per block instead of one per reflector.
// Only the diagonal of R is used, so the factored block is not written back.
constexpr int kQrNb = 16;

__global__ __launch_bounds__(256, 2) void qr_first_conv_blocked_kernel(
    const int32_t* __restrict__ rowoff, const double* __restrict__ Y, int64_t ldy, int dsk,
    const int32_t* __restrict__ incprob, const int32_t* __restrict__ ovprob, const int32_t* __restrict__ nodeprob,
    int32_t* __restrict__ dprob, const double* __restrict__ deltaprob, int32_t* __restrict__ exhausted,
    double* __restrict__ gws, const int64_t* __restrict__ gws_off) {
  extern __shared__ double smem[];
  __shared__ double s_tau[kQrNb], s_z[kQrNb], s_T[kQrNb * kQrNb];
  __shared__ double s_beta;
  const int i = blockIdx.x;
  const int pr = nodeprob[i];
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int dcur = dprob[pr];
  const int inc = incprob[pr];
  const int p = ovprob[pr];
  const double delta = deltaprob[pr];
  auto grid_at_least = [&](int x) {
    if (x <= dcur) return dcur;
    const int g = dcur + ((x - dcur + inc - 1) / inc) * inc;
    return g <= dsk ? g : -1;
  };
  const int dfirst = grid_at_least(m + p);
  const int ncols = min(m, dsk - p);
  if (dfirst == dcur || ncols <= 0) {
    if (tid == 0) {
      if (dfirst < 0) atomicOr(&exhausted[pr], 1);
      else atomicMax(&dprob[pr], dfirst);
    }
    return;
  }
  double* P = gws + gws_off[i];  // element (r, c) at P[r * ncols + c]
  for (int e = tid; e < m * ncols; e += 256) {
    const int r = e % m, c = e / m;
    P[int64_t(r) * ncols + c] = Y[int64_t(c) * ldy + r0 + r];
  }
  __syncthreads();
  constexpr int ld = kQrNb + 1;
  double* V = smem;  // rows jb..m-1 of the block's columns, (m - jb) x ld
  double mn = INFINITY;
  int found = -1;
  bool stop = false;
  for (int jb = 0; jb < ncols && !stop; jb += kQrNb) {
    const int nb = min(kQrNb, ncols - jb);
    const int mr = m - jb;
    // columns nb.. of V and the rows and columns nb.. of T are zero, so the
    // trailing update needs no bounds on the block width
    for (int e = tid; e < mr * kQrNb; e += 256) {
      const int r = e / kQrNb, cl = e % kQrNb;
      V[r * ld + cl] = cl < nb ? P[int64_t(jb + r) * ncols + jb + cl] : 0.0;
    }
    for (int e = tid; e < kQrNb * kQrNb; e += 256) s_T[e] = 0.0;
    __syncthreads();
    // factor the block's columns in LDS
    for (int jl = 0; jl < nb; ++jl) {
      const int j = jb + jl;
      if (wave == 0) {
        double sg = 0.0;
        for (int r = jl + 1 + lane; r < mr; r += kWave) sg += V[r * ld + jl] * V[r * ld + jl];
        sg = wave_sum(sg);
        const double alpha = V[jl * ld + jl];
        double beta, tau, scal;
        if (sg == 0.0) {
          beta = alpha;
          tau = 0.0;
          scal = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + sg);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        for (int r = jl + 1 + lane; r < mr; r += kWave) V[r * ld + jl] *= scal;
        if (lane == 0) {
          s_tau[jl] = tau;
          s_beta = beta;
        }
      }
      __syncthreads();
      mn = fmin(mn, fabs(s_beta));
      if (mn < delta) {
        found = grid_at_least(j + 1 + p);
        stop = true;
        break;
      }
      if (dfirst > 0 && j + 1 + p >= dfirst) {
        stop = true;
        break;
      }
      const double tau = s_tau[jl];
      for (int cl = jl + 1 + wave; cl < nb; cl += 4) {
        double w = 0.0;
        for (int r = jl + 1 + lane; r < mr; r += kWave) w += V[r * ld + jl] * V[r * ld + cl];
        w = (wave_sum(w) + V[jl * ld + cl]) * tau;
        for (int r = jl + 1 + lane; r < mr; r += kWave) V[r * ld + cl] -= w * V[r * ld + jl];
        if (lane == 0) V[jl * ld + cl] -= w;
      }
      __syncthreads();
    }
    if (stop || jb + nb >= ncols) break;  // uniform: s_beta and the counts are shared
    // T: T_ll = tau_l, T[0:l, l] = -tau_l T[0:l, 0:l] (V[:, 0:l]^T v_l)
    for (int l = 0; l < nb; ++l) {
      for (int a = wave; a < l; a += 4) {
        double z = 0.0;
        for (int r = l + 1 + lane; r < mr; r += kWave) z += V[r * ld + a] * V[r * ld + l];
        z = wave_sum(z) + V[l * ld + a];  // v_l is 1 at row l, zero above
        if (lane == 0) s_z[a] = z;
      }
      __syncthreads();
      if (tid == 0) {
        const double tl = s_tau[l];
        for (int a = 0; a < l; ++a) {
          double acc = 0.0;
          for (int b = a; b < l; ++b) acc += s_T[a * kQrNb + b] * s_z[b];
          s_T[a * kQrNb + l] = -tl * acc;
        }
        s_T[l * kQrNb + l] = tl;
      }
      __syncthreads();
    }
    // trailing columns: A -= V (T^T (V^T A)), one thread per column; rows
    // below kQrNb hold only V's dense part, rows above it its unit triangle
    const int rt = min(mr, kQrNb);
    for (int c = jb + nb + tid; c < ncols; c += 256) {
      double w[kQrNb];
#pragma unroll
      for (int l = 0; l < kQrNb; ++l) w[l] = 0.0;
#pragma unroll 1
      for (int r = 0; r < rt; ++r) {
        const double a = P[int64_t(jb + r) * ncols + c];
#pragma unroll
        for (int l = 0; l < kQrNb; ++l) w[l] += (r > l ? V[r * ld + l] : (r == l ? 1.0 : 0.0)) * a;
      }
#pragma unroll 2
      for (int r = kQrNb; r < mr; ++r) {
        const double a = P[int64_t(jb + r) * ncols + c];
#pragma unroll
        for (int l = 0; l < kQrNb; ++l) w[l] += V[r * ld + l] * a;
      }
      // w <- T^T w in place (descending: column l of T only reads w[0..l]);
      // the empty asm keeps T's LDS reads here instead of in registers for
      // the whole loop
      asm volatile("" ::: "memory");
#pragma unroll
      for (int l = kQrNb - 1; l >= 0; --l) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a <= l; ++a) acc += s_T[a * kQrNb + l] * w[a];
        w[l] = acc;
      }
#pragma unroll 1
      for (int r = 0; r < rt; ++r) {
        double a = P[int64_t(jb + r) * ncols + c];
#pragma unroll
        for (int l = 0; l < kQrNb; ++l) a -= (r > l ? V[r * ld + l] : (r == l ? 1.0 : 0.0)) * w[l];
        P[int64_t(jb + r) * ncols + c] = a;
      }
#pragma unroll 2
      for (int r = kQrNb; r < mr; ++r) {
        double a = P[int64_t(jb + r) * ncols + c];
#pragma unroll
        for (int l = 0; l < kQrNb; ++l) a -= V[r * ld + l] * w[l];
        P[int64_t(jb + r) * ncols + c] = a;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    int d = found;
    if (d < 0 || (dfirst > 0 && dfirst < d)) d = dfirst;
    if (d < 0) atomicOr(&exhausted[pr], 1);
    else atomicMax(&dprob[pr], d);
  }
}

// Exclusive scan of n int32 -> out[0..n] (out[n] = total), one workgroup.
__global__ __launch_bounds__(1024) void scan_kernel(int n, const int32_t* __restrict__ in, int32_t* __restrict__ out) {
  __shared__ int32_t part[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < n ? in[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) out[i] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// dst[i] = src[map[i]] for i <= n (n + 1 entries).
__global__ __launch_bounds__(256) void gather_i32_kernel(int n, const int32_t* __restrict__ map,
                                                         const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) dst[i] = src[map[i]];
}

// Per problem p (one workgroup each): nu = ||Y[base, n rows, d0 cols]||_F / sqrt(d0),
// delta = tol * nu / sqrt(#leaves) (mode 0) or tol * nu (mode 1); d = d0.
struct ThresholdJob {
  int64_t base, n;
  int32_t d0, nleaves, mode, pad;
  double tol;
};

__global__ __launch_bounds__(256) void threshold_kernel(const ThresholdJob* __restrict__ jobs,
                                                        const double* __restrict__ Y, int64_t ldy,
                                                        double* __restrict__ nu, double* __restrict__ delta,
                                                        int32_t* __restrict__ d) {
  __shared__ double red[4];
  const ThresholdJob J = jobs[blockIdx.x];
  double acc = 0.0;
  for (int c = 0; c < J.d0; ++c) {
    const double* y = Y + int64_t(c) * ldy + J.base;
    for (int64_t r = threadIdx.x; r < J.n; r += 256) acc += y[r] * y[r];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ss = (red[0] + red[1]) + (red[2] + red[3]);
    const double v = sqrt(ss) / sqrt(double(J.d0));
    nu[blockIdx.x] = v;
    delta[blockIdx.x] = J.mode == 0 ? J.tol * v / sqrt(double(J.nleaves)) : J.tol * v;
    d[blockIdx.x] = J.d0;
  }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = v;
}

// ---------------------------------------------------------------- CPQR / ID

// Column-pivoted Householder QR of A = Y_loc^T (d x m) held in the panel with
// leading dimension lda = d | 1; thread c owns column c (a row of Y_loc).
// Pivot = largest partial norm (ties -> lowest original column), norms are
// downdated and recomputed once they lose about half their digits.  Truncates
// at the first |R_jj| < delta.  Then T = R11^{-1} R12 by back substitution and
// U (m x k) = rows J identity, other rows T^T.
struct PivotCand {
  double v;
  int piv;
  int pos;
};

__device__ __forceinline__ bool better(const PivotCand& a, const PivotCand& b) {
  return a.v > b.v || (a.v == b.v && a.piv < b.piv);
}

__device__ __forceinline__ PivotCand wave_best(PivotCand c) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    PivotCand o;
    o.v = __shfl_xor(c.v, off, kWave);
    o.piv = __shfl_xor(c.piv, off, kWave);
    o.pos = __shfl_xor(c.pos, off, kWave);
    if (better(o, c)) c = o;
  }
  return c;
}

template <bool kLds>
__global__ __launch_bounds__(256) void cpqr_id_kernel(const int32_t* __restrict__ rowoff, const double* __restrict__ Y,
                                                      int64_t ldy, int d, double delta, int32_t* __restrict__ kout,
                                                      int32_t* __restrict__ Jout, const int64_t* __restrict__ joff,
                                                      double* __restrict__ Uout, const int64_t* __restrict__ uoff,
                                                      double* __restrict__ gws, const int64_t* __restrict__ gws_off,
                                                      const int32_t* __restrict__ nodeprob,
                                                      const int32_t* __restrict__ dprob,
                                                      const double* __restrict__ deltaprob) {
  if (nodeprob) {  // batched: the column count and threshold of the cluster's problem
    d = dprob[nodeprob[blockIdx.x]];
    delta = deltaprob[nodeprob[blockIdx.x]];
  }
  extern __shared__ double smem[];
  __shared__ PivotCand s_best[4];
  __shared__ double s_tau, s_scal;
  __shared__ int s_p, s_stop;
  const int i = blockIdx.x;
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int lda = d | 1;
  // LDS layout: vn1[m], vn2[m], piv[m] (as int in a double slot), panel
  double* vn1 = smem;
  double* vn2 = smem + m;
  int* piv = reinterpret_cast<int*>(smem + 2 * m);
  double* A = kLds ? smem + 3 * m : gws + gws_off[i];
  // element (r, c) of the panel: column-major with the odd stride lda in LDS
  // (a thread per column, no bank conflicts), row-major in the global
  // workspace, so that the threads of consecutive columns touch consecutive
  // addresses
  const int cs = kLds ? lda : 1, rs = kLds ? 1 : m;
  auto at = [&](int r, int c) -> double& { return A[c * cs + r * rs]; };

  for (int e = tid; e < m * d; e += nt) {
    const int c = e % m, r = e / m;
    at(r, c) = Y[int64_t(r) * ldy + r0 + c];
  }
  __syncthreads();
  for (int c = tid; c < m; c += nt) {
    double s = 0.0;
    for (int r = 0; r < d; ++r) s += at(r, c) * at(r, c);
    vn1[c] = sqrt(s);
    vn2[c] = vn1[c];
    piv[c] = c;
  }
  if (tid == 0) s_stop = 0;
  __syncthreads();

  const int kmax = min(m, d);
  int k = kmax;
  const double tol3z = 1.4901161193847656e-08;  // sqrt(2^-52)
  for (int j = 0; j < kmax; ++j) {
    // pivot selection
    PivotCand best{-1.0, 0x7fffffff, -1};
    for (int c = j + tid; c < m; c += nt) {
      PivotCand cand{vn1[c], piv[c], c};
      if (better(cand, best)) best = cand;
    }
    best = wave_best(best);
    if (lane == 0) s_best[wave] = best;
    __syncthreads();
    if (tid == 0) {
      PivotCand b = s_best[0];
      for (int w = 1; w < nw; ++w)
        if (better(s_best[w], b)) b = s_best[w];
      s_p = b.pos >= j ? b.pos : j;  // NaN norms never win a comparison: keep column j
    }
    __syncthreads();
    const int p = s_p;
    if (p != j) {
      for (int r = tid; r < d; r += nt) {
        const double t = at(r, j);
        at(r, j) = at(r, p);
        at(r, p) = t;
      }
      if (tid == 0) {
        double t = vn1[j];
        vn1[j] = vn1[p];
        vn1[p] = t;
        t = vn2[j];
        vn2[j] = vn2[p];
        vn2[p] = t;
        const int ti = piv[j];
        piv[j] = piv[p];
        piv[p] = ti;
      }
      __syncthreads();
    }
    // Householder reflector of column j, rows j..d-1
    auto aj = [&](int r) -> double& { return at(r, j); };
    if (wave == 0) {
      double sg = 0.0;
      for (int r = j + 1 + lane; r < d; r += kWave) sg += aj(r) * aj(r);
      sg = wave_sum(sg);
      const double alpha = aj(j);
      double beta, tau, scal;
      if (sg == 0.0) {
        beta = alpha;
        tau = 0.0;
        scal = 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + sg);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      if (lane == 0) {
        s_tau = tau;
        s_scal = scal;
        if (fabs(beta) < delta || beta == 0.0) s_stop = 1;
      }
      // make sure every lane has read alpha before lane 0 overwrites it
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) aj(j) = beta;
    }
    __syncthreads();
    if (s_stop) {
      k = j;
      break;
    }
    {
      const double scal = s_scal;
      for (int r = j + 1 + tid; r < d; r += nt) aj(r) *= scal;
    }
    __syncthreads();
    const double tau = s_tau;
    for (int c = j + 1 + tid; c < m; c += nt) {
      auto ac = [&](int r) -> double& { return at(r, c); };
      double w0 = ac(j), w1 = 0.0;
      int r = j + 1;
      for (; r + 1 < d; r += 2) {
        w0 += aj(r) * ac(r);
        w1 += aj(r + 1) * ac(r + 1);
      }
      if (r < d) w0 += aj(r) * ac(r);
      const double w = (w0 + w1) * tau;
      ac(j) -= w;
      for (int rr = j + 1; rr < d; ++rr) ac(rr) -= w * aj(rr);
      // norm downdate with recompute safeguard
      if (vn1[c] != 0.0) {
        double t = fabs(ac(j)) / vn1[c];
        t = fmax(0.0, 1.0 - t * t);
        const double ratio = vn1[c] / vn2[c];
        const double t2 = t * ratio * ratio;
        if (t2 <= tol3z) {
          double s = 0.0;
          for (int rr = j + 1; rr < d; ++rr) s += ac(rr) * ac(rr);
          vn1[c] = sqrt(s);
          vn2[c] = vn1[c];
        } else {
          vn1[c] = vn1[c] * sqrt(t);
        }
      }
    }
    __syncthreads();
  }

  // T = R11^{-1} R12, in place in rows 0..k-1 of the redundant columns
  for (int c = k + tid; c < m; c += nt) {
    auto ac = [&](int r) -> double& { return at(r, c); };
    for (int r = k - 1; r >= 0; --r) {
      double s = ac(r);
      for (int l = r + 1; l < k; ++l) s -= at(r, l) * ac(l);
      ac(r) = s / at(r, r);
    }
  }
  __syncthreads();
  if (tid == 0) kout[i] = k;
  for (int r = tid; r < k; r += nt) Jout[joff[i] + r] = piv[r];
  double* U = Uout + uoff[i];
  for (int c = tid; c < m; c += nt) {
    const int q = piv[c];
    for (int r = 0; r < k; ++r) U[q + int64_t(r) * m] = (c < k) ? (c == r ? 1.0 : 0.0) : at(r, c);
  }
}

// Register-resident form of the same ID for panels that fit one wave: d <= D
// rows (samples) and m <= 64 C columns (points).  Lane l holds columns l,
// l + 64, .. of A = Y_loc^T with their D rows unrolled in registers, so a
// Householder step is straight-line FP64 arithmetic: the pivot lane copies its
// column to LDS, every lane reads it back (broadcast reads, a block of 16 rows
// at a time ahead of the arithmetic) and updates its own columns and
// downdates their norms.  Rows are visited in blocks of 16 with one uniform
// branch per block (blocks above the step are skipped, the block holding the
// step masks its rows).
// The reflector is applied to every column: on a column already chosen as a
// pivot (rows below its position are zero up to rounding) and on an empty
// lane it changes nothing of use.  Pivoting, ties (lowest original column),
// the norm downdating with its recompute guard, the stopping rule and the
// triangular solve T = R11^-1 R12 (column-oriented back substitution, R11 read
// from the pivot lanes) follow cpqr_id_kernel; the order of the sums differs.
constexpr int kIdRb = 16;  // rows per block of the unrolled row loops

template <int D, int C>
__global__ __launch_bounds__(64) void cpqr_id_wave_kernel(const int32_t* __restrict__ rowoff,
                                                          const double* __restrict__ Y, int64_t ldy, int d,
                                                          double delta, int32_t* __restrict__ kout,
                                                          int32_t* __restrict__ Jout, const int64_t* __restrict__ joff,
                                                          double* __restrict__ Uout, const int64_t* __restrict__ uoff,
                                                          const int32_t* __restrict__ nodeprob,
                                                          const int32_t* __restrict__ dprob,
                                                          const double* __restrict__ deltaprob) {
  static_assert(D % kIdRb == 0, "row blocks");
  __shared__ int s_col[64];     // original column of pivot position l
  __shared__ double s_piv[D];   // the column broadcast to every lane (pivot, or R11 column l)
  const int i = blockIdx.x;
  if (nodeprob) {
    d = dprob[nodeprob[i]];
    delta = deltaprob[nodeprob[i]];
  }
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int lane = threadIdx.x;
  double a[C][D], vn1[C], vn2[C];
  int pos[C];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int col = lane + 64 * s;
    const bool act = col < m;
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      a[s][r] = (act && r < d) ? Y[int64_t(r) * ldy + r0 + col] : 0.0;
      ss = __builtin_fma(a[s][r], a[s][r], ss);
    }
    vn1[s] = sqrt(ss);
    vn2[s] = vn1[s];
    pos[s] = act ? -1 : -2;  // -1: candidate column, -2: no column, >= 0: pivot position
  }
  // the column of slot ps in lane pl, copied to LDS for broadcast reads
  auto publish = [&](int pl, int ps) {
    __syncthreads();
    if (lane == pl) {
      double2* dst = reinterpret_cast<double2*>(s_piv);
#pragma unroll
      for (int r = 0; r < D; r += 2)
        dst[r / 2] = (C == 1 || ps == 0) ? double2{a[0][r], a[0][r + 1]} : double2{a[C - 1][r], a[C - 1][r + 1]};
    }
    __syncthreads();
  };
  // rows rb..rb+15 of the published column, read ahead of their use
  auto pblock = [&](int rb, double* t) {
    const double2* src = reinterpret_cast<const double2*>(s_piv + rb);
#pragma unroll
    for (int q = 0; q < kIdRb / 2; ++q) {
      const double2 v = src[q];
      t[2 * q] = v.x;
      t[2 * q + 1] = v.y;
    }
  };
  const int kmax = min(m, d);
  int k = kmax;
  const double tol3z = 1.4901161193847656e-08;  // sqrt(2^-52)
  for (int j = 0; j < kmax; ++j) {
    // pivot: largest partial norm, ties to the lowest column (NaN norms rank last)
    double bv = -2.0;
    int bc = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int col = lane + 64 * s;
      const double v = __builtin_isnan(vn1[s]) ? -1.0 : vn1[s];
      if (pos[s] == -1 && (v > bv || (v == bv && col < bc))) {
        bv = v;
        bc = col;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, kWave);
      const int oc = __shfl_xor(bc, off, kWave);
      if (ov > bv || (ov == bv && oc < bc)) {
        bv = ov;
        bc = oc;
      }
    }
    const int p = __builtin_amdgcn_readfirstlane(bc);
    const int pl = p & 63, ps = p >> 6;
    publish(pl, ps);
    // one pass over the rows >= j: the pivot's alpha = a_p[j] and
    // sg = sum_{r > j} a_p[r]^2, and each column's a[j] and sum_{r > j} a_p[r] a[r]
    double alpha = 0.0, sg = 0.0, aj[C], dot[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      aj[s] = 0.0;
      dot[s] = 0.0;
    }
#pragma unroll
    for (int rb = 0; rb < D; rb += kIdRb) {
      if (rb + kIdRb <= j) continue;
      double tv[kIdRb];
      pblock(rb, tv);
      if (rb > j) {
#pragma unroll
        for (int r = rb; r < rb + kIdRb; ++r) {
          const double t = tv[r - rb];
          sg = __builtin_fma(t, t, sg);
#pragma unroll
          for (int s = 0; s < C; ++s) dot[s] = __builtin_fma(t, a[s][r], dot[s]);
        }
      } else {
#pragma unroll
        for (int r = rb; r < rb + kIdRb; ++r) {
          const double t = tv[r - rb];
          const bool below = r > j;
          sg = below ? __builtin_fma(t, t, sg) : sg;
          if (r == j) alpha = t;
#pragma unroll
          for (int s = 0; s < C; ++s) {
            dot[s] = below ? __builtin_fma(t, a[s][r], dot[s]) : dot[s];
            if (r == j) aj[s] = a[s][r];
          }
        }
      }
    }
    double beta, tau, scal;
    if (sg == 0.0) {
      beta = alpha;
      tau = 0.0;
      scal = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sg);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (fabs(beta) < delta || beta == 0.0) {
      k = j;
      break;
    }
    // H = I - tau v v^T with v = (1, scal a_p[j+1..]):  w = tau (a[j] + scal dot)
    double w[C], sw[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      w[s] = tau * __builtin_fma(scal, dot[s], aj[s]);
      sw[s] = w[s] * scal;
    }
    // a[j] -= w, a[r] -= (w scal) a_p[r] for r > j; the new trailing norms^2
    double ajn[C], s2[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      ajn[s] = aj[s] - w[s];
      s2[s] = 0.0;
    }
#pragma unroll
    for (int rb = 0; rb < D; rb += kIdRb) {
      if (rb + kIdRb <= j) continue;
      double tv[kIdRb];
      pblock(rb, tv);
      if (rb > j) {
#pragma unroll
        for (int r = rb; r < rb + kIdRb; ++r) {
          const double t = tv[r - rb];
#pragma unroll
          for (int s = 0; s < C; ++s) {
            a[s][r] = __builtin_fma(-sw[s], t, a[s][r]);
            s2[s] = __builtin_fma(a[s][r], a[s][r], s2[s]);
          }
        }
      } else {
#pragma unroll
        for (int r = rb; r < rb + kIdRb; ++r) {
          const bool below = r > j;
          const double t = below ? tv[r - rb] : 0.0;
#pragma unroll
          for (int s = 0; s < C; ++s) {
            if (r == j) a[s][r] = ajn[s];
            a[s][r] = __builtin_fma(-sw[s], t, a[s][r]);
            s2[s] = below ? __builtin_fma(a[s][r], a[s][r], s2[s]) : s2[s];
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
      if (lane == pl && s == ps) {
        pos[s] = j;
      } else if (pos[s] == -1 && vn1[s] != 0.0) {
        // norm downdate with the recompute safeguard (s2 = exact trailing norm^2)
        double t = fabs(ajn[s]) / vn1[s];
        t = fmax(0.0, 1.0 - t * t);
        const double ratio = vn1[s] / vn2[s];
        if (t * ratio * ratio <= tol3z) {
          vn1[s] = sqrt(s2[s]);
          vn2[s] = vn1[s];
        } else {
          vn1[s] = vn1[s] * sqrt(t);
        }
      }
    }
    if (lane == 0) s_col[j] = p;
  }
  __syncthreads();
  // T = R11^-1 R12 in place in rows 0..k-1 of the non-pivot columns, one
  // pivot column l = k-1..0 at a time; R11(r, l) comes from the pivot lane,
  // whose registers the solve leaves untouched (its multiplier t is 0)
  for (int l = k - 1; l >= 0; --l) {
    const int pc = s_col[l];
    const int pl = pc & 63, ps = pc >> 6;
    publish(pl, ps);
    double t[C];
#pragma unroll
    for (int s = 0; s < C; ++s) t[s] = 0.0;
#pragma unroll
    for (int rb = D - kIdRb; rb >= 0; rb -= kIdRb) {
      if (rb > l) continue;
      double tv[kIdRb];
      pblock(rb, tv);
      if (rb + kIdRb <= l) {
#pragma unroll
        for (int r = rb; r < rb + kIdRb; ++r) {
          const double rrl = tv[r - rb];
#pragma unroll
          for (int s = 0; s < C; ++s) a[s][r] = __builtin_fma(-rrl, t[s], a[s][r]);
        }
      } else {
#pragma unroll
        for (int r = rb + kIdRb - 1; r >= rb; --r) {
          if (r == l) {
            const double inv = 1.0 / tv[r - rb];
#pragma unroll
            for (int s = 0; s < C; ++s) {
              if (pos[s] == -1) {
                t[s] = a[s][r] * inv;
                a[s][r] = t[s];
              }
            }
          } else {
            const double rrl = r < l ? tv[r - rb] : 0.0;
#pragma unroll
            for (int s = 0; s < C; ++s) a[s][r] = __builtin_fma(-rrl, t[s], a[s][r]);
          }
        }
      }
    }
  }
  if (lane == 0) kout[i] = k;
  double* U = Uout + uoff[i];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int col = lane + 64 * s;
    if (pos[s] == -2) continue;
    if (pos[s] >= 0) Jout[joff[i] + pos[s]] = col;
#pragma unroll
    for (int r = 0; r < D; ++r)
      if (r < k) U[col + int64_t(r) * m] = pos[s] >= 0 ? (r == pos[s] ? 1.0 : 0.0) : a[s][r];
  }
}

// ------------------------------------------------------ shrink / upsweep

// W(k0 + r, c) = sum_q U_i(q, r) Win(r0 + q, c) on the FP64 matrix cores: the
// node's U (m x k, column-major) and a 64-column slice of Win are staged
// through LDS 16 rows (q) at a time, so that both are read along their
// contiguous dimension; each wave accumulates up to TPW 16 x 16 output tiles
// (tile t of the slice's ceil(k/16) x ceil(w/16) goes to wave t mod 4).
// Yout(k0 + r, c) = Yloc(r0 + J[r], c) as in shrink_up_kernel.
constexpr int kShrMaxK = 256;
constexpr int kShrLdu = kShrMaxK + 2;
constexpr int kShrLdw = 64 + 2;
template <int TPW>
__global__ __launch_bounds__(256) void shrink_up_mfma_kernel(
    const int32_t* __restrict__ rowoff, const int32_t* __restrict__ koff, const int32_t* __restrict__ J,
    const int64_t* __restrict__ joff, const double* __restrict__ U, const int64_t* __restrict__ uoff,
    const double* __restrict__ Yloc, int64_t ldyl, const double* __restrict__ Win, int64_t ldwi,
    double* __restrict__ Yout, int64_t ldyo, double* __restrict__ Wout, int64_t ldwo, int nc) {
  __shared__ double Us[16 * kShrLdu];
  __shared__ double Ws[16 * kShrLdw];
  const int i = blockIdx.x;
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int k0 = koff[i], k = koff[i + 1] - k0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (Yloc) {
    const int* Ji = J + joff[i];
    for (int e = tid; e < k * nc; e += blockDim.x) {
      const int r = e % k, c = e / k;
      Yout[int64_t(c) * ldyo + k0 + r] = Yloc[int64_t(c) * ldyl + r0 + Ji[r]];
    }
  }
  if (!Win || k == 0 || k > kShrMaxK) return;  // uniform; k <= d <= 256 by construction
  const double* Ui = U + uoff[i];
  const int RT = (k + 15) >> 4;
  // tiles beyond 4 x TPW are taken by further passes over the panel
  for (int c0 = 0, t0 = 0; c0 < nc;) {
    const int w = min(64, nc - c0);
    const int CT = (w + 15) >> 4, ntiles = RT * CT;
    dbl4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < m; q0 += 16) {
      __syncthreads();
      for (int e = tid; e < 16 * k; e += 256) {
        const int qq = e & 15, r = e >> 4;
        Us[qq * kShrLdu + r] = q0 + qq < m ? Ui[q0 + qq + int64_t(r) * m] : 0.0;
      }
      for (int e = tid; e < 16 * w; e += 256) {
        const int qq = e & 15, c = e >> 4;
        Ws[qq * kShrLdw + c] = q0 + qq < m ? Win[int64_t(c0 + c) * ldwi + r0 + q0 + qq] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = kk * 4 + lk;
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          const int t = t0 + wave + 4 * u;
          if (t < ntiles) {
            const int rt = t / CT, ct = t - rt * CT;
            // rows r >= k and columns c >= w of the staged panels hold stale
            // values; they reach only output rows and columns that are not written
            const double a = Us[q * kShrLdu + rt * 16 + li];
            const double b = Ws[q * kShrLdw + ct * 16 + li];
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int t = t0 + wave + 4 * u;
      if (t < ntiles) {
        const int rt = t / CT, ct = t - rt * CT;
        const int c = ct * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = rt * 16 + lk + 4 * q;
          if (r < k && c < w) Wout[int64_t(c0 + c) * ldwo + k0 + r] = acc[u][q];
        }
      }
    }
    t0 += 4 * TPW;
    if (t0 >= ntiles) {
      t0 = 0;
      c0 += 64;
    }
  }
}

__global__ __launch_bounds__(256) void shrink_up_kernel(const int32_t* __restrict__ rowoff,
                                                        const int32_t* __restrict__ koff,
                                                        const int32_t* __restrict__ J,
                                                        const int64_t* __restrict__ joff,
                                                        const double* __restrict__ U,
                                                        const int64_t* __restrict__ uoff,
                                                        const double* __restrict__ Yloc, int64_t ldyl,
                                                        const double* __restrict__ Win, int64_t ldwi,
                                                        double* __restrict__ Yout, int64_t ldyo,
                                                        double* __restrict__ Wout, int64_t ldwo, int nc) {
  const int i = blockIdx.x;
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int k0 = koff[i], k = koff[i + 1] - k0;
  const int* Ji = J + joff[i];
  const double* Ui = U + uoff[i];
  for (int e = threadIdx.x; e < k * nc; e += blockDim.x) {
    const int r = e % k, c = e / k;
    if (Yloc) Yout[int64_t(c) * ldyo + k0 + r] = Yloc[int64_t(c) * ldyl + r0 + Ji[r]];
    if (!Win) continue;
    const double* u = Ui + int64_t(r) * m;
    const double* w = Win + int64_t(c) * ldwi + r0;
    double s0 = 0.0, s1 = 0.0;
    int q = 0;
    for (; q + 1 < m; q += 2) {
      s0 += u[q] * w[q];
      s1 += u[q + 1] * w[q + 1];
    }
    if (q < m) s0 += u[q] * w[q];
    Wout[int64_t(c) * ldwo + k0 + r] = s0 + s1;
  }
}

__global__ __launch_bounds__(256) void expand_kernel(const int32_t* __restrict__ rowoff, const int32_t* __restrict__ koff,
                                                     const double* __restrict__ U, const int64_t* __restrict__ uoff,
                                                     const double* __restrict__ Yh, int64_t ldh,
                                                     double* __restrict__ Yt, int64_t ldt, int nc) {
  const int i = blockIdx.x;
  const int r0 = rowoff[i], m = rowoff[i + 1] - r0;
  const int k0 = koff[i], k = koff[i + 1] - k0;
  const double* Ui = U + uoff[i];
  for (int e = threadIdx.x; e < m * nc; e += blockDim.x) {
    const int q = e % m, c = e / m;
    const double* h = Yh + int64_t(c) * ldh + k0;
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += Ui[q + int64_t(r) * m] * h[r];
    Yt[int64_t(c) * ldt + r0 + q] += s;
  }
}

__global__ __launch_bounds__(256) void skeleton_kernel(const int32_t* __restrict__ rowoff,
                                                       const int32_t* __restrict__ koff,
                                                       const int32_t* __restrict__ J,
                                                       const int64_t* __restrict__ joff,
                                                       const int32_t* __restrict__ pos_in,
                                                       int32_t* __restrict__ pos_out, int dim,
                                                       const double* __restrict__ X, int64_t ldx,
                                                       double* __restrict__ Xs, int64_t ldxs) {
  const int i = blockIdx.x;
  const int r0 = rowoff[i];
  const int k0 = koff[i], k = koff[i + 1] - k0;
  for (int r = threadIdx.x; r < k; r += blockDim.x) {
    const int row = r0 + J[joff[i] + r];
    const int pos = pos_in ? pos_in[row] : row;
    pos_out[k0 + r] = pos;
    for (int a = 0; a < dim; ++a) Xs[a * ldxs + k0 + r] = X[a * ldx + pos];
  }
}

__global__ __launch_bounds__(256) void permute_rows_kernel(int64_t n, const int32_t* __restrict__ idx, int scatter,
                                                           const double* __restrict__ src, int64_t lds,
                                                           double* __restrict__ dst, int64_t ldd, int nc) {
  // grid (row blocks, columns): no integer division per element
  const int64_t c = blockIdx.y;
  for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
    if (scatter)
      dst[c * ldd + idx[p]] = src[c * lds + p];
    else
      dst[c * ldd + p] = src[c * lds + idx[p]];
  }
}

__global__ __launch_bounds__(256) void sumsq_kernel(int64_t n, int nc, const double* __restrict__ A, int64_t lda,
                                                    double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t total = n * nc;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    const double v = A[(e / n) * lda + e % n];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = 0.0;
}

// ------------------------------------------------ low-rank update A = H + U V^T
// The update keeps the dense leaf blocks of H and adds the low-rank term
// U_s V_b^T of each near pair through these factored products; all row
// indices are tree positions.

// W_b (r x nc, column-major, ld r, at b*r*nc) = V(leaf b rows, :)^T X(leaf b rows, :).
// One workgroup per leaf: 32-row slices of V and X are staged in LDS and each
// thread accumulates a 4 x 4 tile of W_b (64 x 64 per pass over q, nc <= 64).
constexpr int kLrRows = 32;

__global__ __launch_bounds__(256) void lr_leaf_project_kernel(const int32_t* __restrict__ leafoff,
                                                              const double* __restrict__ V, int64_t ldv, int r,
                                                              const double* __restrict__ X, int64_t ldx, int nc,
                                                              double* __restrict__ W) {
  __shared__ double sv[kLrRows][64 + 1], sx[kLrRows][64 + 1];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int r0 = leafoff[b], m = leafoff[b + 1] - r0;
  double* Wb = W + int64_t(b) * r * nc;
  const int tq = (tid & 15) * 4, tc = (tid >> 4) * 4;
  for (int q0 = 0; q0 < r; q0 += 64) {
    const int qn = min(64, r - q0);
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int p0 = 0; p0 < m; p0 += kLrRows) {
      const int pn = min(kLrRows, m - p0);
      __syncthreads();
      for (int e = tid; e < kLrRows * 64; e += 256) {
        const int p = e % kLrRows, q = e / kLrRows;
        sv[p][q] = (p < pn && q < qn) ? V[int64_t(q0 + q) * ldv + r0 + p0 + p] : 0.0;
        sx[p][q] = (p < pn && q < nc) ? X[int64_t(q) * ldx + r0 + p0 + p] : 0.0;
      }
      __syncthreads();
      for (int p = 0; p < pn; ++p) {
        double v[4], x[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          v[a] = sv[p][tq + a];
          x[a] = sx[p][tc + a];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[a][c] += v[a] * x[c];
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (tq + a < qn && tc + c < nc) Wb[(q0 + tq + a) + int64_t(tc + c) * r] = acc[a][c];
  }
}

// partial[g][e] = sum of W_b[e] over the 64 leaves b of group g (fixed order).
__global__ __launch_bounds__(256) void lr_sum_partial_kernel(int nleaves, int len, const double* __restrict__ W,
                                                             double* __restrict__ partial) {
  const int g = blockIdx.y;
  const int b0 = g * 64, b1 = min(nleaves, b0 + 64);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int b = b0; b < b1; ++b) acc += W[int64_t(b) * len + e];
    partial[int64_t(g) * len + e] = acc;
  }
}

__global__ __launch_bounds__(256) void lr_sum_final_kernel(int ngroups, int len, const double* __restrict__ partial,
                                                           double* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int g = 0; g < ngroups; ++g) acc += partial[int64_t(g) * len + e];
    out[e] = acc;
  }
}

// Near-field low-rank term: Y(leaf s rows, :) += alpha U(leaf s rows, :) sum_{b in N_s} W_b.
// Global form (ptr == nullptr): Y(all n rows) += alpha U W_0, rows split over workgroups.
__global__ __launch_bounds__(256) void lr_apply_kernel(const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ idx,
                                                       const int32_t* __restrict__ leafoff, int64_t n,
                                                       const double* __restrict__ U, int64_t ldu, int r,
                                                       const double* __restrict__ W, int nc, double* __restrict__ Y,
                                                       int64_t ldy, double alpha) {
  extern __shared__ double S[];  // r x nc
  const int len = r * nc;
  int64_t r0, m;
  if (ptr) {
    const int s = blockIdx.x;
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
      double acc = 0.0;
      for (int j = ptr[s]; j < ptr[s + 1]; ++j) acc += W[int64_t(idx[j]) * len + e];
      S[e] = acc;
    }
    r0 = leafoff[s];
    m = leafoff[s + 1] - r0;
  } else {
    for (int e = threadIdx.x; e < len; e += blockDim.x) S[e] = W[e];
    r0 = int64_t(blockIdx.x) * 256;
    m = min(int64_t(256), n - r0);
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < m * nc; e += blockDim.x) {
    const int64_t row = e % m;
    const int c = static_cast<int>(e / m);
    double acc = 0.0;
    for (int q = 0; q < r; ++q) acc += U[int64_t(q) * ldu + r0 + row] * S[q + c * r];
    Y[int64_t(c) * ldy + r0 + row] += alpha * acc;
  }
}

// Rows of the old nested basis at the new skeletons (basis-row extraction):
//   R_i = U_old_i(J_i, :)                                   at the leaves,
//   R_i(a, :) = R_nu(jj, :) U_old_i(off_nu + (0..ko_nu-1), :)   at inner clusters,
// where the in-row J_i[a] of the new ID lies in child nu at its row jj, and
// off_nu is the first row of nu's block in the old transfer matrix
// [E_nu1; E_nu2].  R_i has k_i rows at koff[i] (ld ldr) and ko_i columns.
__global__ __launch_bounds__(256) void basis_rows_kernel(int leaf, const int32_t* __restrict__ koff,
                                                         const int32_t* __restrict__ J,
                                                         const int64_t* __restrict__ joff,
                                                         const int32_t* __restrict__ kold_off,
                                                         const int32_t* __restrict__ kold_child_off,
                                                         const int32_t* __restrict__ leafoff,
                                                         const double* __restrict__ Uold,
                                                         const int64_t* __restrict__ uoff_old,
                                                         const int32_t* __restrict__ koff_child,
                                                         const double* __restrict__ Rc, int64_t ldrc,
                                                         double* __restrict__ R, int64_t ldr) {
  const int i = blockIdx.x;
  const int k0 = koff[i], k = koff[i + 1] - k0;
  const int ko = kold_off[i + 1] - kold_off[i];
  const int* Ji = J + joff[i];
  const double* Ui = Uold + uoff_old[i];
  if (leaf) {
    const int m = leafoff[i + 1] - leafoff[i];
    for (int e = threadIdx.x; e < k * ko; e += blockDim.x) {
      const int a = e % k, c = e / k;
      R[int64_t(c) * ldr + k0 + a] = Ui[int64_t(c) * m + Ji[a]];
    }
    return;
  }
  const int c1 = 2 * i, c2 = 2 * i + 1;
  const int kn1 = koff_child[c2] - koff_child[c1];
  const int ko1 = kold_child_off[c2] - kold_child_off[c1];
  const int ko2 = kold_child_off[c2 + 1] - kold_child_off[c2];
  const int mo = ko1 + ko2;
  for (int e = threadIdx.x; e < k * ko; e += blockDim.x) {
    const int a = e % k, c = e / k;
    const int row = Ji[a];
    const bool first = row < kn1;
    const int nu = first ? c1 : c2, jj = first ? row : row - kn1, off = first ? 0 : ko1, kon = first ? ko1 : ko2;
    const double* rc = Rc + koff_child[nu] + jj;
    const double* u = Ui + int64_t(c) * mo + off;
    double acc = 0.0;
    for (int q = 0; q < kon; ++q) acc += rc[int64_t(q) * ldrc] * u[q];
    R[int64_t(c) * ldr + k0 + a] = acc;
  }
}

// Coupling of the update at an admissible pair (s, b):
//   B_new = R_r_s B_old(s, b) R_c_b^T + U(skel_r_s, :) V(skel_c_b, :)^T
// (k_r_s x k_c_b, column-major at boff_new[j]).  Ug and Vg hold the rows of U
// and V at the level's row and column skeletons (gathered once per level, in
// skeleton order).  One workgroup per pair, on the FP64 matrix cores, 32
// output columns at a time:
//   T      = B_old(s, b) R_c_b(cols)^T              (k_old_s x 32, in LDS)
//   B_new  = [R_r_s | Ug_s] [T ; Vg_b(cols)^T]        (inner dim k_old_s + r)
// Wave w owns the 16-row tiles w, w+4, ... of each product and both 16-column
// tiles of the chunk, so every A operand it loads feeds two MFMAs and the
// waves share the tiles evenly.
// f64 16x16x4: lane l supplies A[l%16][l/16], B[l/16][l%16]; D[l/16 + 4q][l%16].
constexpr int kCuCols = 32;
constexpr int kCuMaxK = 128;
constexpr int kCuLdt = kCuCols + 8;
__global__ __launch_bounds__(256) void coupling_update_kernel(
    const int32_t* __restrict__ frow, const int32_t* __restrict__ fidx, const int32_t* __restrict__ koff_r,
    const int32_t* __restrict__ koff_c, const int32_t* __restrict__ kold_off, const double* __restrict__ Bold,
    const int64_t* __restrict__ boff_old, const double* __restrict__ Rr, int64_t ldrr,
    const double* __restrict__ Rc, int64_t ldrc, const double* __restrict__ Ug, int64_t ldug,
    const double* __restrict__ Vg, int64_t ldvg, int r, double* __restrict__ Bnew,
    const int64_t* __restrict__ boff_new) {
  __shared__ double T[kCuMaxK * kCuLdt];
  const int j = blockIdx.x;
  const int s = frow[j], b = fidx[j];
  const int kr0 = koff_r[s], kr = koff_r[s + 1] - kr0;
  const int kc0 = koff_c[b], kc = koff_c[b + 1] - kc0;
  const int kos = kold_off[s + 1] - kold_off[s];
  const int kob = kold_off[b + 1] - kold_off[b];
  if (kr == 0 || kc == 0) return;  // uniform
  const double* bo = Bold + boff_old[j];
  double* out = Bnew + boff_new[j];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int kin = kos + r;
  const int mt1 = (kos + 15) / 16, mt2 = (kr + 15) / 16;
  for (int c0 = 0; c0 < kc; c0 += kCuCols) {
    const int w = min(kCuCols, kc - c0);
    // ---- T = B_old R_c^T for the chunk's columns
    for (int t = wave; t < mt1; t += 4) {
      const int m = t * 16 + li;
      dbl4 acc[2] = {dbl4{0.0, 0.0, 0.0, 0.0}, dbl4{0.0, 0.0, 0.0, 0.0}};
      for (int k0 = 0; k0 < kob; k0 += 4) {
        const int k = k0 + lk;
        const double a = (m < kos && k < kob) ? bo[m + int64_t(k) * kos] : 0.0;
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
          const int col = tn * 16 + li;
          const double bv = (col < w && k < kob) ? Rc[(kc0 + c0 + col) + int64_t(k) * ldrc] : 0.0;
          acc[tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[tn], 0, 0, 0);
        }
      }
#pragma unroll
      for (int tn = 0; tn < 2; ++tn)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = t * 16 + lk + 4 * q;
          if (row < kos) T[row * kCuLdt + tn * 16 + li] = acc[tn][q];
        }
    }
    __syncthreads();
    // ---- B_new(:, chunk) = [R_r | Ug] [T ; Vg^T]
    for (int t = wave; t < mt2; t += 4) {
      const int m = t * 16 + li;
      dbl4 acc[2] = {dbl4{0.0, 0.0, 0.0, 0.0}, dbl4{0.0, 0.0, 0.0, 0.0}};
      for (int k0 = 0; k0 < kin; k0 += 4) {
        const int k = k0 + lk;
        double a = 0.0;
        if (m < kr && k < kin)
          a = k < kos ? Rr[(kr0 + m) + int64_t(k) * ldrr] : Ug[(kr0 + m) + int64_t(k - kos) * ldug];
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
          const int col = tn * 16 + li;
          double bv = 0.0;
          if (col < w && k < kin)
            bv = k < kos ? T[k * kCuLdt + col] : Vg[(kc0 + c0 + col) + int64_t(k - kos) * ldvg];
          acc[tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[tn], 0, 0, 0);
        }
      }
#pragma unroll
      for (int tn = 0; tn < 2; ++tn)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = t * 16 + lk + 4 * q;
          const int col = tn * 16 + li;
          if (row < kr && col < w) out[int64_t(c0 + col) * kr + row] = acc[tn][q];
        }
    }
    __syncthreads();
  }
}

// The same coupling update in 64-column chunks with only T in LDS (kos x
// kCu2Ld doubles of dynamic LDS, so that several pairs share a CU): T =
// B_old R_c^T for the chunk, then [R_r | Ug] [T ; Vg^T].  Each wave keeps up
// to two 16-row tiles and the chunk's 16-column tiles in registers, and the
// contraction runs in batches of four 4-deep steps whose loads are all issued
// before their matrix-core products, so that a pair waits for memory once
// per batch rather than once per step.  Only the chunk's column tiles are
// computed.
constexpr int kCu2Ld = 64 + 2;
constexpr int kCu2Kb = 4;  // 4-deep steps per batch
__global__ __launch_bounds__(256) void coupling_update2_kernel(
    const int32_t* __restrict__ frow, const int32_t* __restrict__ fidx, const int32_t* __restrict__ koff_r,
    const int32_t* __restrict__ koff_c, const int32_t* __restrict__ kold_off, const double* __restrict__ Bold,
    const int64_t* __restrict__ boff_old, const double* __restrict__ Rr, int64_t ldrr,
    const double* __restrict__ Rc, int64_t ldrc, const double* __restrict__ Ug, int64_t ldug,
    const double* __restrict__ Vg, int64_t ldvg, int r, double* __restrict__ Bnew,
    const int64_t* __restrict__ boff_new) {
  extern __shared__ double T[];
  const int j = blockIdx.x;
  const int s = frow[j], b = fidx[j];
  const int kr0 = koff_r[s], kr = koff_r[s + 1] - kr0;
  const int kc0 = koff_c[b], kc = koff_c[b + 1] - kc0;
  const int kos = kold_off[s + 1] - kold_off[s];
  const int kob = kold_off[b + 1] - kold_off[b];
  if (kr == 0 || kc == 0) return;  // uniform
  const double* bo = Bold + boff_old[j];
  double* out = Bnew + boff_new[j];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int kin = kos + r;
  const int mt1 = (kos + 15) >> 4, RT = (kr + 15) >> 4;
  for (int c0 = 0; c0 < kc; c0 += 64) {
    const int w = min(64, kc - c0), CT = (w + 15) >> 4;
    __syncthreads();  // the previous chunk's products have read T
    // ---- T = B_old R_c^T (tile (rt, ct) to wave (rt * CT + ct) mod 4)
    for (int t = wave; t < mt1 * CT; t += 4) {
      const int rt = t / CT, ct = t - rt * CT;
      const int m = rt * 16 + li, col = ct * 16 + li;
      dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < kob; k0 += 4 * kCu2Kb) {
        double a[kCu2Kb], bv[kCu2Kb];
#pragma unroll
        for (int kb = 0; kb < kCu2Kb; ++kb) {
          const int k = k0 + 4 * kb + lk;
          a[kb] = (m < kos && k < kob) ? bo[m + int64_t(k) * kos] : 0.0;
          bv[kb] = (col < w && k < kob) ? Rc[(kc0 + c0 + col) + int64_t(k) * ldrc] : 0.0;
        }
#pragma unroll
        for (int kb = 0; kb < kCu2Kb; ++kb) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kb], bv[kb], acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rt * 16 + lk + 4 * q;
        if (row < kos) T[row * kCu2Ld + col] = acc[q];
      }
    }
    __syncthreads();
    // ---- B_new(:, chunk) = [R_r | Ug] [T ; Vg^T], 8 row tiles per pass
    for (int rt0 = 0; rt0 < RT; rt0 += 8) {
      dbl4 acc[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[u][ct] = dbl4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < kin; k0 += 4 * kCu2Kb) {
        double a[kCu2Kb][2], bv[kCu2Kb][4];
#pragma unroll
        for (int kb = 0; kb < kCu2Kb; ++kb) {
          const int k = k0 + 4 * kb + lk;
          const bool kok = k < kin;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const int col = ct * 16 + li;
            double v = 0.0;
            if (ct < CT && kok)
              v = k < kos ? T[k * kCu2Ld + col] : (col < w ? Vg[(kc0 + c0 + col) + int64_t(k - kos) * ldvg] : 0.0);
            bv[kb][ct] = v;
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int m = (rt0 + wave + 4 * u) * 16 + li;
            double v = 0.0;
            if (m < kr && kok) v = k < kos ? Rr[(kr0 + m) + int64_t(k) * ldrr] : Ug[(kr0 + m) + int64_t(k - kos) * ldug];
            a[kb][u] = v;
          }
        }
#pragma unroll
        for (int kb = 0; kb < kCu2Kb; ++kb)
#pragma unroll
          for (int u = 0; u < 2; ++u)
            if (rt0 + wave + 4 * u < RT)
#pragma unroll
              for (int ct = 0; ct < 4; ++ct)
                if (ct < CT) acc[u][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kb][u], bv[kb][ct], acc[u][ct], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int rt = rt0 + wave + 4 * u;
        if (rt < RT)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const int col = ct * 16 + li;
            if (ct < CT)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = rt * 16 + lk + 4 * q;
                if (row < kr && col < w) out[int64_t(c0 + col) * kr + row] = acc[u][ct][q];
              }
          }
      }
    }
  }
}

// Dense blocks of the update, written out: out_j = D_j + U(rows s, :) V(rows b, :)^T.
__global__ __launch_bounds__(256) void dense_lowrank_kernel(const int32_t* __restrict__ ptr,
                                                            const int32_t* __restrict__ idx,
                                                            const int32_t* __restrict__ leafoff,
                                                            const int64_t* __restrict__ blkoff,
                                                            const double* __restrict__ Din,
                                                            const double* __restrict__ U, int64_t ldu,
                                                            const double* __restrict__ V, int64_t ldv, int r,
                                                            double* __restrict__ out) {
  const int s = blockIdx.x;
  const int r0 = leafoff[s], m = leafoff[s + 1] - r0;
  for (int j = ptr[s]; j < ptr[s + 1]; ++j) {
    const int b = idx[j];
    const int q0 = leafoff[b], mb = leafoff[b + 1] - q0;
    for (int e = threadIdx.x; e < m * mb; e += blockDim.x) {
      const int row = e % m, c = e / m;
      double lr = 0.0;
      for (int q = 0; q < r; ++q) lr += U[int64_t(q) * ldu + r0 + row] * V[int64_t(q) * ldv + q0 + c];
      out[blkoff[j] + e] = Din[blkoff[j] + e] + lr;
    }
  }
}

unsigned grid_for(int64_t work, int64_t per_block = 256, unsigned cap = 65536) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

// Dynamic LDS above 64 KB needs the per-kernel attribute; prepare_kernels()
// sets it once for every kernel that can ask for it, so launches (including
// those recorded into a graph) make no further runtime calls.
size_t g_lds_prepared = 0;

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536 || bytes <= g_lds_prepared) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

}  // namespace

// ================================================================ launchers

hipError_t gaussian(hipStream_t s, uint64_t seed, int64_t nrows, const int32_t* rows, int64_t col0, int ncols,
                    double* out, int64_t ldo) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  gaussian_kernel<<<grid_for(nrows * ncols), 256, 0, s>>>(seed, nrows, rows, col0, ncols, out, ldo, nullptr, nullptr);
  return hipGetLastError();
}

size_t sketch_sym_scratch_bytes(int64_t n) {
  if (n <= kSkRows) return 0;
  const int64_t tiles = (n + kSkRows - 1) / kSkRows;
  return size_t(sym_slot(tiles - 1, n)) * 64 * sizeof(double);
}

namespace {

template <int DIM, int KIND>
void launch_sketch_sym_k(hipStream_t s, int64_t n, const double* X, int64_t ldx, double c2, int ncr,
                         const double* om, int64_t ldo, double* y, int64_t ldy, double* z) {
  const unsigned tiles = static_cast<unsigned>((n + kSkRows - 1) / kSkRows);
  sketch_sym_f64_kernel<DIM, KIND><<<tiles, 256, 0, s>>>(n, X, ldx, c2, ncr, om, ldo, y, ldy, z);
  if (tiles > 1) sketch_sym_reduce_kernel<<<static_cast<unsigned>((n + 63) / 64), 256, 0, s>>>(n, ncr, z, y, ldy);
}

hipError_t sketch_sym(hipStream_t s, int64_t n, int dim, const double* X, int64_t ldx, KernelFn k, int ncols,
                      const double* omega, int64_t ldo, double* y, int64_t ldy, double* given) {
  const double c2 = kernel_c2(k);
  const size_t bytes = sketch_sym_scratch_bytes(n);
  double* z = given;
  double* own = nullptr;
  if (bytes > 0 && !z) {
    const hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&own), bytes, s);
    if (e != hipSuccess) return e;
    z = own;
  }
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int nc = ncols - c0 < 64 ? ncols - c0 : 64;
    const double* om = omega + int64_t(c0) * ldo;
    double* yy = y + int64_t(c0) * ldy;
#define H2_SYM(D, K) launch_sketch_sym_k<D, K>(s, n, X, ldx, c2, nc, om, ldo, yy, ldy, z)
    if (k.kind == kExp) {
      if (dim == 1) H2_SYM(1, kExp);
      else if (dim == 2) H2_SYM(2, kExp);
      else H2_SYM(3, kExp);
    } else if (k.kind == kHelm) {
      if (dim == 1) H2_SYM(1, kHelm);
      else if (dim == 2) H2_SYM(2, kHelm);
      else H2_SYM(3, kHelm);
    } else {
      if (dim == 1) H2_SYM(1, kGauss);
      else if (dim == 2) H2_SYM(2, kGauss);
      else H2_SYM(3, kGauss);
    }
#undef H2_SYM
  }
  hipError_t e = hipGetLastError();
  if (own) {
    const hipError_t f = hipFreeAsync(own, s);
    if (e == hipSuccess) e = f;
  }
  return e;
}

}  // namespace

hipError_t sketch(hipStream_t s, int precision, int64_t n, int dim, const double* X, int64_t ldx, KernelFn k,
                  int ncols, const double* omega, int64_t ldo, double* y, int64_t ldy, double* sym_scratch) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (precision < 0 || precision > 5) return hipErrorInvalidValue;
  if (k.kind == kHelm && precision != 0 && precision != 5) return hipErrorInvalidValue;
  if (precision == 5) return sketch_sym(s, n, dim, X, ldx, k, ncols, omega, ldo, y, ldy, sym_scratch);
  const double c2 = kernel_c2(k);
  // split-bf16 modes: Omega is split once per launch into stream-ordered scratch
  const int S = precision == 2 ? 2 : (precision == 4 ? 3 : 0);
  const int64_t npairs = (n + 1) / 2;
  uint32_t* w = nullptr;
  if (S > 0) {
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&w), size_t(S) * 64 * size_t(npairs) * sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipSuccess;
  for (int c0 = 0; c0 < ncols && e == hipSuccess; c0 += 64) {
    const int nc = ncols - c0 < 64 ? ncols - c0 : 64;
    const double* om = omega + int64_t(c0) * ldo;
    double* yy = y + int64_t(c0) * ldy;
    if (S > 0) {
      const int64_t total = int64_t(nc) * npairs;
      const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 65535));
      if (S == 2)
        split_omega_kernel<2><<<blocks, 256, 0, s>>>(n, nc, om, ldo, npairs, w);
      else
        split_omega_kernel<3><<<blocks, 256, 0, s>>>(n, nc, om, ldo, npairs, w);
      e = hipGetLastError();
      if (e != hipSuccess) break;
    }
    if (precision == 0)
      e = launch_sketch_p<0>(s, n, dim, k.kind, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    else if (precision == 1)
      e = launch_sketch_p<1>(s, n, dim, k.kind, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    else if (precision == 2)
      e = launch_sketch_p<2>(s, n, dim, k.kind, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    else if (precision == 3)
      e = launch_sketch_p<3>(s, n, dim, k.kind, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
    else
      e = launch_sketch_p<4>(s, n, dim, k.kind, X, ldx, c2, nc, om, ldo, w, npairs, yy, ldy);
  }
  if (w) {
    const hipError_t f = hipFreeAsync(w, s);
    if (e == hipSuccess) e = f;
  }
  return e;
}

hipError_t gen_blocks(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                      const int64_t* blkoff, int dim, const double* X, int64_t ldx, KernelFn k, double* out) {
  if (nrows <= 0) return hipSuccess;
  const double c2 = kernel_c2(k);
  const int parts = gen_parts(nrows);
#define H2_GEN(D, K) \
  gen_blocks_kernel<D, K><<<nrows * parts, 256, 0, s>>>(ptr, idx, rowoff, blkoff, X, ldx, c2, out, parts)
  if (k.kind == kExp) {
    if (dim == 1) H2_GEN(1, kExp);
    else if (dim == 2) H2_GEN(2, kExp);
    else H2_GEN(3, kExp);
  } else if (k.kind == kHelm) {
    if (dim == 1) H2_GEN(1, kHelm);
    else if (dim == 2) H2_GEN(2, kHelm);
    else H2_GEN(3, kHelm);
  } else {
    if (dim == 1) H2_GEN(1, kGauss);
    else if (dim == 2) H2_GEN(2, kGauss);
    else H2_GEN(3, kGauss);
  }
#undef H2_GEN
  return hipGetLastError();
}

template <int NB, bool TR>
void launch_bsr_nb(hipStream_t s, dim3 grid, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                   const int32_t* coloff, const int64_t* tpos, const int64_t* blkoff, const double* blocks,
                   const double* Xr, int ldr, double* Y, int64_t ldy, int nc, double alpha, const int32_t* order) {
  bsr_gemm_kernel<NB, TR><<<grid, 256, 0, s>>>(ptr, idx, rowoff, coloff, tpos, blkoff, blocks, Xr, ldr, Y, ldy, nc,
                                               alpha, order);
}

// 16-column groups per workgroup for nc columns and a tile width of tile_cols.
static int bsr_groups(int nc, int tile_cols) {
  const int cap = tile_cols >= 16 && tile_cols <= 64 ? tile_cols / 16 : 4;
  return std::min(cap, (nc + 15) / 16);
}

size_t bsr_scratch_doubles(int64_t ldx, int nc, int tile_cols) {
  const int nb = std::max(1, bsr_groups(nc, tile_cols));
  const int ldr = ((nc + 16 * nb - 1) / (16 * nb)) * 16 * nb;
  return size_t(ldx) * ldr;
}

hipError_t bsr_gemm2(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                     const int32_t* coloff, const int64_t* tpos, const int64_t* blkoff, const double* blocks,
                     const double* X, int64_t ldx, double* Y, int64_t ldy, int nc, double alpha, int max_m,
                     double* scratch, size_t scratch_doubles, int tile_cols, const int32_t* order) {
  if (nrows <= 0 || nc <= 0 || ldx <= 0) return hipSuccess;
  if (tile_cols != 16 && tile_cols != 32 && tile_cols != 48 && tile_cols != 64) return hipErrorInvalidValue;
  if (max_m < 1) max_m = 1;
  const int nb = bsr_groups(nc, tile_cols);
  const int ngrp = (nc + 16 * nb - 1) / (16 * nb);
  const int ldr = ngrp * 16 * nb;
  const size_t need = size_t(ldx) * ldr;
  double* xr = scratch;
  if (!xr || scratch_doubles < need) return hipErrorInvalidValue;
  const dim3 tgrid(unsigned((ldx + 63) / 64), unsigned((ldr + 63) / 64));
  to_rows_kernel<<<tgrid, 256, 0, s>>>(ldx, nc, ldr, X, ldx, xr);
  const dim3 grid(nrows, ngrp, (max_m + 63) / 64);
#define H2_BSR_NB(NB)                                                                                               \
  (tpos ? launch_bsr_nb<NB, true>(s, grid, ptr, idx, rowoff, coloff, tpos, blkoff, blocks, xr, ldr, Y, ldy, nc, alpha, \
                                  order)                                                                             \
        : launch_bsr_nb<NB, false>(s, grid, ptr, idx, rowoff, coloff, tpos, blkoff, blocks, xr, ldr, Y, ldy, nc, alpha, \
                                   order))
  switch (nb) {
    case 1: H2_BSR_NB(1); break;
    case 2: H2_BSR_NB(2); break;
    case 3: H2_BSR_NB(3); break;
    default: H2_BSR_NB(4); break;
  }
#undef H2_BSR_NB
  return hipGetLastError();
}

hipError_t bsr_gemm(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                    const int64_t* blkoff, const double* blocks, const double* X, int64_t ldx, double* Y,
                    int64_t ldy, int nc, double alpha, int max_m, double* scratch, size_t scratch_doubles,
                    int tile_cols, const int32_t* order) {
  return bsr_gemm2(s, nrows, ptr, idx, rowoff, rowoff, nullptr, blkoff, blocks, X, ldx, Y, ldy, nc, alpha, max_m,
                   scratch, scratch_doubles, tile_cols, order);
}

hipError_t cpqr_id(hipStream_t s, int nnodes, const int32_t* rowoff, const double* Y, int64_t ldy, int d,
                   double delta, int32_t* kout, int32_t* J, const int64_t* joff, double* U, const int64_t* uoff,
                   int max_m, size_t lds_limit, double* gws, const int64_t* gws_off, const int32_t* nodeprob,
                   const int32_t* dprob, const double* deltaprob) {
  if (nnodes <= 0) return hipSuccess;
  // panels that fit one wave's registers: d <= 64 rows, m <= 128 columns
  if (d <= 64 && max_m <= 128) {
#define H2_CPQR_WAVE(DD, CC) \
  cpqr_id_wave_kernel<DD, CC><<<nnodes, 64, 0, s>>>(rowoff, Y, ldy, d, delta, kout, J, joff, U, uoff, nodeprob, dprob, deltaprob)
    if (max_m <= 64) {
      if (d <= 32)
        H2_CPQR_WAVE(32, 1);
      else
        H2_CPQR_WAVE(64, 1);
    } else {
      if (d <= 32)
        H2_CPQR_WAVE(32, 2);
      else
        H2_CPQR_WAVE(64, 2);
    }
#undef H2_CPQR_WAVE
    return hipGetLastError();
  }
  const int threads = max_m <= 64 ? 64 : (max_m <= 128 ? 128 : 256);
  const size_t small = size_t(3) * max_m * sizeof(double);
  const size_t bytes = small + size_t(d | 1) * size_t(max_m) * sizeof(double);
  if (bytes <= lds_limit) {
    hipError_t e = allow_lds(cpqr_id_kernel<true>, bytes);
    if (e != hipSuccess) return e;
    cpqr_id_kernel<true><<<nnodes, threads, bytes, s>>>(rowoff, Y, ldy, d, delta, kout, J, joff, U, uoff, gws,
                                                        gws_off, nodeprob, dprob, deltaprob);
  } else {
    if (!gws || !gws_off) return hipErrorInvalidValue;
    hipError_t e = allow_lds(cpqr_id_kernel<false>, small);
    if (e != hipSuccess) return e;
    cpqr_id_kernel<false><<<nnodes, threads, small, s>>>(rowoff, Y, ldy, d, delta, kout, J, joff, U, uoff, gws,
                                                         gws_off, nodeprob, dprob, deltaprob);
  }
  return hipGetLastError();
}

hipError_t shrink_up(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const int32_t* J,
                     const int64_t* joff, const double* U, const int64_t* uoff, const double* Yloc, int64_t ldyl,
                     const double* Win, int64_t ldwi, double* Yout, int64_t ldyo, double* Wout, int64_t ldwo,
                     int nc, int kmax) {
  if (nnodes <= 0 || nc <= 0) return hipSuccess;
  if (kmax < 0 || kmax > kShrMaxK) return hipErrorInvalidValue;
  if (!Win) {  // gather only
    shrink_up_kernel<<<nnodes, 256, 0, s>>>(rowoff, koff, J, joff, U, uoff, Yloc, ldyl, Win, ldwi, Yout, ldyo, Wout,
                                            ldwo, nc);
    return hipGetLastError();
  }
  const int tiles = ((kmax + 15) / 16) * ((std::min(nc, 64) + 15) / 16);
#define H2_SHR(T)                                                                                                    shrink_up_mfma_kernel<T><<<nnodes, 256, 0, s>>>(rowoff, koff, J, joff, U, uoff, Yloc, ldyl, Win, ldwi, Yout, ldyo,                                                   Wout, ldwo, nc)
  if (tiles <= 16)
    H2_SHR(4);
  else if (tiles <= 32)
    H2_SHR(8);
  else
    H2_SHR(16);
#undef H2_SHR
  return hipGetLastError();
}

hipError_t expand(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const double* U,
                  const int64_t* uoff, const double* Yh, int64_t ldh, double* Yt, int64_t ldt, int nc) {
  if (nnodes <= 0 || nc <= 0) return hipSuccess;
  expand_kernel<<<nnodes, 256, 0, s>>>(rowoff, koff, U, uoff, Yh, ldh, Yt, ldt, nc);
  return hipGetLastError();
}

hipError_t skeleton(hipStream_t s, int nnodes, const int32_t* rowoff, const int32_t* koff, const int32_t* J,
                    const int64_t* joff, const int32_t* pos_in, int32_t* pos_out, int dim, const double* X,
                    int64_t ldx, double* Xs, int64_t ldxs) {
  if (nnodes <= 0) return hipSuccess;
  skeleton_kernel<<<nnodes, 64, 0, s>>>(rowoff, koff, J, joff, pos_in, pos_out, dim, X, ldx, Xs, ldxs);
  return hipGetLastError();
}

hipError_t permute_rows(hipStream_t s, int64_t n, const int32_t* idx, bool scatter, const double* src, int64_t lds,
                        double* dst, int64_t ldd, int nc) {
  if (n <= 0 || nc <= 0) return hipSuccess;
  if (nc > 65535) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536)), static_cast<unsigned>(nc));
  permute_rows_kernel<<<grid, 256, 0, s>>>(n, idx, scatter ? 1 : 0, src, lds, dst, ldd, nc);
  return hipGetLastError();
}

hipError_t sumsq_partial(hipStream_t s, int64_t n, int nc, const double* A, int64_t lda, double* partial,
                         int nblocks) {
  sumsq_kernel<<<nblocks, 256, 0, s>>>(n, nc, A, lda, partial);
  return hipGetLastError();
}

hipError_t fill_zero(hipStream_t s, double* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  fill_zero_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t gaussian_batched(hipStream_t s, int64_t nrows, const int32_t* rows, const int32_t* rowprob,
                            const uint64_t* seeds, int64_t col0, int ncols, double* out, int64_t ldo) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  gaussian_kernel<<<grid_for(nrows * ncols), 256, 0, s>>>(0, nrows, rows, col0, ncols, out, ldo, rowprob, seeds);
  return hipGetLastError();
}

hipError_t sketch_batched(hipStream_t s, int precision, int ntiles, const void* jobs, const int32_t* tiles,
                          const double* X, int64_t ldx, int ncols, const double* omega, int64_t ldo, double* y,
                          int64_t ldy, int chunk_cols) {
  if (ntiles <= 0 || ncols <= 0) return hipSuccess;
  if (chunk_cols != 16 && chunk_cols != 32 && chunk_cols != 48 && chunk_cols != 64) return hipErrorInvalidValue;
  const SketchJob* J = static_cast<const SketchJob*>(jobs);
  for (int c0 = 0; c0 < ncols; c0 += chunk_cols) {
    const int nc = ncols - c0 < chunk_cols ? ncols - c0 : chunk_cols;
    const double* om = omega + int64_t(c0) * ldo;
    double* yy = y + int64_t(c0) * ldy;
#define H2_SKB(K, NCT) K<NCT><<<ntiles, 256, 0, s>>>(J, tiles, X, ldx, nc, om, ldo, yy, ldy)
#define H2_SKB_S(NCT, S) sketch_bf16_batched<NCT, S><<<ntiles, 256, 0, s>>>(J, tiles, X, ldx, nc, om, ldo, yy, ldy)
#define H2_SKB_NC_S(S)                 \
  if (nc <= 16) H2_SKB_S(16, S);      \
  else if (nc <= 32) H2_SKB_S(32, S); \
  else if (nc <= 48) H2_SKB_S(48, S); \
  else H2_SKB_S(64, S);
#define H2_SKB_NC(K)               \
  if (nc <= 16) H2_SKB(K, 16);      \
  else if (nc <= 32) H2_SKB(K, 32); \
  else if (nc <= 48) H2_SKB(K, 48); \
  else H2_SKB(K, 64);
    if (precision == 0) {
      H2_SKB_NC(sketch_f64_batched)
    } else if (precision == 1) {
      H2_SKB_NC(sketch_f32_batched)
    } else if (precision == 2) {
      H2_SKB_NC_S(2)
    } else if (precision == 3) {
      H2_SKB_NC(sketch_e32_batched)
    } else if (precision == 4) {
      H2_SKB_NC_S(3)
    } else {
      return hipErrorInvalidValue;
    }
#undef H2_SKB_NC_S
#undef H2_SKB_S
#undef H2_SKB_NC
#undef H2_SKB
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t sketch_job_bytes() { return sizeof(SketchJob); }
size_t threshold_job_bytes() { return sizeof(ThresholdJob); }

void pack_sketch_job(void* dst, int64_t n, int64_t base, int kind, double scale) {
  SketchJob j{};
  j.n = n;
  j.base = base;
  j.c2 = -scale * kLog2e;
  j.kind = kind;
  *static_cast<SketchJob*>(dst) = j;
}

void pack_threshold_job(void* dst, int64_t base, int64_t n, int d0, int nleaves, int mode, double tol) {
  ThresholdJob j{};
  j.base = base;
  j.n = n;
  j.d0 = d0;
  j.nleaves = nleaves;
  j.mode = mode;
  j.tol = tol;
  *static_cast<ThresholdJob*>(dst) = j;
}

hipError_t gen_blocks_batched(hipStream_t s, int nrows, const int32_t* ptr, const int32_t* idx, const int32_t* rowoff,
                              const int64_t* blkoff, const double* X, int64_t ldx, const int32_t* rowprob,
                              const int32_t* kinds, const double* c2s, double* out) {
  if (nrows <= 0) return hipSuccess;
  const int parts = gen_parts(nrows);
  gen_blocks_batched_kernel<<<nrows * parts, 256, 0, s>>>(ptr, idx, rowoff, blkoff, X, ldx, rowprob, kinds, c2s, out,
                                                          parts);
  return hipGetLastError();
}

hipError_t qr_first_conv(hipStream_t s, int nnodes, const int32_t* rowoff, const double* Y, int64_t ldy, int dsk,
                         const int32_t* incprob, const int32_t* ovprob, const int32_t* nodeprob, int32_t* dprob,
                         const double* deltaprob, int32_t* exhausted, int max_m, size_t lds_limit, double* gws,
                         const int64_t* gws_off) {
  if (nnodes <= 0) return hipSuccess;
  if (max_m <= 128 && std::min(max_m, dsk) <= 64) {  // every panel fits the register form
    if (max_m <= 64)
      qr_conv_reg_kernel<16><<<nnodes, 256, 0, s>>>(rowoff, Y, ldy, dsk, incprob, ovprob, nodeprob, dprob, deltaprob,
                                                     exhausted);
    else
      qr_conv_reg_kernel<32><<<nnodes, 256, 0, s>>>(rowoff, Y, ldy, dsk, incprob, ovprob, nodeprob, dprob, deltaprob,
                                                     exhausted);
    return hipGetLastError();
  }
  const int threads = dsk <= 64 ? 64 : (dsk <= 128 ? 128 : 256);
  const size_t bytes = size_t(max_m | 1) * size_t(dsk) * sizeof(double);
  if (bytes <= lds_limit) {
    hipError_t e = allow_lds(qr_first_conv_kernel<true>, bytes);
    if (e != hipSuccess) return e;
    qr_first_conv_kernel<true><<<nnodes, threads, bytes, s>>>(rowoff, Y, ldy, dsk, incprob, ovprob, nodeprob,
                                                              dprob, deltaprob, exhausted, gws, gws_off);
  } else {
    if (!gws || !gws_off) return hipErrorInvalidValue;
    const size_t blocked = size_t(max_m) * (kQrNb + 1) * sizeof(double);
    if (blocked + 4096 <= lds_limit) {  // + the kernel's static LDS
      hipError_t e = allow_lds(qr_first_conv_blocked_kernel, blocked);
      if (e != hipSuccess) return e;
      qr_first_conv_blocked_kernel<<<nnodes, 256, blocked, s>>>(rowoff, Y, ldy, dsk, incprob, ovprob, nodeprob,
                                                                dprob, deltaprob, exhausted, gws, gws_off);
    } else {
      qr_first_conv_kernel<false><<<nnodes, threads, 0, s>>>(rowoff, Y, ldy, dsk, incprob, ovprob, nodeprob,
                                                             dprob, deltaprob, exhausted, gws, gws_off);
    }
  }
  return hipGetLastError();
}

hipError_t scan_i32(hipStream_t s, int n, const int32_t* in, int32_t* out) {
  scan_kernel<<<1, 1024, 0, s>>>(n, in, out);
  return hipGetLastError();
}

hipError_t gather_i32(hipStream_t s, int n, const int32_t* map, const int32_t* src, int32_t* dst) {
  gather_i32_kernel<<<(n + 256) / 256, 256, 0, s>>>(n, map, src, dst);
  return hipGetLastError();
}

hipError_t thresholds(hipStream_t s, int nprob, const void* jobs, const double* Y, int64_t ldy, double* nu,
                      double* delta, int32_t* d) {
  if (nprob <= 0) return hipSuccess;
  threshold_kernel<<<nprob, 256, 0, s>>>(static_cast<const ThresholdJob*>(jobs), Y, ldy, nu, delta, d);
  return hipGetLastError();
}

hipError_t fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return hipSuccess;
  fill_i32_kernel<<<grid_for(n, 256, 1024), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t prepare_kernels(size_t lds_limit) {
  const int b = static_cast<int>(lds_limit);
  auto set = [b](const void* f) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
  };
  const void* ks[] = {
      reinterpret_cast<const void*>(qr_first_conv_kernel<true>),
      reinterpret_cast<const void*>(cpqr_id_kernel<true>),
      reinterpret_cast<const void*>(cpqr_id_kernel<false>),
      reinterpret_cast<const void*>(coupling_update2_kernel),
  };
  for (const void* f : ks) {
    const hipError_t e = set(f);
    if (e != hipSuccess) return e;
  }
  g_lds_prepared = lds_limit;
  return hipSuccess;
}

// ------------------------------------------------ low-rank update launchers

hipError_t lr_leaf_project(hipStream_t s, int nleaves, const int32_t* leafoff, const double* V, int64_t ldv, int r,
                           const double* X, int64_t ldx, int nc, double* W) {
  if (nleaves <= 0 || r <= 0 || nc <= 0) return hipSuccess;
  if (nc > 64) return hipErrorInvalidValue;
  lr_leaf_project_kernel<<<nleaves, 256, 0, s>>>(leafoff, V, ldv, r, X, ldx, nc, W);
  return hipGetLastError();
}

size_t lr_sum_scratch(int nleaves, int len) { return size_t((nleaves + 63) / 64) * size_t(len); }

hipError_t lr_sum(hipStream_t s, int nleaves, int len, const double* W, double* partial, double* out) {
  if (len <= 0) return hipSuccess;
  const int ng = (nleaves + 63) / 64;
  if (ng == 0) return fill_zero(s, out, len);
  const dim3 grid(grid_for(len, 256, 64), ng);
  lr_sum_partial_kernel<<<grid, 256, 0, s>>>(nleaves, len, W, partial);
  lr_sum_final_kernel<<<grid_for(len, 256, 64), 256, 0, s>>>(ng, len, partial, out);
  return hipGetLastError();
}

hipError_t lr_apply(hipStream_t s, int nleaves, const int32_t* ptr, const int32_t* idx, const int32_t* leafoff,
                    int64_t n, const double* U, int64_t ldu, int r, const double* W, int nc, double* Y, int64_t ldy,
                    double alpha) {
  if (r <= 0 || nc <= 0) return hipSuccess;
  const size_t lds = size_t(r) * nc * sizeof(double);
  if (lds > 65536) return hipErrorInvalidValue;
  const unsigned grid = ptr ? static_cast<unsigned>(nleaves) : static_cast<unsigned>((n + 255) / 256);
  if (grid == 0) return hipSuccess;
  lr_apply_kernel<<<grid, 256, lds, s>>>(ptr, idx, leafoff, n, U, ldu, r, W, nc, Y, ldy, alpha);
  return hipGetLastError();
}

hipError_t basis_rows(hipStream_t s, int nnodes, bool leaf, const int32_t* koff, const int32_t* J,
                      const int64_t* joff, const int32_t* kold_off, const int32_t* kold_child_off,
                      const int32_t* leafoff, const double* Uold, const int64_t* uoff_old, const int32_t* koff_child,
                      const double* Rc, int64_t ldrc, double* R, int64_t ldr) {
  if (nnodes <= 0) return hipSuccess;
  basis_rows_kernel<<<nnodes, 256, 0, s>>>(leaf ? 1 : 0, koff, J, joff, kold_off, kold_child_off, leafoff, Uold,
                                           uoff_old, koff_child, Rc, ldrc, R, ldr);
  return hipGetLastError();
}

hipError_t coupling_update(hipStream_t s, int npairs, const int32_t* frow, const int32_t* fidx,
                           const int32_t* koff_r, const int32_t* koff_c, const int32_t* kold_off, int max_kold,
                           const double* Bold, const int64_t* boff_old, const double* Rr, int64_t ldrr,
                           const double* Rc, int64_t ldrc, const double* Ug, int64_t ldug, const double* Vg,
                           int64_t ldvg, int r, double* Bnew, const int64_t* boff_new) {
  if (npairs <= 0) return hipSuccess;
  if (max_kold > kCuMaxK) return hipErrorInvalidValue;
  const size_t lds = size_t(std::max(max_kold, 1)) * kCu2Ld * sizeof(double);
  if (lds <= 65536 || lds <= g_lds_prepared) {
    coupling_update2_kernel<<<npairs, 256, lds, s>>>(frow, fidx, koff_r, koff_c, kold_off, Bold, boff_old, Rr, ldrr,
                                                     Rc, ldrc, Ug, ldug, Vg, ldvg, r, Bnew, boff_new);
  } else {
    coupling_update_kernel<<<npairs, 256, 0, s>>>(frow, fidx, koff_r, koff_c, kold_off, Bold, boff_old, Rr, ldrr, Rc,
                                                  ldrc, Ug, ldug, Vg, ldvg, r, Bnew, boff_new);
  }
  return hipGetLastError();
}

hipError_t dense_lowrank(hipStream_t s, int nleaves, const int32_t* ptr, const int32_t* idx,
                         const int32_t* leafoff, const int64_t* blkoff, const double* Din, const double* U,
                         int64_t ldu, const double* V, int64_t ldv, int r, double* out) {
  if (nleaves <= 0) return hipSuccess;
  dense_lowrank_kernel<<<nleaves, 256, 0, s>>>(ptr, idx, leafoff, blkoff, Din, U, ldu, V, ldv, r, out);
  return hipGetLastError();
}

}  // namespace h2dev
