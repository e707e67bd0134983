"""FP64 CPU oracle of the adaptive-sketching H^2 construction (arXiv 2506.16759).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C ABI or the Python binding) may import, call or execute this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code, header, table or constant generator with the HIP path.

Plain, slow and meant to be checked by eye against the paper:
  philox   -- counter-based Gaussian test matrix Omega (Philox4x64-10 + Box-Muller)
  tree     -- KD-tree cluster tree, general admissibility, dual-tree traversal,
              near (N_tau) and far (F_tau) interaction lists   [Sec. II-A]
  linalg   -- Householder QR, column-pivoted QR, interpolative decomposition
                                                             [Sec. II-B, Sec. III-B]
  kernels  -- covariance kernels and dense products          [Sec. V-A]
  build    -- Algorithm 1 with the adaptive sampling loop    [Alg. 1, Sec. III]
  h2       -- the H^2 container, matvec (and transposed), dense reconstruction,
              entries from the format's definition, error measures
  update   -- two-sided construction of non-symmetric matrices and the H^2
              low-rank update A = K_H + U V^T          [Sec. II-A, Sec. III, Sec. V]

Every function cites the passage it follows.  Readings of points the paper
leaves open are the ones listed in the design notes; each is restated where it
is used.
"""
