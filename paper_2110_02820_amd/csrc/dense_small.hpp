#pragma once
#include "common.hpp"

namespace nys {

// nu <- max(eps(||Y||_F), u_rel ||Y||_F) for `count` contiguous entries;
// `part` holds frob_partials() doubles.
nys_status frob_shift(const double* Y, int64_t count, double* part, double* nu, double u_rel, hipStream_t s);
size_t frob_partials();
// Y += factor * nu * Omega  (nu read on the device)
nys_status add_shift(double* Y, const double* Om, int64_t count, const double* nu, double factor,
                     hipStream_t s);
nys_status scale_device_scalar(double* x, double factor, hipStream_t s);

// L L^T = (M + M^T)/2 (lower L, upper part zeroed); Dinv receives the inverses
// of the diagonal blocks (chol_ws_doubles(n) doubles); *info = 0 or k+1 for a
// non-positive pivot at column k.
size_t chol_ws_doubles(int64_t n);
nys_status cholesky(const double* M, int64_t n, double* L, double* Dinv, int* info, hipStream_t s);
// X = L^{-1} (lower, full n x n written) using the diagonal-block inverses.
nys_status tri_inverse(const double* L, int64_t n, const double* Dinv, double* X, hipStream_t s);

// Eigen-decomposition of the symmetric l x l matrix G = W diag(s) W^T
// (block Jacobi).  Writes T = W[:, perm] diag(1/sqrt(s)) (l x l) with perm sorting s
// descending, lam = max(0, s - nu) (descending), sig2 = s (descending, nullable).
size_t eig_ws_doubles(int64_t l);
// flags: max_sweeps ints; sweeps_out, conv: device ints.  conv_ratio: the
// sweep in which no rotated pair had |a_pq| / sqrt(|a_pp a_qq|) above it is
// the last (1e-9 leaves off-diagonal ratios ~1e-16; 1e-4 leaves ~1e-8, enough
// for eigenvectors that are stored in float32).
nys_status sym_eig(const double* G, int64_t l, double* work, int* flags, int max_sweeps,
                   int* sweeps_out, int* conv, double* T, double* lam, double* sig2, const double* nu,
                   hipStream_t s, double conv_ratio = 1e-9);

}  // namespace nys
