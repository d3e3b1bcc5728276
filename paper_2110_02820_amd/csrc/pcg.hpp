#pragma once
#include "common.hpp"

namespace nys {

// Validated copy of a nys_precond.
struct PrecDesc {
  int64_t n, ell;
  const void* U;
  int64_t ldu;
  int dtype;
  const double* lam;
};

// Per-column CG scalars (device arrays, k entries each; rz has 2k).
struct CgScalars {
  double* rz;      // [2][k] r^T z, double-buffered by iteration parity
  double* bnorm2;  // [k]
  double* rnorm2;  // [k] recursive ||r||^2 after the last update
  int* done;       // [k]
  int* iters;      // [k]
  int* status;     // [k]
  int* alldone;    // [1]
};

// Z = P^{-1} R (eq. (NysPre)) for k columns (n x k row-major, ld = k).
// f32 selects float vectors (R, Z); U may be float or double.  mu_dev: device
// array indexed by column / nrhs.  done (nullable): columns to leave at Z = R.
// part: partial sums (precond_part_elems doubles); Cs: l x k doubles;
// Ctmp: l x k doubles.
nys_status precond_apply_dev(const PrecDesc& P, const double* mu_dev, int64_t nrhs, const void* R,
                             void* Z, int64_t k, bool f32, const int* done, const int* alldone,
                             double* part, size_t part_elems, double* Cs, void* Ctmp,
                             hipStream_t s);
size_t precond_part_elems(int64_t n, int64_t l, int64_t k);

// R = B - V, partial ||B||^2 (pb) and ||R||^2 (prr); ng groups.
template <typename T>
nys_status cg_kernels_init(int64_t n, int64_t k, const T* B, int64_t ldb, const T* V, T* R,
                           double* pb, double* prr, int ng, hipStream_t s);
// rz from R, Z; scalars; P = Z; stopping flags.
template <typename T>
nys_status cg_kernels_init2(int64_t n, int64_t k, const T* R, const T* Z, T* P, double* pb,
                            double* prr, double* prz, double tol, const CgScalars& sc, int ng,
                            hipStream_t s);
// p^T v partials, alpha, X += alpha P, R -= alpha V, ||R||^2 partials.
template <typename T>
nys_status cg_kernels_step_a(int64_t n, int64_t k, const T* P, const T* V, T* X, int64_t ldx, T* R,
                             double* ppv, double* prr, const CgScalars& sc, int par, int ng,
                             hipStream_t s);
// r^T z partials, beta, P = Z + beta P, stopping test, all-done flag.
template <typename T>
nys_status cg_kernels_step_b(int64_t n, int64_t k, const T* R, const T* Z, T* P, double* prz,
                             const double* prr, const CgScalars& sc, int par, double tol, int ng,
                             hipStream_t s);

}  // namespace nys
