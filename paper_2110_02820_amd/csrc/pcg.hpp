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

// Per-column CG scalars (device arrays of k entries unless noted).
struct CgScalars {
  double* rz;      // [2][k] r^T z, double-buffered by iteration parity
  double* bnorm2;  // ||b||^2
  double* rnorm2;  // recursive ||r||^2 after the last update
  double* alpha;
  double* beta;
  int* done;       // column finished (converged or broken down)
  int* conv;       // stopping test met by the last update
  int* iters;
  int* status;
  int* alldone;    // [1]
  unsigned* ctr;   // [64] arrival counters of the last-workgroup reductions (zeroed once)
};

// Partial-sum buffers of one PCG run.
struct PcgWork {
  double *pb, *prr, *ppv, *prz;  // 512 x k each
  double* apart;                 // precond_part_elems
  size_t apart_elems;
  double *Cs, *Ct;               // l x k each
};

size_t precond_part_elems(int64_t n, int64_t l, int64_t k);

// Z = P^{-1} R (eq. (NysPre)) for k float64 columns, outside the CG loop.
// `ctr` points to 64 zeroed counters.
nys_status precond_apply_standalone(const PrecDesc& P, const double* mu_dev, const double* R, double* Z,
                                    int64_t k, double* part, size_t part_elems, double* Cs, double* Ct,
                                    unsigned* ctr, hipStream_t s);

// R = B - V, Z = P^{-1} R, P = Z, scalars (rz, ||b||, flags).  sc.ctr zeroed.
template <typename T>
nys_status pcg_setup(int64_t n, int64_t k, const PrecDesc& P, const double* mu_dev, int64_t nrhs,
                     const T* B, const T* V, T* R, T* Z, T* Pd, PcgWork& w, const CgScalars& sc, double tol,
                     hipStream_t s);

// One iteration after V = (A + mu I) P: alpha, X/R update, stopping test,
// Z = P^{-1} R, beta, P = Z + beta P.  par = iteration parity.
template <typename T>
nys_status pcg_iteration(int64_t n, int64_t k, const PrecDesc& P, const double* mu_dev, int64_t nrhs,
                         const T* V, T* X, int64_t ldx, T* R, T* Z, T* Pd, PcgWork& w, const CgScalars& sc,
                         int par, double tol, hipStream_t s);

// One iteration for a single column whose product (A p) is given in partial
// form (part: ng x n, A p = scale * sum_g part[g]); fewer launches than
// pcg_iteration (matvec finish, alpha, update and direction are fused).
template <typename T>
nys_status pcg_iteration_fused(int64_t n, const PrecDesc& P, const double* mu_dev, double mu, const T* part,
                               int ng, double scale, T* V, T* X, T* R, T* Z, T* Pd, PcgWork& w,
                               const CgScalars& sc, int par, double tol, hipStream_t s);

// pcg_iteration_fused for a product that also gave pvq (op_matvec_partials:
// npvq parts of p^T A p / scale, then npp parts of ||p||^2): alpha is known before the
// partials are summed, so one launch sums them, updates x and r and forms
// this launch's parts of U^T r; then the scaling of U^T r (with the stopping
// test and the parts of r^T z = ||r||^2 + w^T D w) and the apply with the
// direction update.  Requires pcg_pvq_ok; returns NYS_ERR_ARG otherwise.
template <typename T>
nys_status pcg_iteration_pvq(int64_t n, const PrecDesc& P, const double* mu_dev, double mu, const T* part, int ng,
                             const double* pvq, int npvq, int npp, double scale, T* V, T* X, T* R, T* Z, T* Pd,
                             PcgWork& w, const CgScalars& sc, int par, double tol, hipStream_t s);
// whether pcg_iteration_pvq supports this size and U layout (n <= 16384,
// 16-byte U rows)
bool pcg_pvq_ok(const PrecDesc& P, int64_t n);

// State of column 0 after a batch of iterations, written by the device into
// host memory (pcg_snapshot) for host loops that poll without synchronising.
struct PcgSnap {
  int seq;  // written last: the tag the host waits for
  int alldone;
  int iters;
  int status;
  double rnorm2, bnorm2;
};
nys_status pcg_snapshot(const CgScalars& sc, PcgSnap* out, int seq, hipStream_t s);

// Pieces of one block iteration for callers that supply their own operator
// product and preconditioner apply (n x k blocks, ld = k, per-column scalars):
//   cg_block_init:      R = B - V, ||B||^2, stopping flags (sc.ctr zeroed)
//   cg_block_update:    alpha = r^T z / p^T v, X += alpha P, R -= alpha V, stopping test
//   cg_block_direction: r^T z, beta, P = Z + beta P (init: rz and P = Z)
template <typename T>
nys_status cg_block_init(int64_t n, int64_t k, const T* B, const T* V, T* R, PcgWork& w, const CgScalars& sc,
                         double tol, hipStream_t s);
template <typename T>
nys_status cg_block_update(int64_t n, int64_t k, const T* V, T* X, T* R, const T* Pd, PcgWork& w,
                           const CgScalars& sc, int par, double tol, hipStream_t s);
template <typename T>
nys_status cg_block_direction(int64_t n, int64_t k, const T* R, const T* Z, T* Pd, PcgWork& w,
                              const CgScalars& sc, int par, bool init, hipStream_t s);

}  // namespace nys
