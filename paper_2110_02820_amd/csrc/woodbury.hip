// Nystrom sketch-and-solve (Section "Nystrom sketch-and-solve"): the proxy
// system (A_hat + mu I) x = b with A_hat = U diag(lam) U^T, solved by the
// Woodbury form of the lemma on approximate regularized inversion:
//   x = (1/mu) b + U (g .* (U^T b)),  g_j = 1/(lam_j + mu) - 1/mu
//                                         = -lam_j / (mu (lam_j + mu))
// (the second form has no cancellation).  Two GEMMs through U and two small
// element-wise kernels, all float64 (a float32 U is promoted).
#include <cmath>

#include "common.hpp"
#include "gemm.hpp"

namespace nys {
namespace {

// C[j][c] *= -lam_j / (mu (lam_j + mu))
__global__ void woodbury_scale(int64_t l, int64_t k, const double* __restrict__ lam, double mu,
                               double* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * k) return;
  const double lj = lam[e / k];
  C[e] *= -lj / (mu * (lj + mu));
}

// X[i][c] = B[i][c] / mu
__global__ void scaled_copy(int64_t n, int64_t k, const double* __restrict__ B, int64_t ldb, double inv_mu,
                            double* __restrict__ X, int64_t ldx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t i = e / k, c = e % k;
  X[i * ldx + c] = B[i * ldb + c] * inv_mu;
}

struct WoodWs {
  double* C;
  double* gscr;
  size_t gscr_elems;
};

void carve_wood(Arena& a, int64_t n, int64_t l, int64_t k, WoodWs& w) {
  w.C = a.take<double>((size_t)l * (size_t)k);
  const size_t g1 = gemm_scratch_elems(l, k), g2 = gemm_scratch_elems(n, k);
  w.gscr_elems = g1 > g2 ? g1 : g2;
  w.gscr = a.take<double>(w.gscr_elems);
}

template <typename TU>
nys_status sketch_solve_impl(const nys_precond* P, double mu, const double* B, int64_t k, int64_t ldb, double* X,
                             int64_t ldx, WoodWs& w, hipStream_t s) {
  const int64_t n = P->n, l = P->ell;
  const TU* U = static_cast<const TU*>(P->U);
  NYS_TRY((gemm<double, TU, double>(true, false, l, k, n, 1.0, U, P->ldu, B, ldb, 0.0, w.C, k, w.gscr,
                                    w.gscr_elems, s)));
  hipLaunchKernelGGL(woodbury_scale, dim3((unsigned)cdiv(l * k, 256)), dim3(256), 0, s, l, k, P->lam, mu, w.C);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(scaled_copy, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, B, ldb, 1.0 / mu, X,
                     ldx);
  NYS_CHECK_LAUNCH();
  NYS_TRY((gemm<double, TU, double>(false, false, n, k, l, 1.0, U, P->ldu, w.C, k, 1.0, X, ldx, w.gscr,
                                    w.gscr_elems, s)));
  return NYS_OK;
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_workspace_size_sketch_solve(int64_t n, int64_t ell, int64_t k) {
  if (n < 1 || ell < 1 || k < 1) return 0;
  Arena a(nullptr, 0);
  WoodWs w;
  carve_wood(a, n, ell, k, w);
  return a.off + 256;
}

nys_status nys_sketch_solve(const nys_precond* P, double mu, const double* B, int64_t k, int64_t ldb, double* X,
                            int64_t ldx, void* ws, size_t ws_bytes, void* stream) {
  NYS_ARG(P != nullptr && P->U != nullptr && P->lam != nullptr && B != nullptr && X != nullptr,
          "nys_sketch_solve: NULL argument");
  NYS_ARG(P->n >= 1 && P->ell >= 1 && P->ell <= P->n && P->ldu >= P->ell, "invalid preconditioner shape");
  NYS_ARG(P->dtype == NYS_F64 || P->dtype == NYS_F32, "U must be float64 or float32");
  NYS_ARG(k >= 1 && ldb >= k && ldx >= k, "nys_sketch_solve: invalid block shape");
  NYS_ARG(std::isfinite(mu) && mu > 0.0, "sketch-and-solve needs mu > 0");
  NYS_ARG(B != X, "nys_sketch_solve: B and X must not alias");
  Arena a(ws, ws_bytes);
  WoodWs w;
  carve_wood(a, P->n, P->ell, k, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (P->dtype == NYS_F64) return sketch_solve_impl<double>(P, mu, B, k, ldb, X, ldx, w, s);
  return sketch_solve_impl<float>(P, mu, B, k, ldb, X, ldx, w, s);
}

}  // extern "C"
