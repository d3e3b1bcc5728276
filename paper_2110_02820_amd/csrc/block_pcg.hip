// Block Nystrom PCG (Section "Block Nystrom PCG"): O'Leary's preconditioned
// block conjugate gradient recurrences for s right-hand sides that share mu,
// after Feng, Owen and Peric's orthogonalisation of the right-hand sides
// (here a thin QR by CholeskyQR2).  The n x s block work runs in the library's
// operator, preconditioner and GEMM kernels; the s x s Cholesky solves of the
// recurrences run in one workgroup (spd_small).  Float64 throughout.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"

namespace nys {
namespace {

constexpr int SMAX = 64;  // largest block

// One workgroup: M = (G + G^T)/2 = L L^T (lower, in LDS).  If pivot j is not
// positive, info[0] = j + 1 and nothing else is written (info is left as it
// is on success, so a failure stays visible until the host clears it).
// Otherwise, where the pointers are non-null: out = M^{-1} rhs (s x s),
// Lout = L, Linv = L^{-1}.
__global__ __launch_bounds__(256) void spd_small(const double* __restrict__ G, int s,
                                                 const double* __restrict__ rhs, double* __restrict__ out,
                                                 double* __restrict__ Lout, double* __restrict__ Linv,
                                                 int* __restrict__ info) {
  __shared__ double L[SMAX][SMAX + 1];
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int e = t; e < s * s; e += 256) {
    const int i = e / s, j = e % s;
    L[i][j] = 0.5 * (G[i * s + j] + G[j * s + i]);
  }
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (t == 0) {
      const double p = L[j][j];
      if (!(p > 0.0) || !isfinite(p)) bad = j + 1;
      else L[j][j] = sqrt(p);
    }
    __syncthreads();
    if (bad) break;
    const double dj = L[j][j];
    for (int i = j + 1 + t; i < s; i += 256) L[i][j] /= dj;
    __syncthreads();
    // trailing update of the lower triangle: rows i > j, columns j < k <= i
    const int m = s - j - 1;
    for (int e = t; e < m * m; e += 256) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) info[0] = bad;
    return;
  }
  // one thread per column: forward then backward substitution, L^{-1}
  if (t < s) {
    const int c = t;
    if (rhs && out) {
      double y[SMAX];
      for (int i = 0; i < s; ++i) {
        double v = rhs[i * s + c];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
      }
      for (int i = s - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < s; ++k) v -= L[k][i] * y[k];
        y[i] = v / L[i][i];
      }
      for (int i = 0; i < s; ++i) out[i * s + c] = y[i];
    }
    if (Lout)
      for (int i = 0; i < s; ++i) Lout[i * s + c] = i >= c ? L[i][c] : 0.0;
    if (Linv) {
      // column c of L^{-1}: solve L y = e_c
      double y[SMAX];
      for (int i = 0; i < s; ++i) {
        double v = i == c ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = i < c ? 0.0 : v / L[i][i];
      }
      for (int i = 0; i < s; ++i) Linv[i * s + c] = y[i];
    }
  }
}

// norm2[c] = t_c^T S t_c, t_c = column c of T (s x s): the squared column
// norms of R T from S = R^T R
__global__ void col_norms_t(int s, const double* __restrict__ S, const double* __restrict__ T,
                            double* __restrict__ norm2) {
  const int c = threadIdx.x;
  if (c >= s) return;
  double acc = 0.0;
  for (int i = 0; i < s; ++i) {
    double u = 0.0;
    for (int k = 0; k < s; ++k) u += S[i * s + k] * T[k * s + c];
    acc += T[i * s + c] * u;
  }
  norm2[c] = acc;
}

__global__ void diag_of(int s, const double* __restrict__ G, double* __restrict__ d) {
  const int c = threadIdx.x;
  if (c < s) d[c] = G[c * s + c];
}

__global__ void copy_mat(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                         double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e % cols;
  dst[i * ldd + j] = src[i * lds + j];
}

__global__ void zero_mat(int64_t count, double* __restrict__ p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0.0;
}

__global__ void zero_info(int* __restrict__ p) {
  if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

unsigned nb(int64_t count) { return (unsigned)cdiv(count, 256); }

struct BlockWs {
  void* base;
  size_t base_bytes;
  double *Q, *Xt, *R, *Z, *D, *D2, *V;                               // n x s
  double *G, *rho, *rho2, *alpha, *beta, *T0, *L1, *Li, *L2, *S, *T1;  // s x s
  double *norm2, *bn2;                                                // s
  int* info;                                                          // 4
  double* gscr;
  size_t gscr_elems;
};

void carve_block(Arena& a, size_t base_bytes, int64_t n, int64_t s, BlockWs& w) {
  w.base = a.take<char>(base_bytes);
  w.base_bytes = base_bytes;
  double** big[] = {&w.Q, &w.Xt, &w.R, &w.Z, &w.D, &w.D2, &w.V};
  for (double** p : big) *p = a.take<double>((size_t)n * (size_t)s);
  double** small[] = {&w.G, &w.rho, &w.rho2, &w.alpha, &w.beta, &w.T0, &w.L1, &w.Li, &w.L2, &w.S, &w.T1};
  for (double** p : small) *p = a.take<double>((size_t)s * (size_t)s);
  w.norm2 = a.take<double>(s);
  w.bn2 = a.take<double>(s);
  w.info = a.take<int>(4);
  const size_t g1 = gemm_scratch_elems(s, s), g2 = gemm_scratch_elems(n, s);
  w.gscr_elems = g1 > g2 ? g1 : g2;
  w.gscr = a.take<double>(w.gscr_elems);
}

nys_status spd(const double* G, int64_t s, const double* rhs, double* out, double* Lout, double* Linv, int* info,
               hipStream_t st) {
  hipLaunchKernelGGL(spd_small, dim3(1), dim3(256), 0, st, G, (int)s, rhs, out, Lout, Linv, info);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// C = alpha op(A) op(B) + beta C, all float64 row-major
nys_status mm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc, BlockWs& w, hipStream_t s) {
  return gemm<double, double, double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, w.gscr, w.gscr_elems,
                                      s);
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_workspace_size_block(const nys_operator* A, int64_t ell, int64_t s) {
  if (A == nullptr || s < 1 || s > SMAX) return 0;
  const size_t base = nys_workspace_size(A, ell, s, NYS_PREC_FP64);
  if (base == 0) return 0;
  Arena a(nullptr, 0);
  BlockWs w;
  carve_block(a, base, A->n, s, w);
  return a.off + 256;
}

nys_status nys_block_pcg_solve(const nys_operator* A, const nys_precond* P, double mu, const double* B, int64_t s,
                               int64_t ldb, double* X, int64_t ldx, const nys_solve_opts* o, nys_solve_info* info,
                               void* ws, size_t ws_bytes, void* stream) {
  NYS_ARG(A != nullptr && P != nullptr && B != nullptr && X != nullptr && o != nullptr,
          "nys_block_pcg_solve: NULL argument");
  NYS_ARG(o == nullptr || o->device_info == 0, "nys_block_pcg_solve: the device-info form is not available here");
  NYS_ARG(s >= 1 && s <= SMAX && ldb >= s && ldx >= s, "need 1 <= s <= %d and ld >= s", SMAX);
  NYS_ARG(P->n == A->n && P->ell >= 1, "preconditioner does not match the operator");
  NYS_ARG(std::isfinite(mu) && mu >= 0.0, "mu must be finite and >= 0");
  NYS_ARG(o->prec == NYS_PREC_FP64, "the block solver runs in float64 (prec NYS_PREC_FP64)");
  NYS_ARG(o->tol > 0.0, "tol must be > 0");
  const int64_t n = A->n;
  NYS_ARG(s <= n, "more right-hand sides than unknowns");
  const int maxit = o->maxit > 0 ? o->maxit : 500;
  // host checks synchronise the stream: every 8 steps unless asked otherwise
  const int every = o->check_every > 0 ? o->check_every : 8;
  const size_t base = nys_workspace_size(A, P->ell, s, NYS_PREC_FP64);
  NYS_ARG(base > 0, "nys_block_pcg_solve: invalid operator");
  Arena a(ws, ws_bytes);
  BlockWs w;
  carve_block(a, base, n, s, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* sv = stream;
  const int64_t ns = n * s, ss = s * s;
  auto host_info = [&](int* h) -> nys_status {
    NYS_HIP(hipMemcpyAsync(h, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    NYS_HIP(hipStreamSynchronize(st));
    return NYS_OK;
  };
  hipLaunchKernelGGL(zero_info, dim3(1), dim3(64), 0, st, w.info);
  NYS_CHECK_LAUNCH();
  // ---- orthogonalise the right-hand sides: B = Q T0 (CholeskyQR2)
  NYS_TRY(mm(true, false, s, s, n, 1.0, B, ldb, B, ldb, 0.0, w.G, s, w, st));
  hipLaunchKernelGGL(diag_of, dim3(1), dim3(SMAX), 0, st, (int)s, w.G, w.bn2);
  NYS_CHECK_LAUNCH();
  NYS_TRY(spd(w.G, s, nullptr, nullptr, w.L1, w.Li, w.info, st));
  int hi = 0;
  NYS_TRY(host_info(&hi));
  NYS_ARG(hi == 0, "nys_block_pcg_solve: the right-hand sides are linearly dependent (column %d)", hi - 1);
  NYS_TRY(mm(false, true, n, s, s, 1.0, B, ldb, w.Li, s, 0.0, w.R, s, w, st));  // Q1 = B L1^{-T}
  NYS_TRY(mm(true, false, s, s, n, 1.0, w.R, s, w.R, s, 0.0, w.G, s, w, st));
  NYS_TRY(spd(w.G, s, nullptr, nullptr, w.L2, w.Li, w.info, st));
  NYS_TRY(host_info(&hi));
  NYS_ARG(hi == 0, "nys_block_pcg_solve: the right-hand sides are numerically dependent (column %d)", hi - 1);
  NYS_TRY(mm(false, true, n, s, s, 1.0, w.R, s, w.Li, s, 0.0, w.Q, s, w, st));  // Q = Q1 L2^{-T}
  NYS_TRY(mm(true, true, s, s, s, 1.0, w.L2, s, w.L1, s, 0.0, w.T0, s, w, st));  // T0 = L2^T L1^T
  std::vector<double> bn2(s), nr2(s);
  NYS_HIP(hipMemcpyAsync(bn2.data(), w.bn2, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  // ---- initial state: Xt = 0, R = Q, Z = P^{-1} R, D = Z, rho = Z^T R
  hipLaunchKernelGGL(zero_mat, dim3(nb(ns)), dim3(256), 0, st, ns, w.Xt);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(copy_mat, dim3(nb(ns)), dim3(256), 0, st, n, s, w.Q, s, w.R, s);
  NYS_CHECK_LAUNCH();
  NYS_TRY(static_cast<nys_status>(nys_precond_apply(P, mu, w.R, s, s, w.Z, s, w.base, w.base_bytes, sv)));
  hipLaunchKernelGGL(copy_mat, dim3(nb(ns)), dim3(256), 0, st, n, s, w.Z, s, w.D, s);
  NYS_CHECK_LAUNCH();
  NYS_TRY(mm(true, false, s, s, n, 1.0, w.Z, s, w.R, s, 0.0, w.rho, s, w, st));
  int it = 0;
  bool conv = false, brk = false;
  const double tol2 = o->tol * o->tol;
  auto check = [&]() -> nys_status {
    // squared column norms of R T0 (the original residuals) against tol^2 ||b_c||^2
    NYS_TRY(mm(true, false, s, s, n, 1.0, w.R, s, w.R, s, 0.0, w.S, s, w, st));
    hipLaunchKernelGGL(col_norms_t, dim3(1), dim3(SMAX), 0, st, (int)s, w.S, w.T0, w.norm2);
    NYS_CHECK_LAUNCH();
    NYS_HIP(hipMemcpyAsync(nr2.data(), w.norm2, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    NYS_HIP(hipStreamSynchronize(st));
    conv = true;
    for (int64_t c = 0; c < s; ++c) conv = conv && nr2[c] <= tol2 * bn2[c];
    return NYS_OK;
  };
  NYS_TRY(check());
  while (!conv && it < maxit) {
    // V = A_mu D; alpha = (D^T V)^{-1} rho; Xt += D alpha; R -= V alpha
    NYS_TRY(static_cast<nys_status>(nys_op_apply(A, mu, w.D, s, s, w.V, s, NYS_PREC_FP64, w.base, w.base_bytes, sv)));
    NYS_TRY(mm(true, false, s, s, n, 1.0, w.D, s, w.V, s, 0.0, w.G, s, w, st));
    NYS_TRY(spd(w.G, s, w.rho, w.alpha, nullptr, nullptr, w.info, st));
    NYS_TRY(mm(false, false, n, s, s, 1.0, w.D, s, w.alpha, s, 1.0, w.Xt, s, w, st));
    NYS_TRY(mm(false, false, n, s, s, -1.0, w.V, s, w.alpha, s, 1.0, w.R, s, w, st));
    ++it;
    if (it % every == 0 || it == maxit) {
      NYS_TRY(host_info(&hi));
      if (hi != 0) {
        brk = true;
        break;
      }
      NYS_TRY(check());
      if (conv) break;
    }
    // Z = P^{-1} R; rho2 = Z^T R; beta = rho^{-1} rho2; D = Z + D beta
    NYS_TRY(static_cast<nys_status>(nys_precond_apply(P, mu, w.R, s, s, w.Z, s, w.base, w.base_bytes, sv)));
    NYS_TRY(mm(true, false, s, s, n, 1.0, w.Z, s, w.R, s, 0.0, w.rho2, s, w, st));
    NYS_TRY(spd(w.rho, s, w.rho2, w.beta, nullptr, nullptr, w.info + 1, st));
    hipLaunchKernelGGL(copy_mat, dim3(nb(ns)), dim3(256), 0, st, n, s, w.Z, s, w.D2, s);
    NYS_CHECK_LAUNCH();
    NYS_TRY(mm(false, false, n, s, s, 1.0, w.D, s, w.beta, s, 1.0, w.D2, s, w, st));
    std::swap(w.D, w.D2);
    std::swap(w.rho, w.rho2);
    if (it % every == 0) {
      NYS_HIP(hipMemcpyAsync(&hi, w.info + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      NYS_HIP(hipStreamSynchronize(st));
      if (hi != 0) {
        brk = true;
        break;
      }
    }
  }
  if (!conv && !brk) NYS_TRY(check());
  // X = Xt T0
  NYS_TRY(mm(false, false, n, s, s, 1.0, w.Xt, s, w.T0, s, 0.0, X, ldx, w, st));
  NYS_HIP(hipStreamSynchronize(st));
  (void)ss;
  if (std::getenv("NYS_VERBOSE"))
    std::fprintf(stderr, "[nyspcg] block pcg: s=%lld iterations=%d converged=%d breakdown=%d\n", (long long)s, it,
                 (int)conv, (int)brk);
  const nys_status stc = conv ? NYS_OK : brk ? NYS_ERR_BREAKDOWN : NYS_NOT_CONVERGED;
  if (info) {
    for (int64_t c = 0; c < s; ++c) {
      const bool cc = nr2[c] <= tol2 * bn2[c];
      if (info->iters) info->iters[c] = it;
      if (info->relres) info->relres[c] = bn2[c] > 0.0 ? std::sqrt(nr2[c] / bn2[c]) : 0.0;
      if (info->status) info->status[c] = cc ? NYS_OK : stc;
    }
    info->refine_steps = 0;
    info->total_iters = it;
  }
  return stc;
}

}  // extern "C"
