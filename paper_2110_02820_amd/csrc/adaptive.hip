// Adaptive rank selection for the Nystrom preconditioner: the randomized
// power estimate of ||E|| = ||A - U diag(lam) U^T|| (Appendix, algorithm
// "Randomized Power method for estimating ||E||") and the sketch-doubling
// driver (Section "Adaptive rank selection", Strategies 1 and 2; Appendix,
// algorithm "Adaptive Randomized Nystrom Approximation").  The doubling loop
// is host control over the library's own entry points (sketch, factor, operator
// product); the estimate's vector work runs in the kernels below and the
// library GEMM.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

#include "common.hpp"
#include "gemm.hpp"

namespace nys {
namespace {

constexpr int NT = 256;
constexpr int NB = 256;  // partial sums per reduction (one per workgroup)

// part[b] = sum over the rows of workgroup b of x_i^2 (fixed order)
__global__ __launch_bounds__(NT) void pw_sumsq_part(int64_t n, const double* __restrict__ x,
                                                    double* __restrict__ part) {
  __shared__ double sh[NT / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) acc += x[i] * x[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// v = Av - w (in place in av); part[b] = sum v0_i v_i, part[NB + b] = sum v_i^2
__global__ __launch_bounds__(NT) void pw_residual_part(int64_t n, const double* __restrict__ v0,
                                                       double* __restrict__ av, const double* __restrict__ w,
                                                       double* __restrict__ part) {
  __shared__ double sh[NT / 64];
  double d = 0.0, s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double v = av[i] - w[i];
    av[i] = v;
    d += v0[i] * v;
    s += v * v;
  }
  d = block_sum(d, sh);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = d;
    part[NB + blockIdx.x] = s;
  }
}

// out[r] = sum_b part[r * NB + b] for r < nr (one workgroup, fixed order)
__global__ __launch_bounds__(NT) void pw_final(const double* __restrict__ part, int nr, double* __restrict__ out) {
  __shared__ double sh[NT / 64];
  for (int r = 0; r < nr; ++r) {
    const double v = block_sum(threadIdx.x < NB ? part[r * NB + threadIdx.x] : 0.0, sh);
    if (threadIdx.x == 0) out[r] = v;
  }
}

// dst = src / sqrt(*sq); a zero vector is left as it is (dst = src)
__global__ void pw_normalize(int64_t n, const double* __restrict__ src, const double* __restrict__ sq,
                             double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = *sq;
  dst[i] = q > 0.0 ? src[i] / sqrt(q) : src[i];
}

// c_j *= lam_j
__global__ void pw_scale_lam(int64_t l, const double* __restrict__ lam, double* __restrict__ c) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < l) c[j] *= lam[j];
}

template <typename S, typename D>
__global__ void pw_convert(int64_t n, const S* __restrict__ src, D* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = D(src[i]);
}

// dst[i][j] = src[i][j] for i < n, j < m (row-major, leading dims lds, ldd)
__global__ void copy_block(int64_t n, int64_t m, const double* __restrict__ src, int64_t lds,
                           double* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t i = idx / m, j = idx % m;
  dst[i * ldd + j] = src[i * lds + j];
}

unsigned nblk(int64_t count) { return (unsigned)cdiv(count, 256); }

nys_status copy_cols(int64_t n, int64_t m, const double* src, int64_t lds, double* dst, int64_t ldd,
                     hipStream_t s) {
  hipLaunchKernelGGL(copy_block, dim3(nblk(n * m)), dim3(256), 0, s, n, m, src, lds, dst, ldd);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Buffers of the power estimate beyond the operator product's workspace.
struct PowerWs {
  double *v0, *av, *w, *c, *part, *scal;
  float *vf, *avf;
  double* gscr;
  size_t gscr_elems;
};

void carve_power(Arena& a, int64_t n, int64_t l, PowerWs& p) {
  p.v0 = a.take<double>(n);
  p.av = a.take<double>(n);
  p.w = a.take<double>(n);
  p.c = a.take<double>(l);
  p.part = a.take<double>(2 * NB);
  p.scal = a.take<double>(4);
  p.vf = a.take<float>(n);
  p.avf = a.take<float>(n);
  p.gscr_elems = 16 * (size_t)(n > l ? n : l);
  p.gscr = a.take<double>(p.gscr_elems);
}

template <typename TU>
nys_status lowrank_apply(int64_t n, int64_t l, const TU* U, int64_t ldu, const double* lam, const double* v,
                         PowerWs& p, hipStream_t s) {
  // w = U (lam .* (U^T v))
  NYS_TRY((gemm<double, TU, double>(true, false, l, 1, n, 1.0, U, ldu, v, 1, 0.0, p.c, 1, p.gscr, p.gscr_elems,
                                    s)));
  hipLaunchKernelGGL(pw_scale_lam, dim3(nblk(l)), dim3(256), 0, s, l, lam, p.c);
  NYS_CHECK_LAUNCH();
  NYS_TRY((gemm<double, TU, double>(false, false, n, 1, l, 1.0, U, ldu, p.c, 1, 0.0, p.w, 1, p.gscr,
                                    p.gscr_elems, s)));
  return NYS_OK;
}

// The estimate itself; the operator product uses ws_op (at least
// nys_workspace_size(A, 1, 1, prec) bytes), the vectors p.
nys_status power_est(const nys_operator* A, const nys_precond* P, int32_t q, const double* g, double* est,
                     int32_t prec, void* ws_op, size_t ws_op_bytes, PowerWs& p, hipStream_t s) {
  const int64_t n = P->n, l = P->ell;
  void* st = static_cast<void*>(s);
  // v0 = g / ||g||
  hipLaunchKernelGGL(pw_sumsq_part, dim3(NB), dim3(NT), 0, s, n, g, p.part);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(pw_final, dim3(1), dim3(NT), 0, s, p.part, 1, p.scal + 1);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(pw_normalize, dim3(nblk(n)), dim3(256), 0, s, n, g, p.scal + 1, p.v0);
  NYS_CHECK_LAUNCH();
  for (int it = 0; it < q; ++it) {
    // v = A v0 - U (lam .* (U^T v0))
    if (prec == NYS_PREC_FP64) {
      NYS_TRY(static_cast<nys_status>(nys_op_apply(A, 0.0, p.v0, 1, 1, p.av, 1, prec, ws_op, ws_op_bytes, st)));
    } else {
      hipLaunchKernelGGL((pw_convert<double, float>), dim3(nblk(n)), dim3(256), 0, s, n, p.v0, p.vf);
      NYS_CHECK_LAUNCH();
      NYS_TRY(static_cast<nys_status>(nys_op_apply(A, 0.0, p.vf, 1, 1, p.avf, 1, prec, ws_op, ws_op_bytes, st)));
      hipLaunchKernelGGL((pw_convert<float, double>), dim3(nblk(n)), dim3(256), 0, s, n, p.avf, p.av);
      NYS_CHECK_LAUNCH();
    }
    if (P->dtype == NYS_F64)
      NYS_TRY(lowrank_apply(n, l, static_cast<const double*>(P->U), P->ldu, P->lam, p.v0, p, s));
    else
      NYS_TRY(lowrank_apply(n, l, static_cast<const float*>(P->U), P->ldu, P->lam, p.v0, p, s));
    // E = v0^T v; v0 = v / ||v||
    hipLaunchKernelGGL(pw_residual_part, dim3(NB), dim3(NT), 0, s, n, p.v0, p.av, p.w, p.part);
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(pw_final, dim3(1), dim3(NT), 0, s, p.part, 2, p.scal);
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(pw_normalize, dim3(nblk(n)), dim3(256), 0, s, n, p.av, p.scal + 1, p.v0);
    NYS_CHECK_LAUNCH();
  }
  double e = 0.0;
  NYS_HIP(hipMemcpyAsync(&e, p.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  *est = e;
  return NYS_OK;
}

nys_status check_adaptive_prec(const nys_precond* P, int64_t n, int64_t lcap) {
  NYS_ARG(P != nullptr && P->U != nullptr && P->lam != nullptr, "NULL preconditioner buffers");
  NYS_ARG(P->n == n, "preconditioner n = %lld differs from the operator's n = %lld", (long long)P->n,
          (long long)n);
  NYS_ARG(P->dtype == NYS_F64 || P->dtype == NYS_F32, "U must be float64 or float32");
  NYS_ARG(P->ldu >= lcap, "ldu = %lld < %lld", (long long)P->ldu, (long long)lcap);
  return NYS_OK;
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_workspace_size_adaptive(const nys_operator* A, int64_t ell_max, int32_t prec) {
  if (A == nullptr || ell_max < 1) return 0;
  const size_t base = nys_workspace_size(A, ell_max, 1, prec);
  if (base == 0) return 0;
  const int64_t n = A->n;
  Arena a(nullptr, 0);
  a.take<char>(base);
  a.take<double>((size_t)n * (size_t)ell_max);  // packed Omega
  a.take<double>((size_t)n * (size_t)ell_max);  // packed Y
  a.take<double>(n);                            // start vector
  PowerWs p;
  carve_power(a, n, ell_max, p);
  return a.off + 256;
}

nys_status nys_power_err_est(const nys_operator* A, const nys_precond* P, int32_t q, const double* g,
                             double* est, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  NYS_ARG(A != nullptr && g != nullptr && est != nullptr, "nys_power_err_est: NULL argument");
  NYS_ARG(q >= 1, "nys_power_err_est: q = %d < 1", (int)q);
  NYS_ARG(prec >= NYS_PREC_FP64 && prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  NYS_TRY(check_adaptive_prec(P, A->n, P ? P->ell : 0));
  NYS_ARG(P->ell >= 1 && P->ell <= P->n, "preconditioner rank %lld outside [1, n]", (long long)P->ell);
  const size_t base = nys_workspace_size(A, 1, 1, prec);
  NYS_ARG(base > 0, "nys_power_err_est: invalid operator");
  Arena a(ws, ws_bytes);
  void* ws_op = a.take<char>(base);
  PowerWs p;
  carve_power(a, P->n, P->ell, p);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  return power_est(A, P, q, g, est, prec, ws_op, base, p, static_cast<hipStream_t>(stream));
}

nys_status nys_nystrom_adaptive(const nys_operator* A, int64_t ell0, int64_t ell_max, int32_t q, double tau,
                                double mu, int32_t criterion, uint64_t seed, double* Omega, double* Y, int64_t ld,
                                nys_precond* P, double* err_out, int32_t prec, void* ws, size_t ws_bytes,
                                void* stream) {
  NYS_ARG(A != nullptr && Omega != nullptr && Y != nullptr && err_out != nullptr, "nys_nystrom_adaptive: NULL argument");
  const int64_t n = A->n;
  NYS_ARG(ell0 >= 1 && ell0 <= ell_max && ell_max <= n, "need 1 <= ell0 <= ell_max <= n");
  NYS_ARG(ld >= ell_max, "ld = %lld < ell_max = %lld", (long long)ld, (long long)ell_max);
  NYS_ARG(criterion >= NYS_ADA_ERR && criterion <= NYS_ADA_RATIO, "unknown stopping criterion %d", (int)criterion);
  NYS_ARG(criterion == NYS_ADA_RATIO || q >= 1, "the error criteria need q >= 1 power steps");
  NYS_ARG(std::isfinite(tau) && tau > 0.0 && std::isfinite(mu) && mu >= 0.0, "need tau > 0 and mu >= 0");
  NYS_ARG(prec >= NYS_PREC_FP64 && prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  NYS_TRY(check_adaptive_prec(P, n, ell_max));
  const size_t base = nys_workspace_size(A, ell_max, 1, prec);
  NYS_ARG(base > 0, "nys_nystrom_adaptive: invalid operator");
  Arena a(ws, ws_bytes);
  void* ws_base = a.take<char>(base);
  double* Op = a.take<double>((size_t)n * (size_t)ell_max);
  double* Yp = a.take<double>((size_t)n * (size_t)ell_max);
  double* g = a.take<double>(n);
  PowerWs p;
  carve_power(a, n, ell_max, p);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double tol = tau * mu;
  int64_t l = 0, m = ell0;
  uint64_t j = 0;
  // one more block of m columns: sketch it (packed), append it to Omega and Y
  // (leading dimension ld) and factor the first l + m columns
  auto extend = [&](int64_t mm) -> nys_status {
    NYS_TRY(static_cast<nys_status>(nys_sketch(A, mm, seed + 2 * j, nullptr, Op, Yp, prec, ws_base, base, stream)));
    NYS_TRY(copy_cols(n, mm, Op, mm, Omega + l, ld, s));
    NYS_TRY(copy_cols(n, mm, Yp, mm, Y + l, ld, s));
    l += mm;
    NYS_TRY(copy_cols(n, l, Omega, ld, Op, l, s));
    NYS_TRY(copy_cols(n, l, Y, ld, Yp, l, s));
    P->ell = l;
    return static_cast<nys_status>(nys_factor(Op, Yp, P, prec, ws_base, base, stream));
  };
  while (true) {
    NYS_TRY(extend(m));
    double lam_l = 0.0;
    NYS_HIP(hipMemcpyAsync(&lam_l, P->lam + (l - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
    double E = std::numeric_limits<double>::quiet_NaN();
    bool ok;
    if (criterion == NYS_ADA_RATIO) {
      ok = lam_l <= tol;
    } else {
      NYS_TRY(static_cast<nys_status>(nys_gaussian(seed + 2 * j + 1, n, 1, g, 1, stream)));
      NYS_TRY(power_est(A, P, q, g, &E, prec, ws_base, base, p, s));
      ok = E <= tol && (criterion == NYS_ADA_ERR || lam_l <= tol / 11.0);
    }
    if (std::getenv("NYS_VERBOSE"))
      std::fprintf(stderr, "[nyspcg] adaptive: l=%lld lam_l=%.3e E=%.3e tol=%.3e\n", (long long)l, lam_l, E, tol);
    ++j;
    if (ok) {
      *err_out = E;
      return NYS_OK;
    }
    // the sketch size doubles; past ell_max the last block fills up to ell_max
    if (2 * l > ell_max) {
      if (ell_max > l) NYS_TRY(extend(ell_max - l));
      *err_out = std::numeric_limits<double>::quiet_NaN();
      return NYS_NOT_CONVERGED;
    }
    m = l;
  }
}

}  // extern "C"
