// Nystrom preconditioner apply (Section 5.1.2, eq. (NysPre)) and the PCG
// iteration (Section 5.2, algorithm "Nystrom PCG") on the device.
//
// Vectors are n x k row-major blocks (k independent columns, k <= 256); a
// single right-hand side is k = 1.  Every reduction is two-stage with a fixed
// order (per-workgroup partials, then a fixed-order sum), so results are
// bitwise reproducible run to run.  CG scalars live on the device: the host
// enqueues iterations without reading them and polls the convergence flags
// only every few iterations.  rz (= r^T z) is double-buffered by iteration
// parity so a kernel can read the old value while one workgroup writes the new.
#include "pcg.hpp"
#include "gemm.hpp"

namespace nys {

namespace {

constexpr int NT = 256;

// Thread -> (column, row offset) map for n x k blocks: kp = smallest power of
// two >= k; thread t serves column t % kp and rows t / kp + j * (256 / kp).
struct ColMap {
  int kp, rstep, c, roff;
  __device__ ColMap(int64_t k) {
    kp = 1;
    while (kp < k) kp <<= 1;
    rstep = NT / kp;
    c = threadIdx.x % kp;
    roff = threadIdx.x / kp;
  }
};

// Sum per column over the threads of a block that share a column; result in
// sh[c] (size kp).  `sh` has NT doubles.
__device__ __forceinline__ void colmap_reduce(double v, const ColMap& cm, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s >= cm.kp; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
}

__device__ __forceinline__ double sum_partials(const double* part, int ng, int64_t k, int64_t c) {
  double s = 0.0;
  for (int g = 0; g < ng; ++g) s += part[(int64_t)g * k + c];
  return s;
}

// ---------------------------------------------------------------- set-up

// R = B - V (V = A_mu X); partial ||B||^2 and ||R||^2 per column.
template <typename T>
__global__ __launch_bounds__(NT) void cg_init_residual(int64_t n, int64_t k, const T* __restrict__ B,
                                                       int64_t ldb, const T* __restrict__ V,
                                                       T* __restrict__ R, double* __restrict__ pb,
                                                       double* __restrict__ prr, int64_t rpw) {
  __shared__ double sh[NT];
  ColMap cm(k);
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double sb = 0.0, sr = 0.0;
  if (cm.c < k)
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep) {
      const T b = B[i * ldb + cm.c];
      const T r = b - V[i * k + cm.c];
      R[i * k + cm.c] = r;
      sb += double(b) * double(b);
      sr += double(r) * double(r);
    }
  colmap_reduce(sb, cm, sh);
  if (threadIdx.x < k) pb[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
  colmap_reduce(sr, cm, sh);
  if (threadIdx.x < k) prr[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
}

// P = Z; rz[0][c] = sum partials; bnorm2; done flags for columns already converged.
__global__ void cg_init_scalars(int64_t k, int ng, const double* __restrict__ pb,
                                const double* __restrict__ prr, const double* __restrict__ prz,
                                double tol, CgScalars sc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const double b2 = sum_partials(pb, ng, k, c);
  const double r2 = sum_partials(prr, ng, k, c);
  sc.bnorm2[c] = b2;
  sc.rnorm2[c] = r2;
  sc.rz[c] = sum_partials(prz, ng, k, c);
  sc.iters[c] = 0;
  const bool conv = r2 <= tol * tol * b2;
  sc.done[c] = conv ? 1 : 0;
  sc.status[c] = conv ? NYS_OK : NYS_NOT_CONVERGED;
}

template <typename T>
__global__ void copy_cols(int64_t n, int64_t k, const T* __restrict__ Z, T* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n * k) P[idx] = Z[idx];
}

// ---------------------------------------------------------------- iteration

// partial p^T v per column
template <typename T>
__global__ __launch_bounds__(NT) void cg_pv_partial(int64_t n, int64_t k, const T* __restrict__ P,
                                                    const T* __restrict__ V, double* __restrict__ ppv,
                                                    int64_t rpw, const int* __restrict__ alldone) {
  if (*alldone) return;
  __shared__ double sh[NT];
  ColMap cm(k);
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double s = 0.0;
  if (cm.c < k)
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep)
      s += double(P[i * k + cm.c]) * double(V[i * k + cm.c]);
  colmap_reduce(s, cm, sh);
  if (threadIdx.x < k) ppv[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
}

// alpha = rz / p^T v; X += alpha P; R -= alpha V; partial ||R||^2.
template <typename T>
__global__ __launch_bounds__(NT) void cg_update(int64_t n, int64_t k, int ng_pv,
                                                const double* __restrict__ ppv, CgScalars sc, int par,
                                                const T* __restrict__ P, const T* __restrict__ V,
                                                T* __restrict__ X, int64_t ldx, T* __restrict__ R,
                                                double* __restrict__ prr, int64_t rpw) {
  if (*sc.alldone) return;
  __shared__ double sh[NT];
  __shared__ double alpha_s[NT];
  ColMap cm(k);
  for (int64_t c = threadIdx.x; c < k; c += NT) {
    double a = 0.0;
    if (!sc.done[c]) {
      const double pv = sum_partials(ppv, ng_pv, k, c);
      if (pv > 0.0) {
        a = sc.rz[par * k + c] / pv;
      } else if (blockIdx.x == 0) {
        sc.status[c] = NYS_ERR_BREAKDOWN;
      }
    }
    alpha_s[c] = a;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double s = 0.0;
  if (cm.c < k) {
    const T a = T(alpha_s[cm.c]);
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep) {
      const int64_t e = i * k + cm.c;
      X[i * ldx + cm.c] += a * P[e];
      const T r = R[e] - a * V[e];
      R[e] = r;
      s += double(r) * double(r);
    }
  }
  colmap_reduce(s, cm, sh);
  if (threadIdx.x < k) prr[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
}

// partial rz and the direction update are split: cg_rz_partial computes
// r^T z per column; cg_direction applies beta and the stopping test.
template <typename T>
__global__ __launch_bounds__(NT) void cg_rz_partial(int64_t n, int64_t k, const T* __restrict__ R,
                                                    const T* __restrict__ Z, double* __restrict__ prz,
                                                    int64_t rpw, const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  __shared__ double sh[NT];
  ColMap cm(k);
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double s = 0.0;
  if (cm.c < k)
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep)
      s += double(R[i * k + cm.c]) * double(Z[i * k + cm.c]);
  colmap_reduce(s, cm, sh);
  if (threadIdx.x < k) prz[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
}

// beta = rz_new / rz_old; P = Z + beta P for unfinished columns; stopping test
// ||r||^2 <= tol^2 ||b||^2 on the recursive residual; iteration counters.
template <typename T>
__global__ __launch_bounds__(NT) void cg_direction(int64_t n, int64_t k, int ng, const double* __restrict__ prz,
                                                   const double* __restrict__ prr, CgScalars sc, int par,
                                                   double tol, const T* __restrict__ Z,
                                                   T* __restrict__ P, int64_t rpw) {
  if (*sc.alldone) return;
  __shared__ double beta_s[NT];
  __shared__ int upd_s[NT];
  ColMap cm(k);
  for (int64_t c = threadIdx.x; c < k; c += NT) {
    int upd = 0;
    double beta = 0.0;
    if (!sc.done[c]) {
      const double rzn = sum_partials(prz, ng, k, c);
      const double rr = sum_partials(prr, ng, k, c);
      beta = rzn / sc.rz[par * k + c];
      const bool brk = sc.status[c] == NYS_ERR_BREAKDOWN;
      const bool conv = rr <= tol * tol * sc.bnorm2[c];
      upd = (brk || conv) ? 0 : 1;
      if (blockIdx.x == 0) {
        sc.rz[(1 - par) * k + c] = rzn;
        sc.rnorm2[c] = rr;
        if (!brk) sc.iters[c] += 1;
        if (conv && !brk) sc.status[c] = NYS_OK;
        if (conv || brk) sc.done[c] = 1;
      }
    }
    beta_s[c] = beta;
    upd_s[c] = upd;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  if (cm.c < k && upd_s[cm.c]) {
    const T b = T(beta_s[cm.c]);
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep) {
      const int64_t e = i * k + cm.c;
      P[e] = Z[e] + b * P[e];
    }
  }
}

// all-done flag: 1 when every column is done
__global__ void cg_alldone(int64_t k, CgScalars sc) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int64_t c = threadIdx.x; c < k; c += blockDim.x)
    if (!sc.done[c]) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) *sc.alldone = any ? 0 : 1;
}

// ---------------------------------------------------------------- apply

// part[g][j] = sum_{i in rows of g} U[i][j] r[i]   (k = 1)
template <typename TU, typename T, int LQ>
__global__ __launch_bounds__(NT) void utr_partial(int64_t n, int64_t l, const TU* __restrict__ U,
                                                  int64_t ldu, const T* __restrict__ r,
                                                  double* __restrict__ part, int64_t rpw,
                                                  const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  __shared__ T rs[NT];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  T acc[LQ];
#pragma unroll
  for (int q = 0; q < LQ; ++q) acc[q] = T(0);
  for (int64_t ib = r0; ib < r1; ib += NT) {
    __syncthreads();
    rs[t] = (ib + t < r1) ? r[ib + t] : T(0);
    __syncthreads();
    const int cnt = (int)((r1 - ib) < NT ? (r1 - ib) : NT);
    for (int ii = 0; ii < cnt; ++ii) {
      const T ri = rs[ii];
      const TU* u = U + (ib + ii) * ldu;
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        const int64_t j = t + (int64_t)q * NT;
        if (j < l) acc[q] += T(u[j]) * ri;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < LQ; ++q) {
    const int64_t j = t + (int64_t)q * NT;
    if (j < l) part[(int64_t)blockIdx.x * l + j] = double(acc[q]);
  }
}

// C'[j][c] = ((lam_l + mu_c)/(lam_j + mu_c) - 1) * sum_g part[g][j][c]
__global__ void apply_scale(int64_t l, int64_t k, int ng, const double* __restrict__ part,
                            const double* __restrict__ lam, const double* __restrict__ mu,
                            int64_t nrhs, double* __restrict__ Cs, const int* __restrict__ done) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * k) return;
  const int64_t j = idx / k, c = idx % k;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) s += part[(int64_t)g * l * k + idx];
  const double m = mu[c / nrhs];
  const double f = (lam[l - 1] + m) / (lam[j] + m) - 1.0;
  Cs[idx] = (done && done[c]) ? 0.0 : f * s;
}

// z_i = r_i + sum_j U[i][j] C'[j]  (k = 1), one wave per row, C' in LDS.
template <typename TU, typename T>
__global__ __launch_bounds__(NT) void uc_rows(int64_t n, int64_t l, const TU* __restrict__ U, int64_t ldu,
                                              const double* __restrict__ Cs, const T* __restrict__ r,
                                              T* __restrict__ z, int64_t rows_per_wave,
                                              const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  extern __shared__ char smem[];
  T* cs = reinterpret_cast<T*>(smem);
  for (int64_t j = threadIdx.x; j < l; j += NT) cs[j] = T(Cs[j]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * 4 + wave;
  const int64_t i0 = w * rows_per_wave;
  for (int64_t i = i0; i < i0 + rows_per_wave && i < n; ++i) {
    const TU* u = U + i * ldu;
    T s = T(0);
    for (int64_t j = lane; j < l; j += 64) s += T(u[j]) * cs[j];
    s = wave_sum(s);
    if (lane == 0) z[i] = r[i] + s;
  }
}

int64_t rows_per_group(int64_t n, int ng) { return cdiv(n, ng); }

}  // namespace

// ---------------------------------------------------------------- host API

nys_status precond_apply_dev(const PrecDesc& P, const double* mu_dev, int64_t nrhs, const void* R,
                             void* Z, int64_t k, bool f32, const int* done, const int* alldone,
                             double* part, size_t part_elems, double* Cs, void* Ctmp,
                             hipStream_t s) {
  const int64_t n = P.n, l = P.ell;
  const int ng = 2 * (num_cus() < 256 ? num_cus() : 256);
  if (k == 1) {
    const int64_t rpw = rows_per_group(n, ng);
    const int lq = (int)cdiv(l, NT);
#define LU(TU_, T_, LQ_)                                                                    \
  hipLaunchKernelGGL((utr_partial<TU_, T_, LQ_>), dim3(ng), dim3(NT), 0, s, n, l,          \
                     static_cast<const TU_*>(P.U), P.ldu, static_cast<const T_*>(R), part, rpw, alldone)
#define LUQ(TU_, T_) \
  if (lq <= 1) LU(TU_, T_, 1); else if (lq <= 2) LU(TU_, T_, 2); else if (lq <= 4) LU(TU_, T_, 4); else LU(TU_, T_, 8)
    if (lq > 8) { set_error("preconditioner rank > 2048 not supported"); return NYS_ERR_ARG; }
    if (P.dtype == NYS_F64 && !f32) { LUQ(double, double); }
    else if (P.dtype == NYS_F64 && f32) { LUQ(double, float); }
    else if (P.dtype == NYS_F32 && !f32) { LUQ(float, double); }
    else { LUQ(float, float); }
#undef LUQ
#undef LU
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(apply_scale, dim3((unsigned)cdiv(l, 256)), dim3(256), 0, s, l, (int64_t)1, ng,
                       part, P.lam, mu_dev, nrhs, Cs, done);
    NYS_CHECK_LAUNCH();
    const int64_t rpwave = 4;
    const unsigned nb = (unsigned)cdiv(cdiv(n, rpwave), 4);
    const size_t sh = (size_t)l * (f32 ? 4 : 8);
#define LC(TU_, T_)                                                                               \
  hipLaunchKernelGGL((uc_rows<TU_, T_>), dim3(nb), dim3(NT), sh, s, n, l, static_cast<const TU_*>(P.U), \
                     P.ldu, Cs, static_cast<const T_*>(R), static_cast<T_*>(Z), rpwave, alldone)
    if (P.dtype == NYS_F64 && !f32) LC(double, double);
    else if (P.dtype == NYS_F64 && f32) LC(double, float);
    else if (P.dtype == NYS_F32 && !f32) LC(float, double);
    else LC(float, float);
#undef LC
    NYS_CHECK_LAUNCH();
    return NYS_OK;
  }
  // block form: C = U^T R (l x k), C' = f .* C, Z = R + U C'
  if (f32) {
    set_error("float32 block preconditioner apply is not available; use k = 1 or float64");
    return NYS_ERR_ARG;
  }
  const double* Rd = static_cast<const double*>(R);
  double* Zd = static_cast<double*>(Z);
  double* C = static_cast<double*>(Ctmp);
  if (P.dtype == NYS_F64)
    NYS_TRY((gemm<double, double, double>(true, false, l, k, n, 1.0, static_cast<const double*>(P.U),
                                          P.ldu, Rd, k, 0.0, C, k, part, part_elems, s)));
  else
    NYS_TRY((gemm<double, float, double>(true, false, l, k, n, 1.0, static_cast<const float*>(P.U),
                                         P.ldu, Rd, k, 0.0, C, k, part, part_elems, s)));
  hipLaunchKernelGGL(apply_scale, dim3((unsigned)cdiv(l * k, 256)), dim3(256), 0, s, l, k, 1, C,
                     P.lam, mu_dev, nrhs, Cs, done);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemcpyAsync(Zd, Rd, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
  if (P.dtype == NYS_F64)
    NYS_TRY((gemm<double, double, double>(false, false, n, k, l, 1.0, static_cast<const double*>(P.U),
                                          P.ldu, Cs, k, 1.0, Zd, k, part, part_elems, s)));
  else
    NYS_TRY((gemm<double, float, double>(false, false, n, k, l, 1.0, static_cast<const float*>(P.U),
                                         P.ldu, Cs, k, 1.0, Zd, k, part, part_elems, s)));
  return NYS_OK;
}

size_t precond_part_elems(int64_t n, int64_t l, int64_t k) {
  const size_t a = (size_t)(2 * 256) * (size_t)l * (size_t)k;
  const size_t b = gemm_scratch_elems(l, k);
  const size_t c = gemm_scratch_elems(n, k);
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

template <typename T>
nys_status cg_kernels_init(int64_t n, int64_t k, const T* B, int64_t ldb, const T* V, T* R,
                           double* pb, double* prr, int ng, hipStream_t s) {
  const int64_t rpw = rows_per_group(n, ng);
  hipLaunchKernelGGL(cg_init_residual<T>, dim3(ng), dim3(NT), 0, s, n, k, B, ldb, V, R, pb, prr, rpw);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status cg_kernels_init2(int64_t n, int64_t k, const T* R, const T* Z, T* P, double* pb,
                            double* prr, double* prz, double tol, const CgScalars& sc, int ng,
                            hipStream_t s) {
  const int64_t rpw = rows_per_group(n, ng);
  hipLaunchKernelGGL(cg_rz_partial<T>, dim3(ng), dim3(NT), 0, s, n, k, R, Z, prz, rpw,
                     (const int*)nullptr);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_init_scalars, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, k, ng, pb, prr,
                     prz, tol, sc);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(copy_cols<T>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, Z, P);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_alldone, dim3(1), dim3(256), 0, s, k, sc);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status cg_kernels_step_a(int64_t n, int64_t k, const T* P, const T* V, T* X, int64_t ldx, T* R,
                             double* ppv, double* prr, const CgScalars& sc, int par, int ng,
                             hipStream_t s) {
  const int64_t rpw = rows_per_group(n, ng);
  hipLaunchKernelGGL(cg_pv_partial<T>, dim3(ng), dim3(NT), 0, s, n, k, P, V, ppv, rpw, sc.alldone);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_update<T>, dim3(ng), dim3(NT), 0, s, n, k, ng, ppv, sc, par, P, V, X, ldx, R,
                     prr, rpw);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status cg_kernels_step_b(int64_t n, int64_t k, const T* R, const T* Z, T* P, double* prz,
                             const double* prr, const CgScalars& sc, int par, double tol, int ng,
                             hipStream_t s) {
  const int64_t rpw = rows_per_group(n, ng);
  hipLaunchKernelGGL(cg_rz_partial<T>, dim3(ng), dim3(NT), 0, s, n, k, R, Z, prz, rpw, sc.alldone);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_direction<T>, dim3(ng), dim3(NT), 0, s, n, k, ng, prz, prr, sc, par, tol, Z, P,
                     rpw);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_alldone, dim3(1), dim3(256), 0, s, k, sc);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

#define NYS_INST(T)                                                                                  \
  template nys_status cg_kernels_init<T>(int64_t, int64_t, const T*, int64_t, const T*, T*, double*, \
                                         double*, int, hipStream_t);                                 \
  template nys_status cg_kernels_init2<T>(int64_t, int64_t, const T*, const T*, T*, double*,         \
                                          double*, double*, double, const CgScalars&, int,           \
                                          hipStream_t);                                              \
  template nys_status cg_kernels_step_a<T>(int64_t, int64_t, const T*, const T*, T*, int64_t, T*,    \
                                           double*, double*, const CgScalars&, int, int,             \
                                           hipStream_t);                                             \
  template nys_status cg_kernels_step_b<T>(int64_t, int64_t, const T*, const T*, T*, double*,        \
                                           const double*, const CgScalars&, int, double, int,        \
                                           hipStream_t);
NYS_INST(double)
NYS_INST(float)
#undef NYS_INST

}  // namespace nys
