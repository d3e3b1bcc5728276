// Sketch from sampled columns (Section "Random projection versus column
// sampling"): the test matrix is Omega = I[:, S] for l distinct indices S, so
// Y = A Omega = A[:, S] is read or evaluated directly instead of formed by l
// products.  RBF: O(n l d) kernel evaluations; dense: a gather; X^T X: one
// GEMM X^T X[:, S].  Everything is float64 (operator data promoted exactly).
#include <cmath>

#include "common.hpp"
#include "gemm.hpp"

namespace nys {
namespace {

constexpr int CT = 64;  // rows and sampled columns per workgroup tile
constexpr int CD = 32;  // coordinates staged per pass

// Y[i][j] = scale exp(-|x_i - x_{S_j}|^2 / (2 sigma^2)): 64 x 64 tile per
// workgroup, 256 threads, 16 entries each; coordinates staged through LDS in
// passes of 32 (the difference form, so the entry is float64-accurate).
template <typename TD>
__global__ __launch_bounds__(256) void rbf_columns(const TD* __restrict__ X, int64_t ld, int d, int64_t n,
                                                   const int64_t* __restrict__ idx, int64_t l, double inv2s2,
                                                   double scale, double* __restrict__ Y) {
  __shared__ double xr[CT][CD + 1], xc[CT][CD + 1];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * CT, j0 = (int64_t)blockIdx.y * CT;
  const int ti = t >> 4, tj = t & 15;  // entries (ti + 16 a, tj + 16 b), a, b < 4
  double acc[4][4] = {};
  for (int k0 = 0; k0 < d; k0 += CD) {
    __syncthreads();
    for (int e = t; e < CT * CD; e += 256) {
      const int r = e / CD, k = e % CD;
      const int64_t i = i0 + r, j = j0 + r;
      const bool kin = k0 + k < d;
      xr[r][k] = (i < n && kin) ? double(X[i * ld + k0 + k]) : 0.0;
      xc[r][k] = (j < l && kin) ? double(X[idx[j] * ld + k0 + k]) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < CD; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = xr[ti + 16 * u][k];
        b[u] = xc[tj + 16 * u][k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double df = a[u] - b[v];
          acc[u][v] = fma(df, df, acc[u][v]);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + ti + 16 * u, j = j0 + tj + 16 * v;
      if (i < n && j < l) Y[i * l + j] = scale * exp(-acc[u][v] * inv2s2);
    }
}

// Y[i][j] = scale A[i][S_j]
template <typename TD>
__global__ void gather_columns(const TD* __restrict__ A, int64_t ld, int64_t rows, const int64_t* __restrict__ idx,
                               int64_t l, double scale, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * l) return;
  const int64_t i = e / l, j = e % l;
  Y[e] = scale * double(A[i * ld + idx[j]]);
}

// Omega[i][j] = (S_j == i)
__global__ void selection_fill(int64_t n, int64_t l, const int64_t* __restrict__ idx, double* __restrict__ Om) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * l) return;
  const int64_t i = e / l, j = e % l;
  Om[e] = idx[j] == i ? 1.0 : 0.0;
}

__global__ void zero_ints(int64_t count, int* __restrict__ p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0;
}

// bad[0] = 1 if some index is outside [0, n), bad[1] = 1 if some index repeats
__global__ void check_indices(int64_t n, int64_t l, const int64_t* __restrict__ idx, int* __restrict__ mark,
                              int* __restrict__ bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= l) return;
  const int64_t v = idx[j];
  if (v < 0 || v >= n) {
    atomicOr(&bad[0], 1);
    return;
  }
  if (atomicAdd(&mark[v], 1) != 0) atomicOr(&bad[1], 1);
}

unsigned nb256(int64_t count) { return (unsigned)cdiv(count, 256); }

struct ColWs {
  int* mark;
  int* bad;
  double* Xs;
  double* gscr;
  size_t gscr_elems;
};

void carve_columns(Arena& a, const nys_operator* A, int64_t l, ColWs& w) {
  w.mark = a.take<int>(A->n);
  w.bad = a.take<int>(2);
  if (A->kind == NYS_OP_XTX) {
    w.Xs = a.take<double>((size_t)A->rows * (size_t)l);
    w.gscr_elems = gemm_scratch_elems(A->n, l);
    w.gscr = a.take<double>(w.gscr_elems);
  } else {
    w.Xs = nullptr;
    w.gscr = nullptr;
    w.gscr_elems = 0;
  }
}

template <typename TD>
nys_status columns_impl(const nys_operator* A, int64_t l, const int64_t* idx, double* Y, ColWs& w, hipStream_t s) {
  const TD* X = static_cast<const TD*>(A->data);
  const int64_t n = A->n;
  if (A->kind == NYS_OP_RBF) {
    const dim3 grid((unsigned)cdiv(n, CT), (unsigned)cdiv(l, CT));
    const double inv2s2 = 1.0 / (2.0 * A->sigma * A->sigma);
    hipLaunchKernelGGL((rbf_columns<TD>), grid, dim3(256), 0, s, X, A->ld, (int)A->cols, n, idx, l, inv2s2,
                       A->scale, Y);
    NYS_CHECK_LAUNCH();
  } else if (A->kind == NYS_OP_DENSE) {
    hipLaunchKernelGGL((gather_columns<TD>), dim3(nb256(n * l)), dim3(256), 0, s, X, A->ld, n, idx, l, A->scale, Y);
    NYS_CHECK_LAUNCH();
  } else {
    // Y = scale X^T X[:, S]
    hipLaunchKernelGGL((gather_columns<TD>), dim3(nb256(A->rows * l)), dim3(256), 0, s, X, A->ld, A->rows, idx, l,
                       1.0, w.Xs);
    NYS_CHECK_LAUNCH();
    NYS_TRY((gemm<double, TD, double>(true, false, n, l, A->rows, A->scale, X, A->ld, w.Xs, l, 0.0, Y, l, w.gscr,
                                      w.gscr_elems, s)));
  }
  return NYS_OK;
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_workspace_size_columns(const nys_operator* A, int64_t ell) {
  if (A == nullptr || ell < 1 || A->n < 1 || A->kind == NYS_OP_CALLBACK) return 0;
  Arena a(nullptr, 0);
  ColWs w;
  carve_columns(a, A, ell, w);
  return a.off + 256;
}

nys_status nys_sketch_columns(const nys_operator* A, int64_t ell, const int64_t* idx, double* Omega_out,
                              double* Y_out, void* ws, size_t ws_bytes, void* stream) {
  NYS_ARG(A != nullptr && idx != nullptr && Omega_out != nullptr && Y_out != nullptr,
          "nys_sketch_columns: NULL argument");
  NYS_ARG(A->kind != NYS_OP_CALLBACK, "the column-sampling sketch reads entries of A: a callback operator has none");
  NYS_ARG(A->data != nullptr && A->n >= 1 && (A->dtype == NYS_F64 || A->dtype == NYS_F32), "invalid operator");
  NYS_ARG(A->kind == NYS_OP_DENSE || A->kind == NYS_OP_XTX || A->kind == NYS_OP_RBF, "unknown operator kind");
  NYS_ARG(A->scale > 0.0 && std::isfinite(A->scale), "operator scale must be > 0");
  NYS_ARG(A->kind != NYS_OP_RBF || (A->sigma > 0.0 && std::isfinite(A->sigma)), "RBF sigma must be > 0");
  NYS_ARG(A->ld >= A->cols && A->rows >= 1 && A->cols >= 1, "invalid operator shape");
  NYS_ARG(A->kind != NYS_OP_DENSE || (A->rows == A->n && A->cols == A->n), "dense operator must be n x n");
  NYS_ARG(A->kind != NYS_OP_XTX || A->cols == A->n, "X^T X operator: data must have n columns");
  NYS_ARG(A->weights == nullptr, "column sampling: weighted X^T X operators are not supported");
  NYS_ARG(A->kind != NYS_OP_RBF || A->rows == A->n, "RBF operator: data must have n rows");
  const int64_t n = A->n;
  NYS_ARG(ell >= 1 && ell <= n, "need 1 <= ell <= n");
  Arena a(ws, ws_bytes);
  ColWs w;
  carve_columns(a, A, ell, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the indices must be distinct and inside [0, n)
  hipLaunchKernelGGL(zero_ints, dim3(nb256(n + 2)), dim3(256), 0, s, n, w.mark);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(zero_ints, dim3(1), dim3(256), 0, s, (int64_t)2, w.bad);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(check_indices, dim3(nb256(ell)), dim3(256), 0, s, n, ell, idx, w.mark, w.bad);
  NYS_CHECK_LAUNCH();
  int bad[2] = {0, 0};
  NYS_HIP(hipMemcpyAsync(bad, w.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  NYS_ARG(!bad[0], "nys_sketch_columns: an index lies outside [0, n)");
  NYS_ARG(!bad[1], "nys_sketch_columns: indices must be distinct");
  hipLaunchKernelGGL(selection_fill, dim3(nb256(n * ell)), dim3(256), 0, s, n, ell, idx, Omega_out);
  NYS_CHECK_LAUNCH();
  if (A->dtype == NYS_F64) return columns_impl<double>(A, ell, idx, Y_out, w, s);
  return columns_impl<float>(A, ell, idx, Y_out, w, s);
}

}  // extern "C"
