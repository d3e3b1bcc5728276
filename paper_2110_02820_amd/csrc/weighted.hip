// Weighted normal equations A = scale X^T D X, D = diag(d), d >= 0: the data
// term of the Hessian of a regularised generalised linear model (logistic
// weights p (1 - p)), the operator of approximate leave-one-out
// cross-validation (Section 6.3, "Approximate cross-validation").  The
// solvers take the weights inside every X^T X product (float64 d); this file
// holds the helper that folds them into a copy of the data instead,
// Xw = D^{1/2} X, so that Xw^T Xw = X^T D X up to the rounding of Xw's type.
#include <cmath>
#include <cstdint>

#include "common.hpp"

namespace nys {
namespace {

// bad[0] = 1 if some weight is negative or not finite
__global__ void check_weights(int64_t rows, const double* __restrict__ d, int* __restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = d[i];
    if (!(v >= 0.0) || !std::isfinite(v)) atomicOr(&bad[0], 1);
  }
}

__global__ void clear_flag(int* __restrict__ bad) { bad[0] = 0; }

// Xw[i][:] = sqrt(d_i) X[i][:], one workgroup per row at a time (coalesced
// over the columns; the grid strides over the rows).  X and Xw may be the
// same array (in place, same leading dimension): every entry is read before
// it is written by the same thread.
template <typename T>
__global__ __launch_bounds__(256) void weight_rows(int64_t rows, int64_t cols, const T* X, int64_t ldx,
                                                   const double* __restrict__ d, T* Xw, int64_t ldw) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    const T s = T(sqrt(d[i]));
    const T* xr = X + i * ldx;
    T* wr = Xw + i * ldw;
    for (int64_t j = threadIdx.x; j < cols; j += 256) wr[j] = s * xr[j];
  }
}

// The same with 16-byte accesses (float4 / double2) when every row starts on
// a 16-byte boundary and the columns fill whole vectors; the products are the
// scalar kernel's, element by element.
__global__ __launch_bounds__(256) void weight_rows_f4(int64_t rows, int64_t cvec, const float* X, int64_t ldx,
                                                      const double* __restrict__ d, float* Xw, int64_t ldw) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    const float s = float(sqrt(d[i]));
    const float4* xr = reinterpret_cast<const float4*>(X + i * ldx);
    float4* wr = reinterpret_cast<float4*>(Xw + i * ldw);
    for (int64_t j = threadIdx.x; j < cvec; j += 256) {
      float4 v = xr[j];
      v.x = s * v.x;
      v.y = s * v.y;
      v.z = s * v.z;
      v.w = s * v.w;
      wr[j] = v;
    }
  }
}

__global__ __launch_bounds__(256) void weight_rows_d2(int64_t rows, int64_t cvec, const double* X, int64_t ldx,
                                                      const double* __restrict__ d, double* Xw, int64_t ldw) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    const double s = sqrt(d[i]);
    const double2* xr = reinterpret_cast<const double2*>(X + i * ldx);
    double2* wr = reinterpret_cast<double2*>(Xw + i * ldw);
    for (int64_t j = threadIdx.x; j < cvec; j += 256) {
      double2 v = xr[j];
      v.x = s * v.x;
      v.y = s * v.y;
      wr[j] = v;
    }
  }
}

// at most this many workgroups (the grid strides over further rows)
constexpr int64_t kMaxRowGroups = 65536;

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_workspace_size_weight_rows(void) { return 256; }

nys_status nys_weight_rows(int64_t rows, int64_t cols, int32_t dtype, const void* X, int64_t ldx,
                           const double* d, void* Xw, int64_t ldw, void* ws, size_t ws_bytes, void* stream) {
  NYS_ARG(X != nullptr && d != nullptr && Xw != nullptr, "nys_weight_rows: NULL argument");
  NYS_ARG(rows >= 1 && cols >= 1 && ldx >= cols && ldw >= cols, "nys_weight_rows: invalid shape");
  NYS_ARG(rows <= 0x7fffffff, "nys_weight_rows: more than 2^31 - 1 rows");
  NYS_ARG(dtype == NYS_F64 || dtype == NYS_F32, "nys_weight_rows: dtype must be NYS_F64 or NYS_F32");
  NYS_ARG(X != Xw || ldx == ldw, "nys_weight_rows: in place needs ldw == ldx");
  if (ws == nullptr || ws_bytes < nys_workspace_size_weight_rows()) {
    set_error("workspace too small: need %zu bytes", nys_workspace_size_weight_rows());
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* bad = static_cast<int*>(ws);
  hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, s, bad);
  NYS_CHECK_LAUNCH();
  const int64_t nb = cdiv(rows, 256) < 1024 ? cdiv(rows, 256) : 1024;
  hipLaunchKernelGGL(check_weights, dim3((unsigned)nb), dim3(256), 0, s, rows, d, bad);
  NYS_CHECK_LAUNCH();
  int bad_h = 0;
  NYS_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  NYS_ARG(!bad_h, "nys_weight_rows: weights must be finite and >= 0");
  // 16-byte accesses when each row starts 16-byte aligned and holds whole vectors
  const int w = dtype == NYS_F64 ? 2 : 4;
  const bool vec = aligned16(X) && aligned16(Xw) && cols % w == 0 && ldx % w == 0 && ldw % w == 0;
  const dim3 grid((unsigned)(rows < kMaxRowGroups ? rows : kMaxRowGroups));
  if (dtype == NYS_F64 && vec)
    hipLaunchKernelGGL(weight_rows_d2, grid, dim3(256), 0, s, rows, cols / 2, static_cast<const double*>(X), ldx, d,
                       static_cast<double*>(Xw), ldw);
  else if (dtype == NYS_F64)
    hipLaunchKernelGGL(weight_rows<double>, grid, dim3(256), 0, s, rows, cols, static_cast<const double*>(X), ldx, d,
                       static_cast<double*>(Xw), ldw);
  else if (vec)
    hipLaunchKernelGGL(weight_rows_f4, grid, dim3(256), 0, s, rows, cols / 4, static_cast<const float*>(X), ldx, d,
                       static_cast<float*>(Xw), ldw);
  else
    hipLaunchKernelGGL(weight_rows<float>, grid, dim3(256), 0, s, rows, cols, static_cast<const float*>(X), ldx, d,
                       static_cast<float*>(Xw), ldw);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

}  // extern "C"
