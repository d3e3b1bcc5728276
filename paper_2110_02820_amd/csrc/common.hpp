// Shared device/host utilities for the Nystrom PCG library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "nyspcg.h"

namespace nys {

// ---------------------------------------------------------------- host side
void set_error(const char* fmt, ...);

#define NYS_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::nys::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,              \
                       hipGetErrorString(e_));                                 \
      return NYS_ERR_DEVICE;                                                   \
    }                                                                          \
  } while (0)

#define NYS_CHECK_LAUNCH() NYS_HIP(hipGetLastError())

#define NYS_ARG(cond, ...)                                                     \
  do {                                                                         \
    if (!(cond)) {                                                             \
      ::nys::set_error(__VA_ARGS__);                                           \
      return NYS_ERR_ARG;                                                      \
    }                                                                          \
  } while (0)

#define NYS_TRY(expr)                                                          \
  do {                                                                         \
    nys_status s_ = (expr);                                                    \
    if (s_ != NYS_OK) return s_;                                               \
  } while (0)

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures, so the same code path yields nys_workspace_size().
struct Arena {
  char* base;
  size_t cap;
  size_t off = 0;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  bool ok() const { return base == nullptr || off <= cap; }
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int num_cus();  // compute units of the current device

// Measurement hook around the launch of the X^T X product kernel: records a
// HIP event on s when nys_timing_begin() has enabled timing on this thread.
void timing_mark_begin(hipStream_t s);
void timing_mark_end(hipStream_t s);

// 256 bytes of pinned host memory per host thread, kept for the life of the
// process (null if it cannot be had): state the device writes for host loops
// that poll without synchronising the stream.  Bytes 0..63: eigensolver
// sweeps; bytes 64..127: PCG batch snapshots; bytes 128..151: the pivot
// flags (and shift) of the sketch's CholeskyQR and the factorisation's
// Cholesky; bytes 160..175: a solve's single-column residual and its
// completion tag.
int* pinned_flags();

// Next value of a per-thread sequence that tags what the device writes into
// pinned memory, so a host loop can tell a fresh write from an older one.
int next_pinned_seq();

// Wait until *seq is expect or alt (alt = 0: expect only), written by a
// kernel on stream s.  Spins on the host; after ~2 s without the value it
// synchronises the stream and looks once more.  False (message set) if the
// value never came or the stream failed.
bool wait_pinned(const volatile int* seq, int expect, hipStream_t s, int alt = 0);

// --------------------------------------------------------------- device side
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block reduction (deterministic): wave shuffles then one wave
// combines the per-wave sums.  `sh` needs blockDim.x/64 entries.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  T r = (threadIdx.x < nw) ? sh[threadIdx.x] : T(0);
  if (w == 0) r = wave_sum(r);
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = r;
  __syncthreads();
  r = sh[0];
  __syncthreads();
  return r;
}

// block_sum with one barrier: every thread adds the per-wave sums in the same
// order.  `sh` (blockDim.x/64 entries) must not be written again until every
// thread has read it: give each call its own array, or put a barrier between.
template <typename T>
__device__ __forceinline__ T block_sum1(T v, T* sh) {
  v = wave_sum(v);
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  for (int w = 1; w < nw; ++w) r += sh[w];
  return r;
}

}  // namespace nys
