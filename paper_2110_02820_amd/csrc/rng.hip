// Gaussian test matrix for the randomized Nystrom approximation (Section 2.2,
// first step of algorithm "Randomized Nystrom Approximation"), drawn on the
// device from a counter-based generator so that entry (i, j) depends only on
// (seed, i*l + j): Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011)
// followed by the Box-Muller transform of two 53-bit uniforms.
//   key = (seed mod 2^32, seed div 2^32); counter q = entry div 2 -> (w0..w3)
//   u1 = ((w0>>5) 2^26 + (w1>>6) + 1) 2^-53 in (0,1]
//   u2 = ((w2>>5) 2^26 + (w3>>6)) 2^-53     in [0,1)
//   even entry: sqrt(-2 ln u1) cos(2 pi u2); odd entry: ... sin(2 pi u2)
#include "rng.hpp"

namespace nys {

namespace {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void gaussian_kernel(uint64_t seed, int64_t n, int64_t l, double* __restrict__ out,
                                int64_t ld) {
  const int64_t total = n * l;
  const int64_t npair = (total + 1) / 2;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npair;
       q += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)q, (uint32_t)((uint64_t)q >> 32), 0u, 0u};
    philox10(c, k0, k1);
    const double a1 = (double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6);
    const double a2 = (double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6);
    const double u1 = (a1 + 1.0) * 1.1102230246251565e-16;  // 2^-53
    const double u2 = a2 * 1.1102230246251565e-16;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    const int64_t e0 = 2 * q, e1 = 2 * q + 1;
    out[(e0 / l) * ld + e0 % l] = rad * cos(ang);
    if (e1 < total) out[(e1 / l) * ld + e1 % l] = rad * sin(ang);
  }
}

}  // namespace

nys_status gaussian(uint64_t seed, int64_t n, int64_t l, double* out, int64_t ld, hipStream_t s) {
  const int64_t npair = (n * l + 1) / 2;
  int64_t nb = cdiv(npair, 256);
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)nb), dim3(256), 0, s, seed, n, l, out, ld);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

}  // namespace nys
