// Small dense float64 linear algebra on the l x l core of the Nystrom
// factorisation (Section 2.2, algorithm "Randomized Nystrom Approximation",
// steps 4-9), all on the device and stream-ordered (no host round trips
// except the convergence polls of the eigensolver):
//   * shift nu = eps(||Y||_F) (raised for reduced-precision sketches) and
//     Y_nu = Y + nu Omega
//   * blocked right-looking Cholesky, one launch per block step
//     (diagonal block by one wave, panel, trailing update)
//   * inverse of the lower-triangular factor by recursive doubling over
//     block pairs
//   * symmetric eigensolver: block two-sided Jacobi with the round-robin
//     ordering of block pairs; one launch per round solves the 32 x 32
//     subproblems in LDS and applies the previous round's rotations to the
//     off-diagonal tiles on FP64 MFMA
//   * descending sort of the eigenvalues and the scaled eigenvector matrix
#include <cstdlib>
#include <cstring>

#include "dense_small.hpp"

namespace nys {

namespace {

constexpr int NB = 32;  // block size of the blocked Cholesky / inverse

// Reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64 / v_rsq_f64) refined by one Newton step, which restores full
// float64 accuracy; they replace IEEE division / square root on the short
// dependent chains of the rotation and pivot computations.
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double frsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y * fma(-0.5 * x, y * y, 1.5);
}


// ---------------------------------------------------------------- shift

__global__ void sumsq_partial(const double* __restrict__ Y, int64_t count,
                              double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = Y[i];
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// nu = spacing of ||Y||_F: for |x| = f 2^e (0.5 <= f < 1), 2^(e - 53).
__global__ void finalize_nu(const double* __restrict__ part, int np, double u_rel, double* __restrict__ nu) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s);
    int e = 0;
    frexp(nrm, &e);
    const double eps_nrm = (nrm > 0.0) ? ldexp(1.0, e - 53) : 4.9406564584124654e-324;
    nu[0] = fmax(eps_nrm, u_rel * nrm);
  }
}

__global__ void axpy_nu(double* __restrict__ Y, const double* __restrict__ Om, int64_t count,
                        const double* __restrict__ nu, double factor) {
  const double a = nu[0] * factor;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    Y[i] += a * Om[i];
}

__global__ void scale_scalar(double* __restrict__ nu, double factor) { nu[0] *= factor; }

// ---------------------------------------------------------------- Cholesky

// L (lower, ld = n) <- (M + M^T)/2 lower triangle; upper triangle zeroed.
__global__ void symmetrize_lower(const double* __restrict__ M, int64_t n, double* __restrict__ L) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  L[idx] = (j <= i) ? 0.5 * (M[i * n + j] + M[j * n + i]) : 0.0;
}

struct CholArgs {
  double* L;        // n x n, in: symmetric lower part, out: factor
  int64_t n;
  double* Dinv;     // nblk x NB x NB inverses of the diagonal blocks
  int* info;        // 0 = ok, k+1 = non-positive pivot at column k
};

// Blocked right-looking Cholesky with one launch per step.  Launch kb
// updates the trailing matrix with the panel of block column kb and factors
// diagonal block kb + 1 in the same workgroup that updated it; the
// sub-diagonal blocks keep their Schur-complement values A[ib][kb] until one
// last launch turns them all into L[ib][kb] = A[ib][kb] L_kk^{-T}.

// The 16 x 16 steps of diag_factor run on one wave, lane l holding row
// l mod 16 of the block in registers (four copies of each row): in the
// factorisation, entries of other rows come from v_readlane, so no LDS round
// trip or barrier sits on the chain of dependent column steps.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Right-looking Cholesky of the 16 x 16 block T[o..o+15][o..o+15] (lower part
// read) into L (written back to T, zeros above the diagonal) and its inverse
// into Li[o..o+15][o..o+15] (zeros above).  Column j: the pivot from lane j,
// l_i = a_ij / sqrt(pivot), then a_ik -= l_i l_k for k > j.  A pivot that is
// not positive and finite is replaced by 1 (recorded in *bad, the first one).
// The inverse is forward substitution by columns: lane i forms column i,
// x_m = (delta_mi - sum_{k<m} L_mk x_k) / L_mm, with the rows of L read back
// from LDS.
__device__ __forceinline__ void chol16(double (*T)[NB + 1], double (*Li)[NB + 1], int o, int& bad) {
  const int lane = threadIdx.x & 63, i = lane & 15;
  double r[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) r[j] = (j <= i) ? T[o + i][o + j] : 0.0;
  double ys[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double d = lane_bcast(r[j], j);
    double y;
    if (!(d > 0.0) || !isfinite(d)) {  // the same for every lane
      if (bad < 0) bad = j;
      d = 1.0;
      y = 1.0;
    } else {
      y = frsq(d);
    }
    ys[j] = y;
    const double l = (i > j) ? r[j] * y : (i == j ? d * y : 0.0);
    r[j] = l;
#pragma unroll
    for (int k = j + 1; k < 16; ++k) r[k] -= l * lane_bcast(l, k);  // rows i < k: unused values
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) T[o + i][o + j] = (j <= i) ? r[j] : 0.0;
  }
  wave_lds_sync();
  // rows of L as LDS broadcasts (every lane reads the same address)
  double x[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    double s0 = (m == i) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < m; k += 2) {
      s0 -= T[o + m][o + k] * x[k];
      if (k + 1 < m) s1 -= T[o + m][o + k + 1] * x[k + 1];
    }
    x[m] = (s0 + s1) * ys[m];
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) Li[o + j][o + i] = x[j];  // column i of the inverse (0 above the diagonal)
  }
}

typedef double cd4 __attribute__((ext_vector_type(4)));

// out = sgn * X Y (+ C) for 16 x 16 blocks on MFMA f64 (one wave): X[r][k]
// = xm(r, k), Y[k][c] = ym(k, c); accumulator element q of lane l is
// out[4 q + l / 16][l % 16].
template <typename FX, typename FY>
__device__ __forceinline__ cd4 mm16(FX xm, FY ym, cd4 acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xm(lane & 15, kk), ym(kk, lane & 15), acc, 0, 0, 0);
  }
  return acc;
}

// out = X Y (+ acc) for 32 x 32 blocks on MFMA f64, four waves: wave w
// forms the 16 x 16 quadrant (w / 2, w % 2); X[r][k] = xm(r, k), Y[k][c] =
// ym(k, c); accumulator element q of lane l is out[16 (w / 2) + 4 q + l / 16]
// [16 (w % 2) + l % 16].
template <typename FX, typename FY>
__device__ __forceinline__ cd4 mm32q(FX xm, FY ym, cd4 acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = (wave >> 1) * 16 + (lane & 15), c = (wave & 1) * 16 + (lane & 15);
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xm(r, kk), ym(kk, c), acc, 0, 0, 0);
  }
  return acc;
}

// Cholesky + inverse of one NB x NB (= 32) diagonal block held in T (lower
// part, identity outside the matrix), by one wave in two 16-column halves:
// L11 = chol(A11), L21 = A21 L11^{-T}, L22 = chol(A22 - L21 L21^T), and
// L^{-1} = [L11^{-1} 0; -L22^{-1} L21 L11^{-1}  L22^{-1}], the 16 x 16
// products on MFMA.  Writes the factor block to L, the inverse to Dinv (kb),
// the first bad pivot to info.  Li, Mb: LDS scratch (NB x NB + 1).  Only
// wave 0 of the workgroup may call it, and no barrier is taken inside.
__device__ __forceinline__ void diag_factor(const CholArgs& a, int kb, double (*T)[NB + 1], double (*Li)[NB + 1],
                                            double (*Mb)[NB + 1]) {
  double* __restrict__ Lg = a.L;
  double* __restrict__ Dg = a.Dinv;
  const int64_t n = a.n;
  const int64_t base = (int64_t)kb * NB;
  const int nbk = (int)((n - base) < NB ? (n - base) : NB);
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, q4 = lane >> 4;
  int bad = -1, bad2 = -1;
  chol16(T, Li, 0, bad);
  wave_lds_sync();
  // L21 = A21 L11^{-T}
  cd4 acc = mm16([&](int r, int k) { return T[16 + r][k]; }, [&](int k, int c) { return Li[c][k]; },
                 cd4{0.0, 0.0, 0.0, 0.0});
  wave_lds_sync();  // every lane has read A21
#pragma unroll
  for (int q = 0; q < 4; ++q) T[16 + 4 * q + q4][r16] = acc[q];
  wave_lds_sync();
  // A22 - L21 L21^T
  cd4 c22;
#pragma unroll
  for (int q = 0; q < 4; ++q) c22[q] = T[16 + 4 * q + q4][16 + r16];
  acc = mm16([&](int r, int k) { return -T[16 + r][k]; }, [&](int k, int c) { return T[16 + c][k]; }, c22);
#pragma unroll
  for (int q = 0; q < 4; ++q) T[16 + 4 * q + q4][16 + r16] = acc[q];
  wave_lds_sync();
  chol16(T, Li, 16, bad2);
  if (bad < 0 && bad2 >= 0) bad = 16 + bad2;
  // M = L21 L11^{-1}, then L21' = -L22^{-1} M
  acc = mm16([&](int r, int k) { return T[16 + r][k]; }, [&](int k, int c) { return Li[k][c]; },
             cd4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
  for (int q = 0; q < 4; ++q) Mb[4 * q + q4][r16] = acc[q];
  wave_lds_sync();
  acc = mm16([&](int r, int k) { return -Li[16 + r][16 + k]; }, [&](int k, int c) { return Mb[k][c]; },
             cd4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Li[16 + 4 * q + q4][r16] = acc[q];
    Li[4 * q + q4][16 + r16] = 0.0;
  }
  wave_lds_sync();
  if (bad >= 0 && bad < nbk && lane == 0) atomicCAS(a.info, 0, (int)(base + bad + 1));
  // the block of L (rows and columns inside the matrix) and all of L^{-1}
#pragma unroll
  for (int u = 0; u < NB * NB / 64; ++u) {
    const int e = lane + 64 * u, i = e / NB, j = e % NB;
    if (i < nbk && j < nbk) Lg[(base + i) * n + base + j] = T[i][j];
    Dg[(int64_t)kb * NB * NB + e] = Li[i][j];
  }
}

// Diagonal block kb by one wave (the first block; later ones are factored
// inside chol_step).
__global__ __launch_bounds__(64) void chol_diag(CholArgs a, int kb) {
  if (*((volatile int*)a.info) != 0) return;
  __shared__ double T[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double Mb[NB][NB + 1];
  const int64_t n = a.n;
  const int64_t base = (int64_t)kb * NB;
  const int nbk = (int)((n - base) < NB ? (n - base) : NB);
  const int t = threadIdx.x;
  double v[NB * NB / 64];
#pragma unroll
  for (int u = 0; u < NB * NB / 64; ++u) {
    const int e = t + 64 * u, i = e / NB, j = e % NB;
    v[u] = (i < nbk && j < nbk && j <= i) ? a.L[(base + i) * n + base + j] : (i == j ? 1.0 : 0.0);
  }
#pragma unroll
  for (int u = 0; u < NB * NB / 64; ++u) {
    const int e = t + 64 * u;
    T[e / NB][e % NB] = v[u];  // padding outside the matrix: identity
  }
  __syncthreads();
  diag_factor(a, kb, T, Li, Mb);
}

// Row and column (ii >= jj) of lower-triangle tile number tt.
__device__ __forceinline__ void tri_tile(int tt, int& ii, int& jj) {
  ii = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= tt) ++ii;
  while (ii * (ii + 1) / 2 > tt) --ii;
  jj = tt - ii * (ii + 1) / 2;
}

// Step kb, tile (ib, jb) with kb < jb <= ib, one workgroup each:
// A[ib][jb] -= L[ib][kb] L[jb][kb]^T, where the workgroup forms the panel
// blocks it needs itself, L[xb][kb] = A[xb][kb] Dinv_kb^T (column kb still
// holds Schur-complement values in this launch).  The workgroup of tile
// (kb + 1, kb + 1), which no other workgroup of the launch reads or writes,
// then factors and inverts that block.
__global__ __launch_bounds__(256) void chol_step(CholArgs a, int kb) {
  __shared__ double Pi[NB][NB + 1], Pj[NB][NB + 1], Di[NB][NB + 1], T[NB][NB + 1];
  __shared__ int stop;
  const int64_t n = a.n;
  const int t = threadIdx.x;
  int ii, jj;
  tri_tile((int)blockIdx.x, ii, jj);
  const int ib = kb + 1 + ii, jb = kb + 1 + jj;
  const int64_t c0 = (int64_t)kb * NB, cj = (int64_t)jb * NB;
  double* __restrict__ Lg = a.L;
  if (t == 0) stop = *((volatile int*)a.info);  // read once: the flag may change during the launch
  {
    double vi[NB * NB / 256], vj[NB * NB / 256], vd[NB * NB / 256], vt[NB * NB / 256];
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = t + 256 * u, i = e / NB, k = e % NB;
      const int64_t ri = (int64_t)ib * NB + i, rj = cj + i;
      vi[u] = ri < n ? Lg[ri * n + c0 + k] : 0.0;
      vj[u] = rj < n ? Lg[rj * n + c0 + k] : 0.0;
      vd[u] = a.Dinv[c0 * NB + e];
      vt[u] = (ri < n && cj + k < n) ? Lg[ri * n + cj + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = t + 256 * u;
      Pi[e / NB][e % NB] = vi[u];
      Pj[e / NB][e % NB] = vj[u];
      Di[e / NB][e % NB] = vd[u];
      T[e / NB][e % NB] = vt[u];
    }
  }
  __syncthreads();
  if (stop != 0) return;  // the same value for every thread
  static_assert(NB == 32, "the MFMA quadrants assume 32 x 32 blocks");
  const int lane = t & 63, wave = t >> 6;
  const int qr = (wave >> 1) * 16 + (lane >> 4), qc = (wave & 1) * 16 + (lane & 15);  // + 4 q: this lane's rows
  // panel blocks: P <- P Dinv^T (Dinv lower triangular, zeros above)
  {
    const cd4 zero = {0.0, 0.0, 0.0, 0.0};
    const cd4 ai = mm32q([&](int r, int k) { return Pi[r][k]; }, [&](int k, int c) { return Di[c][k]; }, zero);
    const cd4 aj = mm32q([&](int r, int k) { return Pj[r][k]; }, [&](int k, int c) { return Di[c][k]; }, zero);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Pi[qr + 4 * q][qc] = ai[q];
      Pj[qr + 4 * q][qc] = aj[q];
    }
  }
  __syncthreads();
  const bool diag_next = ii == 0;  // tile (kb + 1, kb + 1)
  const int nbk = (int)((n - cj) < NB ? (n - cj) : NB);
  // A[ib][jb] - L[ib][kb] L[jb][kb]^T
  cd4 upd;
#pragma unroll
  for (int q = 0; q < 4; ++q) upd[q] = T[qr + 4 * q][qc];
  upd = mm32q([&](int r, int k) { return -Pi[r][k]; }, [&](int k, int c) { return Pj[c][k]; }, upd);
  if (!diag_next) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gi = (int64_t)ib * NB + qr + 4 * q, gj = cj + qc;
      if (gi < n && gj < n && gj <= gi) Lg[gi * n + gj] = upd[q];
    }
    return;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = qr + 4 * q, j = qc;
    T[i][j] = (i < nbk && j < nbk && j <= i) ? upd[q] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  // the panels and Dinv_kb are no longer read: their LDS serves as scratch
  if (t < 64) diag_factor(a, jb, T, Di, Pi);
}

// All sub-diagonal blocks: L[ib][kb] = A[ib][kb] Dinv_kb^T, one workgroup
// per block (strict lower-triangle tile number tt).
__global__ __launch_bounds__(256) void chol_panels(CholArgs a) {
  if (*((volatile int*)a.info) != 0) return;
  __shared__ double Ti[NB][NB + 1];
  __shared__ double Lb[NB][NB + 1];
  const int64_t n = a.n;
  const int t = threadIdx.x;
  int ii, kb;
  tri_tile((int)blockIdx.x, ii, kb);
  const int ib = ii + 1;
  double* __restrict__ Lg = a.L;
  const double* __restrict__ Di = a.Dinv + (int64_t)kb * NB * NB;
  const int64_t r0 = (int64_t)ib * NB, c0 = (int64_t)kb * NB;
  {
    double v[NB * NB / 256], w[NB * NB / 256];
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = t + 256 * u, i = e / NB, j = e % NB;
      v[u] = (r0 + i < n) ? Lg[(r0 + i) * n + c0 + j] : 0.0;
      w[u] = Di[e];
    }
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = t + 256 * u;
      Lb[e / NB][e % NB] = v[u];
      Ti[e / NB][e % NB] = w[u];
    }
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  const int qr = (wave >> 1) * 16 + (lane >> 4), qc = (wave & 1) * 16 + (lane & 15);
  const cd4 acc = mm32q([&](int r, int k) { return Lb[r][k]; }, [&](int k, int c) { return Ti[c][k]; },
                        cd4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (r0 + qr + 4 * q < n) Lg[(r0 + qr + 4 * q) * n + c0 + qc] = acc[q];
}

// ---------------------------------------------------------------- L^{-1}

// L^{-1} by recursive doubling over the diagonal blocks.  With X11, X22 the
// inverses of two neighbouring diagonal blocks of size bs and L21 the block
// below the first, the inverse of the pair is [X11 0; X21 X22] with
// X21 = -X22 (L21 X11).  Level bs = NB, 2 NB, ... doubles the inverted blocks;
// each level is two launches (T = L21 X11, then X21 = -X22 T), parallel over
// pairs and 32 x 32 output tiles.  T is kept in the mirror block X12 of the
// strict upper triangle, which is cleared at the end; only block-lower tiles
// of X11 and X22 are read, so stale T blocks are never used.

// X = 0 except the diagonal blocks (Dinv).
__global__ void trinv_init(int64_t n, const double* __restrict__ Dinv, double* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  const int64_t bi = i / NB, bj = j / NB;
  X[idx] = (bi == bj) ? Dinv[bi * NB * NB + (i % NB) * NB + (j % NB)] : 0.0;
}

// phase 0: T = L21 X11 (stored at X12); phase 1: X21 = -X22 T.
// Grid: (tiles per pair (bs/NB)^2, pairs).  256 threads, 4 outputs each.
__global__ __launch_bounds__(256) void trinv_level(const double* __restrict__ L, int64_t n, double* X,
                                                   int64_t bs, int phase) {
  __shared__ double As[NB][NB + 1];
  __shared__ double Bs[NB][NB + 1];
  const int64_t tb = bs / NB;
  const int64_t ti = blockIdx.x / tb, tj = blockIdx.x % tb;
  const int64_t o1 = (int64_t)blockIdx.y * 2 * bs, o2 = o1 + bs;  // offsets of blocks 1 and 2
  if (o2 >= n) return;
  const int t = threadIdx.x;
  const int ci = t >> 3, cj0 = (t & 7) * 4;  // row ci, columns cj0 .. cj0 + 3 of the tile
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // phase 0: sum over k-blocks kb >= tj (X11 block-lower); phase 1: kb <= ti (X22 block-lower)
  const int64_t kb0 = phase == 0 ? tj : 0, kb1 = phase == 0 ? tb : ti + 1;
  for (int64_t kb = kb0; kb < kb1; ++kb) {
    __syncthreads();
    double va[4], vb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u, r = e / NB, c = e % NB;
      int64_t ar, ac, br, bc;
      const double* Ap;
      if (phase == 0) {  // A = L21 tile (ti, kb), B = X11 tile (kb, tj)
        ar = o2 + ti * NB + r; ac = o1 + kb * NB + c; Ap = L;
        br = o1 + kb * NB + r; bc = o1 + tj * NB + c;
      } else {           // A = X22 tile (ti, kb), B = T tile (kb, tj) at X12 (transposed position)
        ar = o2 + ti * NB + r; ac = o2 + kb * NB + c; Ap = X;
        br = o1 + tj * NB + c; bc = o2 + kb * NB + r;
      }
      va[u] = (ar < n && ac < n) ? Ap[ar * n + ac] : 0.0;
      vb[u] = (br < n && bc < n) ? X[br * n + bc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u;
      As[e / NB][e % NB] = va[u];
      Bs[e / NB][e % NB] = vb[u];
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < NB; ++k) {
      const double av = As[ci][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += av * Bs[k][cj0 + q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t r = ti * NB + ci, c = tj * NB + cj0 + q;
    if (phase == 0) {  // T[r][c] -> X[o1 + c][o2 + r]
      if (o1 + c < n && o2 + r < n) X[(o1 + c) * n + o2 + r] = acc[q];
    } else {
      if (o2 + r < n && o1 + c < n) X[(o2 + r) * n + o1 + c] = -acc[q];
    }
  }
}

// zero the strict upper triangle
__global__ void trinv_clear_upper(int64_t n, double* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  if (j > i && j / NB != i / NB) X[idx] = 0.0;
}

// ---------------------------------------------------------------- Jacobi

constexpr int JB = 16;       // Jacobi block size
constexpr int JS = 2 * JB;   // order of one block-pair subproblem
constexpr int JH = JS / 2;   // rotation pairs per inner round
constexpr int JSS = JS + 16;  // LDS row stride of the subproblem rounds

// Position pos of round r of the round-robin schedule over m slots (pos, r < m):
// slot 0 stays, the others rotate.  32-bit, no division.
__device__ __forceinline__ int rr_index(int pos, int r, int m) {
  int x = pos - 1 + r;
  if (x >= m - 1) x -= m - 1;
  return pos == 0 ? 0 : 1 + x;
}

// Rotation (c, s) with J_pp = c, J_pq = s, J_qp = -s, J_qq = c that zeroes
// entry (p, q) of J^T A J (symmetric 2x2 Schur decomposition).  Returns false
// (identity) when |a_pq| is below max(eps sqrt(|a_pp a_qq|), floor_abs).
__device__ __forceinline__ bool jacobi_rot(double app, double aqq, double apq, double floor_abs,
                                           double& c, double& s) {
  const double a2 = apq * apq;
  const double thr2 = fmax(4.930380657631324e-32 * fabs(app * aqq), floor_abs * floor_abs);
  if (!(a2 > thr2) || fabs(apq) < 1e-300) {
    c = 1.0;
    s = 0.0;
    return false;
  }
  const double tau = (aqq - app) * 0.5 * frcp(apq);
  double t;
  if (fabs(tau) > 1e100) {
    t = 0.5 * frcp(tau);
  } else {
    const double h = fma(tau, tau, 1.0);
    const double root = h * frsq(h);  // sqrt(1 + tau^2)
    t = frcp(fabs(tau) + root);
    if (tau < 0.0) t = -t;
  }
  c = frsq(fma(t, t, 1.0));
  s = t * c;
  return true;
}

// Branch-free rotation for the subproblem rounds, same test as jacobi_rot.
// Only the rotation's exact orthogonality matters for the accuracy of the
// eigenvectors; its angle only has to annihilate a_pq well enough for the
// sweeps to converge.  So tau = (a_qq - a_pp) / (2 a_pq) is formed in float64
// with the hardware reciprocal (relative error ~2^-24, below float32 rounding),
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)) in float32 (relative error ~1e-7:
// the rotated a_pq drops by that factor, and later sweeps remove the rest),
// and c = 1/sqrt(1 + t^2), s = t c in float64 from that t, which keeps
// c^2 + s^2 = 1 to float64 rounding.  No branches, so the two rotations a
// thread needs are computed interleaved.
__device__ __forceinline__ bool jacobi_rot_bf(double app, double aqq, double apq, double floor_abs, double& c,
                                              double& s) {
  const double thr2 = fmax(4.930380657631324e-32 * fabs(app * aqq), floor_abs * floor_abs);
  const bool did = (apq * apq > thr2) && !(fabs(apq) < 1e-300);
  // hardware reciprocal alone (relative error ~2^-24, measured): tau is only
  // needed to float32 accuracy
  const double tau = (aqq - app) * 0.5 * __builtin_amdgcn_rcp(did ? apq : 1.0);
  const float tf = (float)tau;  // |tau| beyond float range: t rounds to 0 (angle < 1e-38)
  const float at = fabsf(tf);
  const float h = fmaf(at, at, 1.0f);
  const float t_small = __builtin_amdgcn_rcpf(at + h * __builtin_amdgcn_rsqf(h));
  const float t_big = 0.5f * __builtin_amdgcn_rcpf(at);  // |tau| > 1e15: t = 1 / (2 |tau|)
  const float t = at > 1e15f ? t_big : t_small;
  const double td = (double)(tf < 0.0f ? -t : t);
  const double cc = frsq(fma(td, td, 1.0));
  c = did ? cc : 1.0;
  s = did ? td * cc : 0.0;
  return did;
}

// Block two-sided Jacobi.  The m x m matrix (m = nblk * JB, nblk even) is cut
// into JB x JB blocks; a round pairs the blocks by the round-robin schedule.
// Phase 1 (one workgroup per block pair (P, Q)): form the JS x JS subproblem
// [A_PP A_PQ; A_QP A_QQ] in LDS, rotate its index pairs (all of them in the
// first round of a sweep, only the P-Q pairs in later rounds), keep the
// accumulated rotation J_k and write the rotated subproblem.  Phase 2 (one
// workgroup per tile): A <- J^T A J on the off-diagonal pair tiles
// (J_k^T A_kk' J_k') and V <- V J.
//
// One launch per round g runs phase 1 of round g and phase 2 of round g - 1
// side by side.  A^(g) (the matrix entering round g) lives in buffer g mod 3:
// phase 2 of round g - 1 writes its off-diagonal tiles from A^(g-1), phase 1
// of round g - 1 wrote its pair tiles the launch before, and phase 1 of
// round g, which cannot wait for phase 2, forms each block of its subproblem
// that phase 2 is still producing from A^(g-1) and the two rotations of round
// g - 1 itself (a 16 x 16 block of J^T T J).  Rotations are double buffered.
// A round whose index reaches conv_round (set when a sweep converges) does
// nothing, so the host may enqueue whole sweeps and poll the flag now and then.
struct JacArgs {
  double* A[3];     // m x m each: A^(g) in A[g % 3]
  double* V;        // m x m eigenvectors (columns), updated in place
  double* J[2];     // (nblk/2) x JS x JS rotations of round g in J[g % 2]
  int64_t m;
  int nblk;
  int inner_sweeps;
  int* flags;       // [max_sweeps] largest a_pq^2 / |a_pp a_qq| met by the sweep's subproblems, float bits (zeroed)
  int* conv;        // converged flag (zeroed)
  int* conv_round;  // first round not to run (INT_MAX-like until convergence)
  int* sweeps_out;
  double* floor;    // rotation floor (device scalar)
  float conv_r2;    // a sweep whose largest ratio^2 stays below this is the last
};

// Pair k and half h (0: first block, 1: second) of block X in round r.
__device__ __forceinline__ void locate_block(int X, int r, int nblk, int& k, int& h) {
  int pos = 0;
  if (X != 0) {
    int x = X - 1 - r;
    if (x < 0) x += nblk - 1;
    pos = 1 + x;
  }
  h = pos < nblk / 2 ? 0 : 1;
  k = h ? nblk - 1 - pos : pos;
}

__device__ __forceinline__ int64_t pair_index(int nblk, int k, int64_t r, int t) {
  const int blk = (t < JB) ? rr_index(k, (int)r, nblk) : rr_index(nblk - 1 - k, (int)r, nblk);
  return (int64_t)blk * JB + (t & (JB - 1));
}

typedef double jd4 __attribute__((ext_vector_type(4)));

// out(JS x JS) = opX(X) * Y on MFMA f64: 4 waves, wave w computes the 16 x 16
// quadrant (w/2, w%2).  TRANS_X: use X^T (X[p][i]) instead of X (X[i][p]).
// Accumulator element q of lane l is out[wm*16 + 4q + l/16][wn*16 + l%16].
static_assert(JS == 32, "quadrant layout assumes 32 x 32 subproblems");
template <bool TRANS_X>
__device__ __forceinline__ jd4 mmjs(const double (*X)[JS + 1], const double (*Y)[JS + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  jd4 acc = jd4{0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < JS; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    const int r = wm * 16 + (lane & 15), c = wn * 16 + (lane & 15);
    const double av = TRANS_X ? X[kk][r] : X[r][kk];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Y[kk][c], acc, 0, 0, 0);
  }
  return acc;
}

template <typename F>
__device__ __forceinline__ void mmjs_store(const jd4 acc, F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) f(wm * 16 + 4 * q + (lane >> 4), wn * 16 + (lane & 15), acc[q]);
}

// floor = 1e-14 * max diagonal entry: the tile updates leave off-diagonal
// rounding noise of a few eps ||A||; rotations below the floor move the
// eigenvalues by less than it, so converged sweeps stop.
__global__ void jac_floor(const double* __restrict__ A, int64_t m, double* __restrict__ floor) {
  __shared__ double red[256];
  double dm = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) dm = fmax(dm, A[i * m + i]);
  red[threadIdx.x] = dm;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) floor[0] = 1e-14 * red[0];
}

// Round-robin partner of position pos in inner round ir of a JS-index sweep
// (small-int form of rr_index for the subproblem).
__device__ __forceinline__ int rr_js(int pos, int ir) {
  if (pos == 0) return 0;
  const int x = pos - 1 + ir;
  return 1 + (x >= JS - 1 ? x - (JS - 1) : x);
}

// Inner rounds of one subproblem (see phase1_task): thread (k1, k2) updates the
// 2 x 2 block (rows of pair k1, columns of pair k2) of S = Sb[cur] into
// Sb[cur ^ 1] and its J entries, one barrier per round.  CROSS: round ir
// pairs i with JB + (i + ir) mod JB; else the round-robin over JS indices.
// Each lane computes the rotation of its column pair k2 = lane mod 16 (so
// lanes 0..15 of every wave hold all 16 rotations) and takes its row pair's
// rotation from lane k1 of its own wave: one rotation per thread instead of
// two, and no barrier for the exchange.
template <bool CROSS>
__device__ __forceinline__ void jac_inner(double (*Sb)[JS][JSS], double (*Jm)[JSS], int k1, int k2,
                                          int nround, double floor_abs, int& cur, bool& any_local,
                                          float& r2loc) {
  for (int ir = 0; ir < nround; ++ir) {
    double(*Si)[JSS] = Sb[cur];
    double(*So)[JSS] = Sb[cur ^ 1];
    int p1, q1, p2, q2;
    if (CROSS) {
      p1 = k1;
      q1 = JB + ((k1 + ir) & (JB - 1));
      p2 = k2;
      q2 = JB + ((k2 + ir) & (JB - 1));
    } else {
      p1 = rr_js(k1, ir);
      q1 = rr_js(JS - 1 - k1, ir);
      p2 = rr_js(k2, ir);
      q2 = rr_js(JS - 1 - k2, ir);
    }
    // every LDS read of the round first: the entries of this lane's
    // rotation, the 2 x 2 block and this thread's J entries
    const double r2pp = Si[p2][p2], r2qq = Si[q2][q2], r2pq = Si[p2][q2];
    const double app = Si[p1][p2], apq = Si[p1][q2], aqp = Si[q1][p2], aqq = Si[q1][q2];
    double jp[2], jq[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      jp[h] = Jm[k1 + h * JH][p2];
      jq[h] = Jm[k1 + h * JH][q2];
    }
    double c2, s2;
    const bool d2 = jacobi_rot_bf(r2pp, r2qq, r2pq, floor_abs, c2, s2);
    // row rotation from lane k1 (k1 < 16) of this wave: bit-identical to
    // the one every other thread of pair k1 uses
    const double c1 = __shfl(c2, k1, 64), s1 = __shfl(s2, k1, 64);
    any_local |= d2;
    if (k1 == 0 && d2) {  // each pair's ratio once: the threads of row pair 0
      const float r2 = (float)(r2pq * r2pq) * __builtin_amdgcn_rcpf(fmaxf((float)fabs(r2pp * r2qq), 1e-30f));
      r2loc = fmaxf(r2loc, fminf(r2, 1e30f));
    }
    // S <- R^T S R on the 2 x 2 block (on the diagonal blocks the rotated
    // a_pq is kept as computed, not set to zero: the float32 tangent leaves a
    // small remainder that later rounds remove, and S must stay J^T A J)
    const double bpp = c1 * app - s1 * aqp, bpq = c1 * apq - s1 * aqq;
    const double bqp = s1 * app + c1 * aqp, bqq = s1 * apq + c1 * aqq;
    So[p1][p2] = c2 * bpp - s2 * bpq;
    So[p1][q2] = s2 * bpp + c2 * bpq;
    So[q1][p2] = c2 * bqp - s2 * bqq;
    So[q1][q2] = s2 * bqp + c2 * bqq;
    // Jm <- Jm R: rows k1 and k1 + 16, columns of pair k2 (only this thread
    // touches them in this round; the identity rotation leaves them as they are)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Jm[k1 + h * JH][p2] = c2 * jp[h] - s2 * jq[h];
      Jm[k1 + h * JH][q2] = s2 * jp[h] + c2 * jq[h];
    }
    __syncthreads();
    cur ^= 1;
  }
}

// One block pair per workgroup: solve its JS x JS subproblem (inner cyclic
// sweeps in LDS) and store the accumulated rotation J and the rotated block.
// Thread (k1, k2) = (t / 16, t % 16) owns the 2 x 2 block (rows of rotation
// pair k1, columns of pair k2) of S and rows {k1, k1 + 16} x pair k2 of J.
// It computes the two rotations it needs itself (every thread that needs
// pair k derives it from the same entries, so they agree), and S is double
// buffered, so an inner round costs one barrier.
__device__ void phase1_task(const JacArgs& a, int64_t g, int k) {
  const int nb = a.nblk, R = nb - 1;
  const int r = (int)(g % R), sweep = (int)(g / R);
  const double* __restrict__ Ain = a.A[g % 3];         // A^(g): pair tiles of round g - 1
  const double* __restrict__ Aold = a.A[(g + 2) % 3];  // A^(g-1)
  double* __restrict__ Aout = a.A[(g + 1) % 3];        // A^(g+1): pair tiles of this round
  const double* __restrict__ Jold = a.J[(g + 1) % 2];  // rotations of round g - 1
  double* __restrict__ Jg = a.J[g % 2];
  __shared__ double Sb[2][JS][JSS];
  __shared__ double Jm[JS][JSS];
  __shared__ int64_t gi[JS];
  __shared__ int rotated, any_s;
  __shared__ unsigned maxr;  // float bits of the largest ratio^2 on entry (non-negative: int order)
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t m = a.m;
  double floor_abs;
  {
    // wave w forms block (w / 2, w % 2) of the subproblem: read from A^(g)
    // when its two blocks were one pair of round g - 1 (or g == 0), else as
    // J_kX^T T J_kY restricted to the two halves, T the tile of A^(g-1) and
    // J of round g - 1.  Lane l holds entries (4 q + l / 16, l % 16), the
    // f64 MFMA result layout.  The loads, the floor and the round limit are
    // issued together (in bounds whatever the limit says).
    const int P = rr_index(k, r, nb), Q = rr_index(nb - 1 - k, r, nb);
    const int bx = wave >> 1, by = wave & 1;
    const int X = bx ? Q : P, Y = by ? Q : P;
    floor_abs = *a.floor;
    const int cr = *a.conv_round;
    int kX = 0, hX = 0, kY = 0, hY = 0;
    const int rp = g > 0 ? (int)((g - 1) % R) : 0;
    bool direct = g == 0;
    if (!direct) {
      locate_block(X, rp, nb, kX, hX);
      locate_block(Y, rp, nb, kY, hY);
      direct = kX == kY;
    }
    double blk[4];
    if (direct) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        blk[q] = Ain[((int64_t)X * JB + 4 * q + (lane >> 4)) * m + (int64_t)Y * JB + (lane & 15)];
    } else {
      double ta[2][JS / 4], jy[JS / 4], jx[JS / 4];
#pragma unroll
      for (int ks = 0; ks < JS / 4; ++ks) {
        const int kk = 4 * ks + (lane >> 4);
        const int64_t col = pair_index(nb, kY, rp, kk);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) ta[rt][ks] = Aold[pair_index(nb, kX, rp, rt * 16 + (lane & 15)) * m + col];
        jy[ks] = Jold[(int64_t)kY * JS * JS + kk * JS + hY * JB + (lane & 15)];
        jx[ks] = Jold[(int64_t)kX * JS * JS + kk * JS + hX * JB + (lane & 15)];
      }
      // W = T J_kY[:, half hY] (32 x 16, two row tiles), then J_kX[:, half hX]^T W;
      // W's result registers are the second product's B operand as they stand
      jd4 w0 = jd4{0, 0, 0, 0}, w1 = jd4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < JS / 4; ++ks) {
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[0][ks], jy[ks], w0, 0, 0, 0);
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[1][ks], jy[ks], w1, 0, 0, 0);
      }
      jd4 o = jd4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < JS / 4; ++ks) {
        const double bw = ks < 4 ? w0[ks & 3] : w1[ks & 3];
        o = __builtin_amdgcn_mfma_f64_16x16x4f64(jx[ks], bw, o, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) blk[q] = o[q];
    }
    if (g >= cr) return;
    if (t < JS) gi[t] = pair_index(nb, k, r, t);
    if (t == 0) {
      rotated = 0;
      maxr = 0u;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Sb[0][bx * JB + 4 * q + (lane >> 4)][by * JB + (lane & 15)] = blk[q];
#pragma unroll
    for (int u = 0; u < JS * JS / 256; ++u) {
      const int e = t + 256 * u, i = e / JS, j = e % JS;
      Jm[i][j] = (i == j) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const int k1 = t >> 4, k2 = t & 15;
  // Inner ordering.  The first round of a sweep runs a full round-robin sweep
  // over the JS indices of each pair, which also covers the pairs inside
  // every block (each block is in exactly one pair of that round).  Later
  // rounds only pair an index of P with one of Q: JB inner rounds, round ir
  // pairing P's i with Q's (i + ir) mod JB, so every pair of indices of the
  // matrix is still rotated once per sweep, with half the inner rounds.
  // Every pair's ratio a_pq^2 / |a_pp a_qq| is taken when it is rotated (by
  // the threads with k2 == 0, which own each row rotation once), so the
  // sweep's maximum covers every pair once.
  const bool cross = r > 0 && a.inner_sweeps == 1;
  int cur = 0;
  float r2loc = 0.0f;
  if (a.inner_sweeps == 1) {
    // one inner sweep: no early exit to decide, so no barrier around it
    // (every writer of `rotated` stores 1; the barrier below publishes it)
    bool any_local = false;
    if (cross)
      jac_inner<true>(Sb, Jm, k1, k2, JB, floor_abs, cur, any_local, r2loc);
    else
      jac_inner<false>(Sb, Jm, k1, k2, JS - 1, floor_abs, cur, any_local, r2loc);
    if (any_local) rotated = 1;
  } else {
    for (int isw = 0; isw < a.inner_sweeps; ++isw) {
      if (t == 0) any_s = 0;
      __syncthreads();
      bool any_local = false;
      jac_inner<false>(Sb, Jm, k1, k2, JS - 1, floor_abs, cur, any_local, r2loc);
      if (any_local) any_s = 1;
      __syncthreads();
      if (any_s) rotated = 1;
      __syncthreads();
      if (!any_s) break;
      __syncthreads();
    }
  }
  {  // wave maximum of the rotated ratios first: one LDS atomic per wave
    for (int off = 32; off > 0; off >>= 1) r2loc = fmaxf(r2loc, __shfl_xor(r2loc, off));
    if ((t & 63) == 0 && r2loc > 0.0f) atomicMax(&maxr, __float_as_uint(r2loc));
  }
  __syncthreads();
  // the sweep's flag first, so its latency overlaps the stores below
  if (t == 0 && rotated) atomicMax(reinterpret_cast<unsigned*>(a.flags) + sweep, maxr > 1u ? maxr : 1u);
  #pragma unroll
  for (int e = t; e < JS * JS; e += 256) {
    Jg[(int64_t)k * JS * JS + e] = Jm[e / JS][e % JS];
    Aout[gi[e / JS] * m + gi[e % JS]] = Sb[cur][e / JS][e % JS];
  }
}

// Phase 2 of round g - 1: A^(g) off-diagonal pair tiles from A^(g-1); V <- V J.
__device__ void phase2_task(const JacArgs& a, int64_t g, int64_t task) {
  const int r = (int)((g - 1) % (a.nblk - 1));
  const double* __restrict__ Ag = a.A[(g + 2) % 3];
  double* __restrict__ An = a.A[g % 3];
  double* __restrict__ Vg = a.V;
  const double* __restrict__ Jg = a.J[(g + 1) % 2];
  __shared__ double S[JS][JS + 1];
  __shared__ double Jm[JS][JS + 1];
  __shared__ int64_t gi[JS], gj[JS];
  const int t = threadIdx.x;
  const int64_t m = a.m;
  const int nblk = a.nblk, npair = nblk / 2;
  const int64_t ntile_a = (int64_t)npair * npair;
  jd4 acc;
  if (task < ntile_a) {
    const int k1 = (int)(task / npair), k2 = (int)(task % npair);
    if (k1 == k2) return;  // written by phase 1
    // the tile, both rotations and the converged flag in one round of loads
    double v[JS * JS / 256], w[JS * JS / 256], w2[JS * JS / 256];
#pragma unroll
    for (int u = 0; u < JS * JS / 256; ++u) {
      const int e = t + 256 * u;
      v[u] = Ag[pair_index(nblk, k1, r, e / JS) * m + pair_index(nblk, k2, r, e % JS)];
      w[u] = Jg[(int64_t)k1 * JS * JS + e];
      w2[u] = Jg[(int64_t)k2 * JS * JS + e];
    }
    if (g - 1 >= *a.conv_round) return;
    if (t < JS) {
      gi[t] = pair_index(nblk, k1, r, t);
      gj[t] = pair_index(nblk, k2, r, t);
    }
#pragma unroll
    for (int u = 0; u < JS * JS / 256; ++u) {
      const int e = t + 256 * u;
      S[e / JS][e % JS] = v[u];
      Jm[e / JS][e % JS] = w[u];
    }
    __syncthreads();
    acc = mmjs<true>(Jm, S);  // T = J_k1^T S
    __syncthreads();
    mmjs_store(acc, [&](int i, int j, double v) { S[i][j] = v; });
#pragma unroll
    for (int u = 0; u < JS * JS / 256; ++u) Jm[(t + 256 * u) / JS][(t + 256 * u) % JS] = w2[u];
    __syncthreads();
    acc = mmjs<false>(S, Jm);  // T J_k2
    mmjs_store(acc, [&](int i, int j, double v) { An[gi[i] * m + gj[j]] = v; });
  } else {
    const int64_t vt = task - ntile_a;
    const int64_t rb = vt / npair;
    const int k = (int)(vt % npair);
    {
      double v[JS * JS / 256], w[JS * JS / 256];
#pragma unroll
      for (int u = 0; u < JS * JS / 256; ++u) {
        const int e = t + 256 * u;
        v[u] = Vg[(rb * JS + e / JS) * m + pair_index(nblk, k, r, e % JS)];
        w[u] = Jg[(int64_t)k * JS * JS + e];
      }
      if (g - 1 >= *a.conv_round) return;
      if (t < JS) gj[t] = pair_index(nblk, k, r, t);
#pragma unroll
      for (int u = 0; u < JS * JS / 256; ++u) {
        const int e = t + 256 * u;
        S[e / JS][e % JS] = v[u];
        Jm[e / JS][e % JS] = w[u];
      }
    }
    __syncthreads();
    acc = mmjs<false>(S, Jm);
    mmjs_store(acc, [&](int i, int j, double v) { Vg[(rb * JS + i) * m + gj[j]] = v; });
  }
}

// Converged when a sweep rotated nothing, or when every off-diagonal entry its
// subproblems met had |a_pq| <= c sqrt(|a_pp a_qq|), c^2 = conv_r2.  In the
// second case the sweep's own rotations leave each entry they annihilate at
// most at the float32-tangent remainder (1e-7 of its ratio) and mix in
// products of two such ratios from rotations sharing an index, so the matrix
// it leaves has ratios of about max(c^2, 1e-7 c): with c = 1e-9 about 1e-16,
// the level a further, confirming sweep would reach; with c = 1e-4 about 1e-8,
// below the rounding of a float32 U.  These ratios set the orthogonality of
// U = B W S^{-1/2}.
// host_conv (host memory visible to the device, may be null) receives the
// flag for the host's sweep loop in [0] and then the sequence tag in [1].
__global__ void jac_end_sweep(JacArgs a, int sweep, int* host_conv, int seq) {
  if (!*a.conv) {
    a.sweeps_out[0] = sweep + 1;
    const unsigned r2 = static_cast<unsigned>(a.flags[sweep]);
    if (r2 == 0u || r2 < __float_as_uint(a.conv_r2)) {
      a.conv[0] = 1;
      a.conv_round[0] = (sweep + 1) * (a.nblk - 1);
    }
  }
  if (host_conv) {
    host_conv[0] = a.conv[0];
    host_conv[2] = a.flags[sweep];  // the sweep's largest ratio^2 (float bits)
    __threadfence_system();
    ((volatile int*)host_conv)[1] = seq;
  }
}

// Round g: blocks [0, nblk/2) run phase 1 of round g (when with_phase1), the
// rest phase 2 of round g - 1 (when g > 0).
__global__ __launch_bounds__(256) void jac_round(JacArgs a, int64_t g, int with_phase1) {
  int64_t b = blockIdx.x;
  if (with_phase1) {
    if (b < a.nblk / 2) {
      phase1_task(a, g, (int)b);
      return;
    }
    b -= a.nblk / 2;
  }
  phase2_task(a, g, b);
}

// Diagonal of the final matrix A^(ge), ge = rounds run (all launched rounds
// up to the converged one).
__global__ void jac_evals(JacArgs a, int64_t glaunched, double* __restrict__ ev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cr = *a.conv_round;
  const int64_t ge = cr < glaunched ? cr : glaunched;
  const double* A = a.A[ge % 3];
  if (i < a.m) ev[i] = A[i * a.m + i];
}

// A = (G + G^T)/2 padded to m x m (padding: isolated eigenvalue -1), V = I.
__global__ void jacobi_init(const double* __restrict__ G, int64_t l, int64_t m,
                            double* __restrict__ A0, double* __restrict__ V) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx / m, j = idx % m;
  double v;
  if (i < l && j < l) v = 0.5 * (G[i * l + j] + G[j * l + i]);
  else v = (i == j) ? -1.0 : 0.0;
  A0[idx] = v;
  V[idx] = (i == j) ? 1.0 : 0.0;
}

// Sort eigenvalues descending (rank by counting; ties by index) and build
//   T[:, rank(i)] = V[:, i] / sqrt(s_i),   lam[rank(i)] = max(0, s_i - nu).
// Rank of eigenvalue i in descending order (ties by index), lam, sig2 and the
// column scale 1/sqrt(s_i); one thread per eigenvalue.
__global__ void eig_rank(const double* __restrict__ ev, int64_t l, const double* __restrict__ nu,
                         int* __restrict__ rank_out, double* __restrict__ inv_out, double* __restrict__ lam,
                         double* __restrict__ sig2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double si = ev[i];
  int64_t rank = 0;
  for (int64_t j = 0; j < l; ++j) {
    const double sj = ev[j];
    rank += (sj > si) || (sj == si && j < i);
  }
  rank_out[i] = (int)rank;
  inv_out[i] = (si > 0.0) ? 1.0 / sqrt(si) : 0.0;
  const double sh = nu ? nu[0] : 0.0;
  lam[rank] = fmax(0.0, si - sh);
  if (sig2) sig2[rank] = si;
}

// T[r][rank_i] = V[r][i] / sqrt(s_i): the eigenvectors in descending order,
// scaled; one thread per entry.
__global__ void eig_permute(const double* __restrict__ V, int64_t l, int64_t m, const int* __restrict__ rank,
                            const double* __restrict__ inv, double* __restrict__ T) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int64_t r = idx / l, i = idx % l;
  T[r * l + rank[i]] = V[r * m + i] * inv[i];
}

}  // namespace

nys_status frob_shift(const double* Y, int64_t count, double* part, double* nu, double u_rel, hipStream_t s) {
  const int nb = 1024;
  hipLaunchKernelGGL(sumsq_partial, dim3(nb), dim3(256), 0, s, Y, count, part);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(finalize_nu, dim3(1), dim3(256), 0, s, part, nb, u_rel, nu);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

size_t frob_partials() { return 1024; }

nys_status add_shift(double* Y, const double* Om, int64_t count, const double* nu, double factor,
                     hipStream_t s) {
  hipLaunchKernelGGL(axpy_nu, dim3(2048), dim3(256), 0, s, Y, Om, count, nu, factor);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

nys_status scale_device_scalar(double* x, double factor, hipStream_t s) {
  hipLaunchKernelGGL(scale_scalar, dim3(1), dim3(1), 0, s, x, factor);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

size_t chol_ws_doubles(int64_t n) { return (size_t)(cdiv(n, NB) * NB * NB); }

nys_status cholesky(const double* M, int64_t n, double* L, double* Dinv, int* info, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_lower, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s, M, n, L);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemsetAsync(info, 0, sizeof(int), s));
  CholArgs a{L, n, Dinv, info};
  const int nblk = (int)cdiv(n, NB);
  hipLaunchKernelGGL(chol_diag, dim3(1), dim3(64), 0, s, a, 0);
  for (int kb = 0; kb + 1 < nblk; ++kb) {
    const int rem = nblk - kb - 1;
    hipLaunchKernelGGL(chol_step, dim3((unsigned)(rem * (rem + 1) / 2)), dim3(256), 0, s, a, kb);
  }
  if (nblk > 1) hipLaunchKernelGGL(chol_panels, dim3((unsigned)(nblk * (nblk - 1) / 2)), dim3(256), 0, s, a);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

nys_status tri_inverse(const double* L, int64_t n, const double* Dinv, double* X, hipStream_t s) {
  const unsigned ne = (unsigned)cdiv(n * n, 256);
  hipLaunchKernelGGL(trinv_init, dim3(ne), dim3(256), 0, s, n, Dinv, X);
  NYS_CHECK_LAUNCH();
  for (int64_t bs = NB; bs < n; bs *= 2) {
    const int64_t tb = bs / NB;
    dim3 grid((unsigned)(tb * tb), (unsigned)cdiv(n, 2 * bs));
    hipLaunchKernelGGL(trinv_level, grid, dim3(256), 0, s, L, n, X, bs, 0);
    hipLaunchKernelGGL(trinv_level, grid, dim3(256), 0, s, L, n, X, bs, 1);
    NYS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(trinv_clear_upper, dim3(ne), dim3(256), 0, s, n, X);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// one inner sweep per round for large problems (the outer sweeps refine the
// pairs again); small problems are a single block pair, solved to convergence
int inner_sweeps_for(int64_t l) { return l <= JS ? 40 : 1; }

int jac_nblk(int64_t l) {
  int nb = (int)cdiv(l, JB);
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  return nb;
}

size_t eig_ws_doubles(int64_t l) {
  const int64_t nb = jac_nblk(l);
  const int64_t m = nb * JB;
  return (size_t)(4 * m * m + m + 2 * (nb / 2) * JS * JS + 2 * m + 8);
}

int* pinned_flags() {
  static thread_local int* p = nullptr;
  static thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void* q = nullptr;
    if (hipHostMalloc(&q, 256, hipHostMallocDefault) == hipSuccess) p = static_cast<int*>(q);
  }
  return p;
}

nys_status sym_eig(const double* G, int64_t l, double* work, int* flags, int max_sweeps,
                   int* sweeps_out, int* conv, double* T, double* lam, double* sig2, const double* nu,
                   hipStream_t s, double conv_ratio) {
  const int nb = jac_nblk(l);
  const int64_t m = (int64_t)nb * JB;
  double* A0 = work;
  double* V = work + 3 * m * m;
  double* ev = work + 4 * m * m;
  double* J0 = ev + m;
  double* J1 = J0 + (int64_t)(nb / 2) * JS * JS;
  double* floor = J1 + (int64_t)(nb / 2) * JS * JS;
  int* conv_round = reinterpret_cast<int*>(floor + 1);
  hipLaunchKernelGGL(jacobi_init, dim3((unsigned)cdiv(m * m, 256)), dim3(256), 0, s, G, l, m, A0, V);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemsetAsync(flags, 0, sizeof(int) * max_sweeps, s));
  NYS_HIP(hipMemsetAsync(conv, 0, sizeof(int), s));
  NYS_HIP(hipMemsetAsync(conv_round, 0x7f, sizeof(int), s));  // 0x7f7f7f7f: no limit yet
  NYS_HIP(hipMemsetAsync(sweeps_out, 0, sizeof(int), s));
  hipLaunchKernelGGL(jac_floor, dim3(1), dim3(256), 0, s, A0, m, floor);
  NYS_CHECK_LAUNCH();
  JacArgs a{{A0, A0 + m * m, A0 + 2 * m * m}, V, {J0, J1}, m, nb, inner_sweeps_for(l), flags, conv,
            conv_round, sweeps_out, floor, (float)(conv_ratio * conv_ratio)};
  const int npair = nb / 2;
  const int64_t tasks = (int64_t)npair * npair + (m / JS) * npair;
  int64_t g = 0;
  // Convergence is read one sweep behind: the flag of sweep s - 1 (written to
  // pinned host memory with a sequence tag by its end-of-sweep kernel) is
  // awaited while sweep s runs, so the GPU never idles on the poll and at
  // most one sweep of early-returning launches follows convergence.  Without
  // pinned memory the flag is copied and the stream synchronised every third
  // sweep.
  int* hpin = pinned_flags();  // [0] converged flag, [1] sequence tag, [2] sweep ratio^2
  int seqs[2] = {0, 0};
  int last_seq = 0;  // tag of the last end-of-sweep kernel enqueued
  nys_status st = NYS_OK;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int64_t r = 0; r < nb - 1; ++r, ++g)
      hipLaunchKernelGGL(jac_round, dim3((unsigned)(npair + (g > 0 ? tasks : 0))), dim3(256), 0, s, a, g, 1);
    seqs[sweep & 1] = hpin ? next_pinned_seq() : 0;
    last_seq = seqs[sweep & 1];
    hipLaunchKernelGGL(jac_end_sweep, dim3(1), dim3(1), 0, s, a, sweep, hpin, seqs[sweep & 1]);
    if (hipGetLastError() != hipSuccess) {
      set_error("sym_eig: kernel launch failed");
      st = NYS_ERR_DEVICE;
      break;
    }
    if (hpin) {
      if (sweep >= 6) {
        // the tag slot holds the latest sweep's tag; sweep s - 1's or later
        // means sweep s - 1 has ended (tags increase within the call)
        if (!wait_pinned(hpin + 1, seqs[(sweep - 1) & 1], s, seqs[sweep & 1])) {
          st = NYS_ERR_DEVICE;
          break;
        }
        if (*(volatile int*)hpin) break;
        // Near the end the sweep ratios fall quadratically: when sweep s - 1
        // ended within a factor 5 of the stopping ratio, sweep s (running
        // now) is most likely the last, so its flag is awaited before another
        // sweep is enqueued.  That saves the sweep of early-returning launches
        // that would follow convergence; a wrong guess costs one host round
        // trip of device idle time.
        const int tag = ((volatile int*)hpin)[1];
        float r2prev;
        const int bits = ((volatile int*)hpin)[2];
        std::memcpy(&r2prev, &bits, sizeof(float));
        if (tag != seqs[sweep & 1] && r2prev < 25.0f * a.conv_r2) {
          if (!wait_pinned(hpin + 1, seqs[sweep & 1], s, 0)) {
            st = NYS_ERR_DEVICE;
            break;
          }
          if (*(volatile int*)hpin) break;
        }
      }
    } else if (sweep >= 5 && (sweep % 3 == 2)) {
      int c = 0;
      NYS_HIP(hipMemcpyAsync(&c, conv, sizeof(int), hipMemcpyDeviceToHost, s));
      NYS_HIP(hipStreamSynchronize(s));
      if (c) break;
    }
  }
  if (st != NYS_OK) return st;
  // phase 2 of the last round that ran (a no-op if a later launch did it)
  hipLaunchKernelGGL(jac_round, dim3((unsigned)tasks), dim3(256), 0, s, a, g, 0);
  hipLaunchKernelGGL(jac_evals, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, s, a, g, ev);
  int* rk = reinterpret_cast<int*>(floor + 2);
  double* inv = floor + 2 + cdiv(m, 2);
  hipLaunchKernelGGL(eig_rank, dim3((unsigned)cdiv(l, 256)), dim3(256), 0, s, ev, l, nu, rk, inv, lam, sig2);
  hipLaunchKernelGGL(eig_permute, dim3((unsigned)cdiv(l * l, 256)), dim3(256), 0, s, V, l, m, rk, inv, T);
  NYS_CHECK_LAUNCH();
  // The last end-of-sweep kernel writes the pinned flags; it has run before
  // the call returns, so a later call that reuses them (on any stream) never
  // meets a late write.  The kernels above are already enqueued behind it.
  if (hpin && last_seq != 0 && !wait_pinned(hpin + 1, last_seq, s)) return NYS_ERR_DEVICE;
  return NYS_OK;
}

}  // namespace nys
