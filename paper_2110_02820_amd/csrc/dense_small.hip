// Small dense float64 linear algebra on the l x l core of the Nystrom
// factorisation (Section 2.2, algorithm "Randomized Nystrom Approximation",
// steps 4-9), all on the device:
//   * shift nu = eps(||Y||_F) and Y_nu = Y + nu Omega
//   * Cholesky factorisation (blocked, right-looking, cooperative launch)
//   * inverse of the lower-triangular factor (independent column-block chains)
//   * symmetric eigensolver: cyclic two-sided Jacobi with the round-robin
//     parallel ordering (every round rotates m/2 disjoint pairs), cooperative
//     launch with one grid barrier per round
//   * descending sort of the eigenvalues and the scaled eigenvector matrix
#include "dense_small.hpp"

namespace nys {

namespace {

constexpr int NB = 32;  // block size of the blocked Cholesky / inverse

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
__global__ void finalize_nu(const double* __restrict__ part, int np, double* __restrict__ nu) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s);
    int e = 0;
    frexp(nrm, &e);
    nu[0] = (nrm > 0.0) ? ldexp(1.0, e - 53) : 4.9406564584124654e-324;
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
  unsigned* bar;
  int* bar_err;
};

// Unblocked Cholesky + inverse of one NB x NB diagonal block in LDS.
__device__ void factor_diag_block(CholArgs a, int kb, double (*T)[NB + 1], double (*Ti)[NB + 1]) {
  const int64_t n = a.n;
  const int64_t base = (int64_t)kb * NB;
  const int nbk = (int)((n - base) < NB ? (n - base) : NB);
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    double v = 0.0;
    if (i < nbk && j < nbk && j <= i) v = a.L[(base + i) * n + base + j];
    else if (i == j) v = 1.0;  // padding outside the matrix: identity
    T[i][j] = v;
    Ti[i][j] = 0.0;
  }
  __syncthreads();
  __shared__ int bad;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < NB; ++k) {
    if (t == 0) {
      const double d = T[k][k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        if (k < nbk && atomicCAS(a.info, 0, (int)(base + k + 1)) == 0) {}
        T[k][k] = 1.0;
      } else {
        T[k][k] = sqrt(d);
      }
    }
    __syncthreads();
    const double dk = T[k][k];
    for (int i = k + 1 + t; i < NB; i += blockDim.x) T[i][k] /= dk;
    __syncthreads();
    for (int e = t; e < NB * NB; e += blockDim.x) {
      const int i = e / NB, j = e % NB;
      if (i > k && j > k && j <= i) T[i][j] -= T[i][k] * T[j][k];
    }
    __syncthreads();
  }
  // inverse by forward substitution, one column per thread
  if (t < NB) {
    const int j = t;
    for (int i = 0; i < NB; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= T[i][k] * Ti[k][j];
      Ti[i][j] = (i >= j) ? s / T[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    if (i < nbk && j < nbk) a.L[(base + i) * n + base + j] = (j <= i) ? T[i][j] : 0.0;
    a.Dinv[(int64_t)kb * NB * NB + e] = Ti[i][j];
  }
  (void)bad;
}

__global__ __launch_bounds__(256) void chol_coop(CholArgs a) {
  __shared__ double T[NB][NB + 1];
  __shared__ double Ti[NB][NB + 1];
  __shared__ double Lb[NB][NB + 1];
  GridBarrier gb{a.bar, a.bar_err, gridDim.x, 0};
  const int64_t n = a.n;
  const int nblk = (int)cdiv(n, NB);
  const int t = threadIdx.x;
  for (int kb = 0; kb < nblk; ++kb) {
    if (blockIdx.x == 0) factor_diag_block(a, kb, T, Ti);
    gb.sync();
    if (*((volatile int*)a.info) != 0) break;
    // panel: L[ib,kb] = A[ib,kb] * Dinv_kb^T for ib > kb
    const double* Di = a.Dinv + (int64_t)kb * NB * NB;
    for (int ib = kb + 1 + blockIdx.x; ib < nblk; ib += gridDim.x) {
      const int64_t r0 = (int64_t)ib * NB, c0 = (int64_t)kb * NB;
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        Lb[i][j] = (r0 + i < n && c0 + j < n) ? a.L[(r0 + i) * n + c0 + j] : 0.0;
        Ti[i][j] = Di[e];
      }
      __syncthreads();
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        double s = 0.0;
        for (int k = 0; k <= j; ++k) s += Lb[i][k] * Ti[j][k];
        T[i][j] = s;
      }
      __syncthreads();
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        if (r0 + i < n && c0 + j < n) a.L[(r0 + i) * n + c0 + j] = T[i][j];
      }
      __syncthreads();
    }
    gb.sync();
    // trailing update: A[ib,jb] -= L[ib,kb] L[jb,kb]^T for kb < jb <= ib
    const int rem = nblk - kb - 1;
    const int ntile = rem * (rem + 1) / 2;
    for (int tt = blockIdx.x; tt < ntile; tt += gridDim.x) {
      // tile index -> (ib, jb) with jb <= ib
      int ii = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
      while ((ii + 1) * (ii + 2) / 2 <= tt) ++ii;
      while (ii * (ii + 1) / 2 > tt) --ii;
      const int jj = tt - ii * (ii + 1) / 2;
      const int ib = kb + 1 + ii, jb = kb + 1 + jj;
      const int64_t c0 = (int64_t)kb * NB;
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, k = e % NB;
        const int64_t ri = (int64_t)ib * NB + i, rj = (int64_t)jb * NB + i;
        Lb[i][k] = (ri < n) ? a.L[ri * n + c0 + k] : 0.0;
        T[i][k] = (rj < n) ? a.L[rj * n + c0 + k] : 0.0;
      }
      __syncthreads();
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        const int64_t gi = (int64_t)ib * NB + i, gj = (int64_t)jb * NB + j;
        if (gi < n && gj < n && gj <= gi) {
          double s = 0.0;
#pragma unroll 8
          for (int k = 0; k < NB; ++k) s += Lb[i][k] * T[j][k];
          a.L[gi * n + gj] -= s;
        }
      }
      __syncthreads();
    }
    gb.sync();
  }
}

// ---------------------------------------------------------------- L^{-1}

// One workgroup per column block jb: X[jb][jb] = Dinv_jb and, for ib > jb,
// X[ib][jb] = -Dinv_ib * sum_{kb=jb}^{ib-1} L[ib][kb] X[kb][jb].
__global__ __launch_bounds__(256) void trinv_blocks(const double* __restrict__ L, int64_t n,
                                                    const double* __restrict__ Dinv,
                                                    double* __restrict__ X) {
  __shared__ double Acc[NB][NB + 1];
  __shared__ double Lt[NB][NB + 1];
  __shared__ double Xt[NB][NB + 1];
  const int nblk = (int)cdiv(n, NB);
  const int jb = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)jb * NB;
  // zero the strictly-upper column blocks of this column block
  for (int64_t r = t; r < c0; r += blockDim.x)
    for (int j = 0; j < NB && c0 + j < n; ++j) X[r * n + c0 + j] = 0.0;
  // diagonal block
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    if (c0 + i < n && c0 + j < n) X[(c0 + i) * n + c0 + j] = Dinv[(int64_t)jb * NB * NB + e];
  }
  __threadfence_block();
  __syncthreads();
  for (int ib = jb + 1; ib < nblk; ++ib) {
    const int64_t r0 = (int64_t)ib * NB;
    for (int e = t; e < NB * NB; e += blockDim.x) Acc[e / NB][e % NB] = 0.0;
    __syncthreads();
    for (int kb = jb; kb < ib; ++kb) {
      const int64_t k0 = (int64_t)kb * NB;
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        Lt[i][j] = (r0 + i < n && k0 + j < n) ? L[(r0 + i) * n + k0 + j] : 0.0;
        Xt[i][j] = (k0 + i < n && c0 + j < n) ? X[(k0 + i) * n + c0 + j] : 0.0;
      }
      __syncthreads();
      for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < NB; ++k) s += Lt[i][k] * Xt[k][j];
        Acc[i][j] += s;
      }
      __syncthreads();
    }
    const double* Di = Dinv + (int64_t)ib * NB * NB;
    for (int e = t; e < NB * NB; e += blockDim.x) {
      const int i = e / NB, j = e % NB;
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += Di[i * NB + k] * Acc[k][j];
      if (r0 + i < n && c0 + j < n) X[(r0 + i) * n + c0 + j] = -s;
    }
    __threadfence_block();
    __syncthreads();
  }
}

// ---------------------------------------------------------------- Jacobi

constexpr int JB = 32;       // Jacobi block size
constexpr int JS = 2 * JB;   // order of one block-pair subproblem

__device__ __forceinline__ int64_t rr_index(int64_t pos, int64_t r, int64_t m) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (m - 1));
}

// Rotation (c, s) with J_pp = c, J_pq = s, J_qp = -s, J_qq = c that zeroes
// entry (p, q) of J^T A J (symmetric 2x2 Schur decomposition).  Returns false
// (identity) when |a_pq| is negligible relative to sqrt(|a_pp a_qq|).
__device__ __forceinline__ bool jacobi_rot(double app, double aqq, double apq, double floor_abs,
                                           double& c, double& s) {
  const double thr = fmax(2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq)), floor_abs);
  if (!(fabs(apq) > thr) || fabs(apq) < 1e-300) {
    c = 1.0;
    s = 0.0;
    return false;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double tt = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                 : -1.0 / (-tau + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
  return true;
}

// Block two-sided Jacobi.  The m x m matrix (m = nblk * JB, nblk even) is cut
// into JB x JB blocks; a round pairs the blocks by the round-robin schedule.
// Phase 1: one workgroup per block pair (P, Q) loads the JS x JS subproblem
// [A_PP A_PQ; A_QP A_QQ] into LDS, runs cyclic Jacobi sweeps on it and keeps
// the accumulated rotation J_k.  Phase 2: every workgroup applies the
// rotations, A <- J^T A J (tiles pair k x pair k': J_k^T A_kk' J_k') and
// V <- V J.  Two grid barriers per round; nblk - 1 rounds per sweep.
struct JacArgs {
  double* A;       // m x m
  double* V;       // m x m eigenvectors (columns)
  double* J;       // (nblk/2) x JS x JS rotations of the current round
  int64_t m;
  int nblk;
  int max_sweeps;
  int inner_sweeps;
  int* flags;      // [max_sweeps] "a rotation happened" per sweep (zeroed)
  int* sweeps_out;
  double* evals;   // m: diagonal of the final matrix
  unsigned* bar;
  int* bar_err;
};

__device__ __forceinline__ int64_t pair_index(int nblk, int k, int64_t r, int t) {
  const int64_t blk = (t < JB) ? rr_index(k, r, nblk) : rr_index(nblk - 1 - k, r, nblk);
  return blk * JB + (t & (JB - 1));
}

typedef double jd4 __attribute__((ext_vector_type(4)));

// out(64x64) = opA(X) * Y on MFMA f64 (4 waves, each a 32x32 quadrant).
// TRANS_X: use X^T (X[p][i]) instead of X (X[i][p]).  Results are returned in
// the wave's accumulators; element q of lane l of tile (ti, tj) is
// out[wm*32 + ti*16 + 4q + l/16][wn*32 + tj*16 + l%16].
template <bool TRANS_X>
__device__ __forceinline__ void mm64(const double (*X)[JS + 1], const double (*Y)[JS + 1], jd4 acc[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = jd4{0, 0, 0, 0};
#pragma unroll 4
  for (int k0 = 0; k0 < JS; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    const int r0 = wm * 32 + (lane & 15), r1 = r0 + 16;
    const int c0 = wn * 32 + (lane & 15), c1 = c0 + 16;
    const double a0 = TRANS_X ? X[kk][r0] : X[r0][kk];
    const double a1 = TRANS_X ? X[kk][r1] : X[r1][kk];
    const double b0 = Y[kk][c0], b1 = Y[kk][c1];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

template <typename F>
__device__ __forceinline__ void mm64_store(const jd4 acc[2][2], F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        f(wm * 32 + i * 16 + 4 * q + (lane >> 4), wn * 32 + j * 16 + (lane & 15), acc[i][j][q]);
}

__global__ __launch_bounds__(256) void jacobi_block_coop(JacArgs a) {
  __shared__ double S[JS][JS + 1];
  __shared__ double Jm[JS][JS + 1];
  __shared__ double cs[JS / 2], sn[JS / 2];
  __shared__ int pp[JS / 2], qq[JS / 2];
  __shared__ int64_t gi[JS], gj[JS];
  __shared__ int rotated, any_s;
  GridBarrier gb{a.bar, a.bar_err, gridDim.x, 0};
  const int t = threadIdx.x;
  const int64_t m = a.m;
  const int nblk = a.nblk, npair = nblk / 2;
  // absolute floor of the rotation test: eps times the largest diagonal entry
  // of the input (rotations below it change eigenvalues by less than that)
  __shared__ double dmax_s;
  {
    double dm = 0.0;
    for (int64_t i = t; i < m; i += 256) dm = fmax(dm, a.A[i * m + i]);
    __shared__ double red[256];
    red[t] = dm;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (t < st) red[t] = fmax(red[t], red[t + st]);
      __syncthreads();
    }
    if (t == 0) dmax_s = red[0];
    __syncthreads();
  }
  const double floor_abs = 2.220446049250313e-16 * dmax_s;
  gb.sync();  // every workgroup has read the input diagonal before any rotation
  int sweep = 0;
  for (sweep = 0; sweep < a.max_sweeps; ++sweep) {
    for (int64_t r = 0; r < nblk - 1; ++r) {
      // ---- phase 1: block-pair subproblems in LDS
      for (int k = blockIdx.x; k < npair; k += gridDim.x) {
        if (t < JS) gi[t] = pair_index(nblk, k, r, t);
        if (t == 0) rotated = 0;
        __syncthreads();
        for (int e = t; e < JS * JS; e += 256) {
          const int i = e / JS, j = e % JS;
          S[i][j] = a.A[gi[i] * m + gi[j]];
          Jm[i][j] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int isw = 0; isw < a.inner_sweeps; ++isw) {
          if (t == 0) any_s = 0;
          __syncthreads();
          for (int ir = 0; ir < JS - 1; ++ir) {
            if (t < JS / 2) {
              const int p = (int)rr_index(t, ir, JS), q = (int)rr_index(JS - 1 - t, ir, JS);
              double c, sv;
              if (jacobi_rot(S[p][p], S[q][q], S[p][q], floor_abs, c, sv)) any_s = 1;
              cs[t] = c;
              sn[t] = sv;
              pp[t] = p;
              qq[t] = q;
            }
            __syncthreads();
            // S <- R^T S R on 2x2 blocks (rows pair k1, cols pair k2)
            for (int e = t; e < (JS / 2) * (JS / 2); e += 256) {
              const int k1 = e >> 5, k2 = e & 31;
              const double s1 = sn[k1], s2 = sn[k2];
              if (s1 == 0.0 && s2 == 0.0) continue;
              const int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
              const double c1 = cs[k1], c2 = cs[k2];
              const double app = S[p1][p2], apq = S[p1][q2], aqp = S[q1][p2], aqq = S[q1][q2];
              const double bpp = c1 * app - s1 * aqp, bpq = c1 * apq - s1 * aqq;
              const double bqp = s1 * app + c1 * aqp, bqq = s1 * apq + c1 * aqq;
              double npp = c2 * bpp - s2 * bpq, npq = s2 * bpp + c2 * bpq;
              double nqp = c2 * bqp - s2 * bqq, nqq = s2 * bqp + c2 * bqq;
              if (k1 == k2) {
                npq = 0.0;
                nqp = 0.0;
              }
              S[p1][p2] = npp;
              S[p1][q2] = npq;
              S[q1][p2] = nqp;
              S[q1][q2] = nqq;
            }
            // Jm <- Jm R (row i, pair kk)
            for (int e = t; e < JS * (JS / 2); e += 256) {
              const int i = e >> 5, kk = e & 31;
              const double sv = sn[kk];
              if (sv == 0.0) continue;
              const double c = cs[kk];
              const int p = pp[kk], q = qq[kk];
              const double vp = Jm[i][p], vq = Jm[i][q];
              Jm[i][p] = c * vp - sv * vq;
              Jm[i][q] = sv * vp + c * vq;
            }
            __syncthreads();
          }
          if (any_s) rotated = 1;
          __syncthreads();
          if (!any_s) break;
          __syncthreads();
        }
        for (int e = t; e < JS * JS; e += 256) {
          a.J[(int64_t)k * JS * JS + e] = Jm[e / JS][e % JS];
          a.A[gi[e / JS] * m + gi[e % JS]] = S[e / JS][e % JS];
        }
        if (t == 0 && rotated) a.flags[sweep] = 1;
        __syncthreads();
      }
      gb.sync();
      // ---- phase 2: A <- J^T A J on off-diagonal pair tiles, V <- V J (MFMA)
      const int ntile_a = npair * npair;
      const int64_t nrb = m / JS;
      const int64_t ntile_v = nrb * npair;
      for (int64_t task = blockIdx.x; task < ntile_a + ntile_v; task += gridDim.x) {
        jd4 acc[2][2];
        if (task < ntile_a) {
          const int k1 = (int)(task / npair), k2 = (int)(task % npair);
          if (k1 == k2) continue;  // written by phase 1
          if (t < JS) {
            gi[t] = pair_index(nblk, k1, r, t);
            gj[t] = pair_index(nblk, k2, r, t);
          }
          __syncthreads();
          for (int e = t; e < JS * JS; e += 256) {
            const int i = e / JS, j = e % JS;
            S[i][j] = a.A[gi[i] * m + gj[j]];
            Jm[i][j] = a.J[(int64_t)k1 * JS * JS + e];
          }
          __syncthreads();
          mm64<true>(Jm, S, acc);  // T = J_k1^T S
          __syncthreads();
          mm64_store(acc, [&](int i, int j, double v) { S[i][j] = v; });
          for (int e = t; e < JS * JS; e += 256) Jm[e / JS][e % JS] = a.J[(int64_t)k2 * JS * JS + e];
          __syncthreads();
          mm64<false>(S, Jm, acc);  // T J_k2
          mm64_store(acc, [&](int i, int j, double v) { a.A[gi[i] * m + gj[j]] = v; });
          __syncthreads();
        } else {
          const int64_t vt = task - ntile_a;
          const int64_t rb = vt / npair;
          const int k = (int)(vt % npair);
          if (t < JS) gj[t] = pair_index(nblk, k, r, t);
          __syncthreads();
          for (int e = t; e < JS * JS; e += 256) {
            const int i = e / JS, j = e % JS;
            S[i][j] = a.V[(rb * JS + i) * m + gj[j]];
            Jm[i][j] = a.J[(int64_t)k * JS * JS + e];
          }
          __syncthreads();
          mm64<false>(S, Jm, acc);
          mm64_store(acc, [&](int i, int j, double v) { a.V[(rb * JS + i) * m + gj[j]] = v; });
          __syncthreads();
        }
      }
      gb.sync();
    }
    if (*((volatile int*)&a.flags[sweep]) == 0) {
      ++sweep;
      break;
    }
  }
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + t;
  if (gtid == 0) a.sweeps_out[0] = sweep;
  for (int64_t i = gtid; i < m; i += (int64_t)gridDim.x * blockDim.x) a.evals[i] = a.A[i * m + i];
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
__global__ void eig_finalize(const double* __restrict__ ev, const double* __restrict__ V,
                             int64_t l, int64_t m, const double* __restrict__ nu,
                             double* __restrict__ T, double* __restrict__ lam,
                             double* __restrict__ sig2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double si = ev[i];
  int64_t rank = 0;
  for (int64_t j = 0; j < l; ++j) {
    const double sj = ev[j];
    rank += (sj > si) || (sj == si && j < i);
  }
  const double inv = (si > 0.0) ? 1.0 / sqrt(si) : 0.0;
  for (int64_t r = 0; r < l; ++r) T[r * l + rank] = V[r * m + i] * inv;
  const double sh = nu ? nu[0] : 0.0;
  lam[rank] = fmax(0.0, si - sh);
  if (sig2) sig2[rank] = si;
}

int coop_blocks(const void* fn, int threads, size_t shmem, int want) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, shmem) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int cap = per_cu * num_cus();
  return want < cap ? want : cap;
}

}  // namespace

nys_status frob_shift(const double* Y, int64_t count, double* part, double* nu, hipStream_t s) {
  const int nb = 1024;
  hipLaunchKernelGGL(sumsq_partial, dim3(nb), dim3(256), 0, s, Y, count, part);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(finalize_nu, dim3(1), dim3(256), 0, s, part, nb, nu);
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

nys_status cholesky(const double* M, int64_t n, double* L, double* Dinv, int* info, unsigned* bar,
                    int* bar_err, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_lower, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s, M, n, L);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemsetAsync(info, 0, sizeof(int), s));
  NYS_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned), s));
  NYS_HIP(hipMemsetAsync(bar_err, 0, sizeof(int), s));
  CholArgs a{L, n, Dinv, info, bar, bar_err};
  const int nblk = (int)cdiv(n, NB);
  const int want = nblk * (nblk + 1) / 2 > 1 ? nblk * (nblk + 1) / 2 : 1;
  const int g = coop_blocks((const void*)chol_coop, 256, 0, want < 512 ? want : 512);
  void* args[] = {&a};
  NYS_HIP(hipLaunchCooperativeKernel((const void*)chol_coop, dim3(g), dim3(256), args, 0, s));
  return NYS_OK;
}

nys_status tri_inverse(const double* L, int64_t n, const double* Dinv, double* X, hipStream_t s) {
  hipLaunchKernelGGL(trinv_blocks, dim3((unsigned)cdiv(n, NB)), dim3(256), 0, s, L, n, Dinv, X);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// one inner sweep per round for large problems (the outer sweeps refine the
// pairs again); small problems are a single block pair, solved to convergence
int inner_sweeps_for(int64_t l) { return l <= JS ? 30 : 1; }

int jac_nblk(int64_t l) {
  int nb = (int)cdiv(l, JB);
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  return nb;
}

size_t eig_ws_doubles(int64_t l) {
  const int64_t nb = jac_nblk(l);
  const int64_t m = nb * JB;
  return (size_t)(2 * m * m + m + (nb / 2) * JS * JS);
}

nys_status sym_eig(const double* G, int64_t l, double* work, int* flags, int max_sweeps,
                   int* sweeps_out, unsigned* bar, int* bar_err, double* T, double* lam,
                   double* sig2, const double* nu, hipStream_t s) {
  const int nb = jac_nblk(l);
  const int64_t m = (int64_t)nb * JB;
  double* A = work;
  double* V = work + m * m;
  double* ev = work + 2 * m * m;
  double* J = ev + m;
  hipLaunchKernelGGL(jacobi_init, dim3((unsigned)cdiv(m * m, 256)), dim3(256), 0, s, G, l, m, A, V);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemsetAsync(flags, 0, sizeof(int) * max_sweeps, s));
  NYS_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned), s));
  NYS_HIP(hipMemsetAsync(bar_err, 0, sizeof(int), s));
  JacArgs a{A, V, J, m, nb, max_sweeps, inner_sweeps_for(l), flags, sweeps_out, ev, bar, bar_err};
  const int64_t tasks = (int64_t)(nb / 2) * (nb / 2) + (m / JS) * (nb / 2);
  const int g = coop_blocks((const void*)jacobi_block_coop, 256, 0, (int)(tasks < 256 ? tasks : 256));
  void* args[] = {&a};
  NYS_HIP(hipLaunchCooperativeKernel((const void*)jacobi_block_coop, dim3(g), dim3(256), args, 0, s));
  hipLaunchKernelGGL(eig_finalize, dim3((unsigned)cdiv(l, 256)), dim3(256), 0, s, ev, V, l, m,
                     nu, T, lam, sig2);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

}  // namespace nys
