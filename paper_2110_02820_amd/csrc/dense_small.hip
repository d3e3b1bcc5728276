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

struct JacArgs {
  double* A0;      // m x m working copy (round parity 0)
  double* A1;      // m x m working copy (round parity 1)
  double* V;       // m x m eigenvectors (columns)
  int64_t m;       // even order (l or l+1)
  int max_sweeps;
  int* flags;      // [max_sweeps] "a rotation happened" per sweep (zeroed)
  int* sweeps_out; // sweeps executed
  double* evals;   // m: diagonal of the final matrix (the eigenvalues)
  unsigned* bar;
  int* bar_err;
};

__device__ __forceinline__ int64_t rr_index(int64_t pos, int64_t r, int64_t m) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (m - 1));
}

// Rotation (c, s) with J_pp = c, J_pq = s, J_qp = -s, J_qq = c that zeroes
// entry (p, q) of J^T A J (symmetric 2x2 Schur decomposition).
__device__ __forceinline__ bool jacobi_rot(double app, double aqq, double apq, double& c,
                                           double& s) {
  const double thr = 2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq));
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

__global__ __launch_bounds__(256) void jacobi_coop(JacArgs a) {
  extern __shared__ double rot[];  // [2 * (m/2)] : c then s
  GridBarrier gb{a.bar, a.bar_err, gridDim.x, 0};
  const int64_t m = a.m, half = m / 2;
  double* cs = rot;
  double* sn = rot + half;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  int64_t round = 0;
  int sweep = 0;
  for (sweep = 0; sweep < a.max_sweeps; ++sweep) {
    for (int64_t r = 0; r < m - 1; ++r, ++round) {
      const double* Ar = (round & 1) ? a.A1 : a.A0;
      double* Aw = (round & 1) ? a.A0 : a.A1;
      bool any = false;
      for (int64_t k = threadIdx.x; k < half; k += blockDim.x) {
        const int64_t p = rr_index(k, r, m), q = rr_index(m - 1 - k, r, m);
        double c, s;
        any |= jacobi_rot(Ar[p * m + p], Ar[q * m + q], Ar[p * m + q], c, s);
        cs[k] = c;
        sn[k] = s;
      }
      if (any && blockIdx.x == 0) a.flags[sweep] = 1;
      __syncthreads();
      // A blocks: rows pair k1, cols pair k2
      for (int64_t e = gtid; e < half * half; e += gsz) {
        const int64_t k1 = e / half, k2 = e % half;
        const int64_t p1 = rr_index(k1, r, m), q1 = rr_index(m - 1 - k1, r, m);
        const int64_t p2 = rr_index(k2, r, m), q2 = rr_index(m - 1 - k2, r, m);
        const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
        const double app = Ar[p1 * m + p2], apq = Ar[p1 * m + q2];
        const double aqp = Ar[q1 * m + p2], aqq = Ar[q1 * m + q2];
        // rows: row_p' = c row_p - s row_q ; row_q' = s row_p + c row_q
        const double bpp = c1 * app - s1 * aqp, bpq = c1 * apq - s1 * aqq;
        const double bqp = s1 * app + c1 * aqp, bqq = s1 * apq + c1 * aqq;
        // cols: col_p' = c col_p - s col_q ; col_q' = s col_p + c col_q
        double npp = c2 * bpp - s2 * bpq, npq = s2 * bpp + c2 * bpq;
        double nqp = c2 * bqp - s2 * bqq, nqq = s2 * bqp + c2 * bqq;
        if (k1 == k2 && sn[k1] != 0.0) { npq = 0.0; nqp = 0.0; }
        Aw[p1 * m + p2] = npp;
        Aw[p1 * m + q2] = npq;
        Aw[q1 * m + p2] = nqp;
        Aw[q1 * m + q2] = nqq;
      }
      // V <- V J (row i, pair k)
      for (int64_t e = gtid; e < m * half; e += gsz) {
        const int64_t i = e / half, k = e % half;
        const double s = sn[k];
        if (s == 0.0) continue;
        const double c = cs[k];
        const int64_t p = rr_index(k, r, m), q = rr_index(m - 1 - k, r, m);
        const double vp = a.V[i * m + p], vq = a.V[i * m + q];
        a.V[i * m + p] = c * vp - s * vq;
        a.V[i * m + q] = s * vp + c * vq;
      }
      gb.sync();
    }
    if (*((volatile int*)&a.flags[sweep]) == 0) {
      ++sweep;
      break;
    }
  }
  if (gtid == 0) a.sweeps_out[0] = sweep;
  // after `round` rounds the newest copy is A1 when round is odd
  const double* Afin = (round & 1) ? a.A1 : a.A0;
  for (int64_t i = gtid; i < m; i += gsz) a.evals[i] = Afin[i * m + i];
}

__global__ void jacobi_init(const double* __restrict__ G, int64_t l, int64_t m,
                            double* __restrict__ A0, double* __restrict__ V) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx / m, j = idx % m;
  double v;
  if (i < l && j < l) v = 0.5 * (G[i * l + j] + G[j * l + i]);
  else v = (i == j) ? -1.0 : 0.0;  // padding index: isolated eigenvalue -1
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

size_t eig_ws_doubles(int64_t l) {
  const int64_t m = l + (l & 1);
  return (size_t)(3 * m * m + m);
}

nys_status sym_eig(const double* G, int64_t l, double* work, int* flags, int max_sweeps,
                   int* sweeps_out, unsigned* bar, int* bar_err, double* T, double* lam,
                   double* sig2, const double* nu, hipStream_t s) {
  const int64_t m = l + (l & 1);
  double* A0 = work;
  double* A1 = work + m * m;
  double* V = work + 2 * m * m;
  double* ev = work + 3 * m * m;
  hipLaunchKernelGGL(jacobi_init, dim3((unsigned)cdiv(m * m, 256)), dim3(256), 0, s, G, l, m, A0, V);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipMemsetAsync(flags, 0, sizeof(int) * max_sweeps, s));
  NYS_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned), s));
  NYS_HIP(hipMemsetAsync(bar_err, 0, sizeof(int), s));
  JacArgs a{A0, A1, V, m, max_sweeps, flags, sweeps_out, ev, bar, bar_err};
  const size_t shmem = sizeof(double) * m;
  const int64_t need = cdiv((m / 2) * (m / 2) + m * (m / 2), 256);
  const int g = coop_blocks((const void*)jacobi_coop, 256, shmem,
                            (int)(need < 256 ? (need > 0 ? need : 1) : 256));
  void* args[] = {&a};
  NYS_HIP(hipLaunchCooperativeKernel((const void*)jacobi_coop, dim3(g), dim3(256), args, shmem, s));
  hipLaunchKernelGGL(eig_finalize, dim3((unsigned)cdiv(l, 256)), dim3(256), 0, s, ev, V, l, m,
                     nu, T, lam, sig2);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

}  // namespace nys
