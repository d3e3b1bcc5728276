// Nystrom preconditioner apply (Section 5.1.2, eq. (NysPre)) and the PCG
// iteration (Section 5.2, algorithm "Nystrom PCG") on the device.
//
// Vectors are n x k row-major blocks (k independent columns, k <= 256); a
// single right-hand side is k = 1.  CG scalars live on the device.  Each
// dot product is reduced in a fixed order by the LAST workgroup of the kernel
// that produced the per-workgroup partials (an arrival counter tells a
// workgroup that it is last), so results are bitwise reproducible and no
// separate reduction launch is needed; that workgroup also derives the CG
// scalars (alpha, beta, stopping flags).  rz (= r^T z) is double-buffered by
// iteration parity.
#include "pcg.hpp"
#include "gemm.hpp"

namespace nys {

#ifndef NYS_UC_MIN_RPW
#define NYS_UC_MIN_RPW 8  // rows per wave: >= 8 keeps small applies to fewer workgroups
#endif

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

// Per-column sum over the threads of a block that share a column; result in
// sh[c] for c < kp.  `sh` has NT doubles.
__device__ __forceinline__ void colmap_reduce(double v, const ColMap& cm, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s >= cm.kp; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
}

// True in exactly one workgroup: the last of `nblocks` to arrive.  Partial
// results written before the call are visible to it afterwards.  The last
// workgroup re-arms the counter for the next kernel.  Arriving workgroups
// publish with a release fence only (an L2 write-back, no invalidate) and
// only the last one acquires: each arrival costs ~20 ns of serialised
// fence and atomic traffic on this GPU (~9 us for 481 workgroups, measured),
// so the launches that use this keep their workgroup counts modest.
__device__ __forceinline__ bool last_block(unsigned* ctr, unsigned nblocks) {
  __shared__ int am;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned t = atomicAdd(ctr, 1u);
    am = (t == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  if (am) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *ctr = 0u;
  }
  return am != 0;
}

// Fixed-order sum of part[g][c], g < ng, by a whole block (all threads get it).
__device__ __forceinline__ double block_reduce_col(const double* part, int ng, int64_t k, int64_t c,
                                                   double* sh) {
  double s = 0.0;
  for (int g = threadIdx.x; g < ng; g += NT) s += part[(int64_t)g * k + c];
  return block_sum(s, sh);
}

// Fixed-order sum by one thread with four independent accumulators.
__device__ __forceinline__ double thread_reduce_col(const double* part, int ng, int64_t k, int64_t c) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int g = 0;
  for (; g + 3 < ng; g += 4) {
    a0 += part[(int64_t)g * k + c];
    a1 += part[(int64_t)(g + 1) * k + c];
    a2 += part[(int64_t)(g + 2) * k + c];
    a3 += part[(int64_t)(g + 3) * k + c];
  }
  for (; g < ng; ++g) a0 += part[(int64_t)g * k + c];
  return (a0 + a1) + (a2 + a3);
}

// Call f(c, total) for every column c < k from the partials (last block only).
template <typename F>
__device__ __forceinline__ void reduce_cols_last(const double* part, int ng, int64_t k, double* sh, F f) {
  if (k <= 8) {
    for (int64_t c = 0; c < k; ++c) {
      const double v = block_reduce_col(part, ng, k, c, sh);
      if (threadIdx.x == 0) f(c, v);
      __syncthreads();
    }
  } else {
    for (int64_t c = threadIdx.x; c < k; c += NT) f(c, thread_reduce_col(part, ng, k, c));
    __syncthreads();
  }
}

// ---------------------------------------------------------------- set-up

// R = B - V; ||B||^2, ||R||^2 -> scalars (last block): stopping flags, iters = 0.
template <typename T>
__global__ __launch_bounds__(NT) void cg_init_residual(int64_t n, int64_t k, const T* __restrict__ B,
                                                       const T* __restrict__ V, T* __restrict__ R,
                                                       double* __restrict__ pb, double* __restrict__ prr,
                                                       int64_t rpw, double tol, CgScalars sc) {
  __shared__ double sh[NT];
  ColMap cm(k);
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double sb = 0.0, sr = 0.0;
  if (cm.c < k)
    for (int64_t i = r0 + cm.roff; i < r1; i += cm.rstep) {
      const T b = B[i * k + cm.c];
      const T r = b - V[i * k + cm.c];
      R[i * k + cm.c] = r;
      sb += double(b) * double(b);
      sr += double(r) * double(r);
    }
  colmap_reduce(sb, cm, sh);
  if (threadIdx.x < k) pb[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
  colmap_reduce(sr, cm, sh);
  if (threadIdx.x < k) prr[blockIdx.x * k + threadIdx.x] = sh[threadIdx.x];
  if (!last_block(sc.ctr, gridDim.x)) return;
  const int ng = gridDim.x;
  reduce_cols_last(pb, ng, k, sh, [&](int64_t c, double v) { sc.bnorm2[c] = v; });
  reduce_cols_last(prr, ng, k, sh, [&](int64_t c, double v) {
    sc.rnorm2[c] = v;
    const bool conv = v <= tol * tol * sc.bnorm2[c];
    sc.done[c] = conv ? 1 : 0;
    sc.conv[c] = conv ? 1 : 0;
    sc.status[c] = conv ? NYS_OK : NYS_NOT_CONVERGED;
    sc.iters[c] = 0;
  });
}

// ---------------------------------------------------------------- iteration

// partial p^T v; last block: alpha = rz / p^T v (breakdown when p^T v <= 0).
template <typename T>
__global__ __launch_bounds__(NT) void cg_pv_alpha(int64_t n, int64_t k, const T* __restrict__ P,
                                                  const T* __restrict__ V, double* __restrict__ ppv,
                                                  int64_t rpw, CgScalars sc, int par) {
  if (*sc.alldone) return;
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
  if (!last_block(sc.ctr, gridDim.x)) return;
  reduce_cols_last(ppv, gridDim.x, k, sh, [&](int64_t c, double pv) {
    double a = 0.0;
    if (!sc.done[c]) {
      if (pv > 0.0) {
        a = sc.rz[par * k + c] / pv;
      } else {
        sc.status[c] = NYS_ERR_BREAKDOWN;
        sc.done[c] = 1;
      }
    }
    sc.alpha[c] = a;
  });
}

// X += alpha P; R -= alpha V; ||R||^2 -> last block: stopping test, iters++.
template <typename T>
__global__ __launch_bounds__(NT) void cg_update(int64_t n, int64_t k, const T* __restrict__ P,
                                                const T* __restrict__ V, T* __restrict__ X,
                                                int64_t ldx, T* __restrict__ R,
                                                double* __restrict__ prr, int64_t rpw, double tol,
                                                CgScalars sc) {
  if (*sc.alldone) return;
  __shared__ double sh[NT];
  ColMap cm(k);
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < n ? r0 + rpw : n;
  double s = 0.0;
  if (cm.c < k) {
    const T a = T(sc.alpha[cm.c]);
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
  if (!last_block(sc.ctr, gridDim.x)) return;
  reduce_cols_last(prr, gridDim.x, k, sh, [&](int64_t c, double rr) {
    if (!sc.done[c]) {
      sc.rnorm2[c] = rr;
      sc.iters[c] += 1;
      const bool conv = rr <= tol * tol * sc.bnorm2[c];
      sc.conv[c] = conv ? 1 : 0;
      if (conv) sc.status[c] = NYS_OK;
    }
  });
}

// Last-block tail of the r^T z kernels.  init: rz[0] = r^T z.  Iteration:
// beta = rz_new / rz[par], rz[1-par] = rz_new, done |= conv; all-done flag.
__device__ void rz_tail(const double* prz, int ng, int64_t k, double* sh, CgScalars sc, int par,
                        bool init) {
  reduce_cols_last(prz, ng, k, sh, [&](int64_t c, double rzn) {
    if (init) {
      sc.rz[c] = rzn;
      sc.beta[c] = 0.0;
    } else if (!sc.done[c]) {
      sc.beta[c] = rzn / sc.rz[par * k + c];
      sc.rz[(1 - par) * k + c] = rzn;
      if (sc.conv[c]) sc.done[c] = 1;
    }
  });
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int64_t c = threadIdx.x; c < k; c += NT)
    if (!sc.done[c]) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) *sc.alldone = any ? 0 : 1;
}

template <typename T>
__global__ __launch_bounds__(NT) void cg_rz(int64_t n, int64_t k, const T* __restrict__ R,
                                            const T* __restrict__ Z, double* __restrict__ prz,
                                            int64_t rpw, CgScalars sc, int par, int init) {
  if (!init && *sc.alldone) return;
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
  if (!last_block(sc.ctr, gridDim.x)) return;
  rz_tail(prz, gridDim.x, k, sh, sc, par, init != 0);
}

// P = Z + beta P for unfinished columns (init: P = Z for every column).
template <typename T>
__global__ void cg_direction(int64_t n, int64_t k, const T* __restrict__ Z, T* __restrict__ P,
                             CgScalars sc, int init) {
  if (!init && *sc.alldone) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t c = idx % k;
  if (init) {
    P[idx] = Z[idx];
  } else if (!sc.done[c]) {
    P[idx] = Z[idx] + T(sc.beta[c]) * P[idx];
  }
}

// k = 1 after the partial-only apply (mode 3): every workgroup sums the
// apply's per-workgroup parts of r^T z in the same fixed order (the order of
// the last-workgroup tail), so all agree on beta without a hand-off between
// workgroups; then P = Z + beta P on its slice.  Workgroup 0 records beta,
// r^T z, the done flag and the all-done flag as the tail would; the others
// may read those flags before or after that store and decide the same.
template <typename T>
__global__ __launch_bounds__(NT) void cg_beta_direction(int64_t n, const T* __restrict__ Z, T* __restrict__ P,
                                                        const double* __restrict__ prz, int nprz, CgScalars sc,
                                                        int par) {
  if (*sc.alldone) return;
  __shared__ double sh[NT];
  double s = 0.0;
  for (int g = threadIdx.x; g < nprz; g += NT) s += prz[g];
  const double rzn = block_sum(s, sh);
  const int done_old = sc.done[0];
  const int done_new = done_old || sc.conv[0];
  const double beta = done_old ? 0.0 : rzn / sc.rz[par];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!done_old) {
      sc.beta[0] = beta;
      sc.rz[1 - par] = rzn;
      sc.done[0] = done_new;
    }
    *sc.alldone = done_new;  // also after a breakdown flagged earlier in the iteration
  }
  if (done_new) return;
  const T b = T(beta);
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    P[i] = Z[i] + b * P[i];
}

// x += a p, r -= a v over a whole vector by one workgroup, UN entries per
// thread in flight per pass; returns this thread's part of ||r||^2 (entries in
// increasing order, so the sum does not depend on UN).
template <typename T, int UN>
__device__ __forceinline__ double update_xr(int64_t n, T a, const T* __restrict__ P, const T* __restrict__ V,
                                            T* __restrict__ X, T* __restrict__ R) {
  double rr = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += UN * NT) {
    T xv[UN], pv[UN], rv[UN], vv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      const int64_t ic = i < n ? i : n - 1;
      xv[u] = X[ic];
      pv[u] = P[ic];
      rv[u] = R[ic];
      vv[u] = V[ic];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      if (i < n) {
        X[i] = xv[u] + a * pv[u];
        const T r = rv[u] - a * vv[u];
        R[i] = r;
        rr += double(r) * double(r);
      }
    }
  }
  return rr;
}

// P = Z + b P over a whole vector by one workgroup (set-up: P = Z, P not read).
template <typename T, int UN>
__device__ __forceinline__ void update_dir(int64_t n, T b, bool setup, const T* __restrict__ Z, T* __restrict__ P) {
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += UN * NT) {
    T zv[UN], pv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      const int64_t ic = i < n ? i : n - 1;
      zv[u] = Z[ic];
      pv[u] = setup ? T(0) : P[ic];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      if (i < n) P[i] = zv[u] + b * pv[u];
    }
  }
}

// Single vector, fused: finish the operator product from its partial sums,
// v = scale * sum_g part[g] + mu p (block: 32 entries x 8 slices of g), then
// partial p^T v; the last block derives alpha and, when `fuse` is set (small
// n), also performs x += alpha p, r -= alpha v and the stopping test over the
// whole vector (saving two launches per iteration).
template <typename T>
__global__ __launch_bounds__(NT) void cg_finish_mv(int64_t n, const T* __restrict__ part, int ng, double scale,
                                                   double mu, const T* __restrict__ P, T* __restrict__ V,
                                                   double* __restrict__ ppv, CgScalars sc, int par, int fuse,
                                                   T* __restrict__ X, T* __restrict__ R,
                                                   double* __restrict__ prr, double tol) {
  // the flag is read with the first partial loads (one memory latency) and
  // tested before anything is stored; every block has at least one tile
  const int skip_all = *sc.alldone;
  __shared__ T shp[8][33];
  __shared__ double sh[NT];
  const int c = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int64_t ntiles = cdiv(n, 32);
  double pvp = 0.0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t j = tile * 32 + c;
    const int64_t jc = j < n ? j : n - 1;
    T a0 = T(0);
    // slice sl: groups sl, sl + 8, ...; 32 loads in flight per pass (one pass
    // for ng <= 256), summed in group order
    for (int g0 = sl; g0 < ng; g0 += 256) {
      T v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const int g = g0 + 8 * u;
        v[u] = g < ng ? part[(int64_t)g * n + jc] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 32; ++u) a0 += v[u];
    }
    if (skip_all) return;
    __syncthreads();
    shp[sl][c] = a0;
    __syncthreads();
    if (sl == 0 && j < n) {
      const T sum = ((shp[0][c] + shp[1][c]) + (shp[2][c] + shp[3][c])) +
                    ((shp[4][c] + shp[5][c]) + (shp[6][c] + shp[7][c]));
      const T pj = P[j];
      const T vj = T(scale) * sum + T(mu) * pj;
      V[j] = vj;
      pvp += double(pj) * double(vj);
    }
  }
  const double tot = block_sum(pvp, sh);
  if (threadIdx.x == 0) ppv[blockIdx.x] = tot;
  if (!last_block(sc.ctr, gridDim.x)) return;
  const double pv = block_reduce_col(ppv, gridDim.x, 1, 0, sh);
  __shared__ double alpha_s;
  if (threadIdx.x == 0) {
    double a = 0.0;
    if (!sc.done[0]) {
      if (pv > 0.0) {
        a = sc.rz[par] / pv;
      } else {
        sc.status[0] = NYS_ERR_BREAKDOWN;
        sc.done[0] = 1;
      }
    }
    sc.alpha[0] = a;
    alpha_s = a;
  }
  __syncthreads();
  if (!fuse) return;
  const T a = T(alpha_s);
  double rr = n <= 16 * NT ? update_xr<T, 16>(n, a, P, V, X, R) : update_xr<T, 4>(n, a, P, V, X, R);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0 && !sc.done[0]) {
    sc.rnorm2[0] = rr;
    sc.iters[0] += 1;
    const bool conv = rr <= tol * tol * sc.bnorm2[0];
    sc.conv[0] = conv ? 1 : 0;
    if (conv) sc.status[0] = NYS_OK;
  }
}

// ---------------------------------------------------------------- apply, k = 1

// Partial U^T r: part[chunk][j].  Grid (column blocks of 64, row chunks);
// thread (tx, ty): column tx of the block, rows ty (mod 4) of the chunk, RU
// loads in flight at a time.
template <typename TU, typename T, int RU>
__global__ __launch_bounds__(NT) void utr_part(int64_t n, int64_t l, const TU* __restrict__ U, int64_t ldu,
                                               const T* __restrict__ r, double* __restrict__ part,
                                               int64_t rows_per_chunk, const int* __restrict__ alldone) {
  const int skip_all = alldone ? *alldone : 0;  // tested once the first loads are issued
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + tx;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t i1 = i0 + rows_per_chunk < n ? i0 + rows_per_chunk : n;
  const int64_t jc = j < l ? j : l - 1;
  double acc = 0.0;
  for (int64_t ib = i0 + ty; ib < i1; ib += 4 * RU) {
    double uv[RU], rv[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = ib + 4 * u;
      const int64_t ic = i < i1 ? i : i1 - 1;
      uv[u] = double(U[ic * ldu + jc]);
      rv[u] = i < i1 ? double(r[ic]) : 0.0;
    }
    if (skip_all) return;
#pragma unroll
    for (int u = 0; u < RU; ++u) acc += uv[u] * rv[u];
  }
  if (skip_all) return;
  red[ty][tx] = j < l ? acc : 0.0;
  __syncthreads();
  if (ty == 0 && j < l)
    part[(int64_t)blockIdx.y * l + j] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// C'[j] = ((lam_l + mu)/(lam_j + mu) - 1) sum_chunk part[chunk][j].  Thread
// (tx, ty): column tx of the block of 64, chunks ty, ty + 4, ... (up to 32
// loads in flight per pass); the four slices are added in a fixed order.
__global__ __launch_bounds__(NT) void utr_final(int64_t l, int nch, const double* __restrict__ part,
                                                const double* __restrict__ lam, const double* __restrict__ mu,
                                                double* __restrict__ Cs, const int* __restrict__ alldone) {
  const int skip_all = alldone ? *alldone : 0;  // tested once the first loads are issued
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + tx;
  const int64_t jc = j < l ? j : l - 1;
  double acc = 0.0;
  for (int q0 = ty; q0 < nch; q0 += 4 * 32) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int q = q0 + 4 * u;
      v[u] = q < nch ? part[(int64_t)q * l + jc] : 0.0;
    }
    if (skip_all) return;
#pragma unroll
    for (int u = 0; u < 32; ++u) acc += v[u];
  }
  if (skip_all) return;
  red[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && j < l) {
    const double tot = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
    const double m = mu[0];
    Cs[j] = ((lam[l - 1] + m) / (lam[j] + m) - 1.0) * tot;
  }
}

// z_i = r_i + sum_j U[i][j] C'[j]: one wave per group of four rows, whose
// 4 x NJ loads per lane (columns lane + 64 jj, l <= 64 NJ) are issued together.
// mode 0: plain apply; mode 1: also r^T z for the set-up; mode 2: r^T z,
// beta and flags; mode 3: per-workgroup parts of r^T z only (cg_beta_direction
// finishes them); mode 4 (uc_vec only): r^T z from utr_final_rr's parts, beta
// and the direction update on each wave's own rows.
template <typename TU, typename T, int NJ>
__global__ __launch_bounds__(NT) void uc_rz(int64_t n, int64_t l, const TU* __restrict__ U, int64_t ldu,
                                            const double* __restrict__ Cs, const T* __restrict__ r,
                                            T* __restrict__ z, int64_t rows_per_wave,
                                            double* __restrict__ prz, CgScalars sc, int par, int mode,
                                            T* __restrict__ Pd) {
  // the flag is read with the first loads and tested before anything is stored
  const int skip_all = mode >= 2 ? *sc.alldone : 0;
  __shared__ double sh[NT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T cs[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int64_t j = lane + 64 * jj;
    cs[jj] = j < l ? T(Cs[j]) : T(0);
  }
  const int64_t w0 = ((int64_t)blockIdx.x * 4 + wave) * rows_per_wave;
  const int64_t w1 = w0 + rows_per_wave < n ? w0 + rows_per_wave : n;
  double rzp = 0.0;
  for (int64_t ib = w0; ib < w1; ib += 4) {
    const int64_t nr = (w1 - ib) < 4 ? (w1 - ib) : 4;
    TU u[4][NJ];
    T rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = r[ib + (q < nr ? q : 0)];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = ib + (q < nr ? q : 0);
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const int64_t j = lane + 64 * jj;
        u[q][jj] = U[row * ldu + (j < l ? j : l - 1)];
      }
    }
    if (skip_all) return;
    T sv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T acc = T(0);
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) acc += T(u[q][jj]) * cs[jj];  // cs = 0 past l
      sv[q] = wave_sum(acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < nr) {
        const T zi = rv[q] + sv[q];
        if (lane == q) z[ib + q] = zi;
        rzp += double(rv[q]) * double(zi);
      }
    }
  }
  if (mode == 0 || skip_all) return;
  // every lane of a wave holds the same rzp; lane 0 contributes it
  const double tot = block_sum(lane == 0 ? rzp : 0.0, sh);
  if (threadIdx.x == 0) prz[blockIdx.x] = tot;
  if (mode == 3) return;
  if (!last_block(sc.ctr, gridDim.x)) return;
  rz_tail(prz, gridDim.x, 1, sh, sc, par, mode == 1);
  if (Pd == nullptr) return;
  // fused direction update (small n): P = Z (set-up) or P = Z + beta P
  __syncthreads();
  const T b = mode == 1 ? T(0) : T(sc.beta[0]);
  if (mode == 1 || !sc.done[0]) {  // set-up: P = Z (P not read: it is uninitialised)
    if (n <= 16 * NT) update_dir<T, 16>(n, b, mode == 1, z, Pd);
    else update_dir<T, 4>(n, b, mode == 1, z, Pd);
  }
}

// ---------------------------------------------------------------- apply, k = 1, 16-byte U loads
//
// Rows of U that are 16-byte aligned with ell a multiple of the vector width
// (4 floats or 2 doubles) are read with one 16-byte load per lane, a wave
// covering 64 vectors of a row.  U^T r: each thread accumulates its columns
// over its rows (in float32 for a float32 U, float64 otherwise); the four
// waves are combined in float64 in a fixed order.  U c: the wave forms four
// rows' dot products at a time from 16-byte loads.

template <typename TU>
struct UVec;
template <>
struct UVec<float> {
  typedef float4 type;
  typedef float acc;
  static constexpr int E = 4;
  static __device__ __forceinline__ float get(const float4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
  }
};
template <>
struct UVec<double> {
  typedef double2 type;
  typedef double acc;
  static constexpr int E = 2;
  static __device__ __forceinline__ double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
};

// part[chunk][j] = sum over the chunk's rows of U[i][j] r[i]; grid (column
// groups of 64 E, row chunks); wave w takes rows w, w + 4, ... of the chunk,
// RU rows in flight per pass.
template <typename TU, typename T, int RU>
__global__ __launch_bounds__(NT) void utr_vec(int64_t n, int64_t l, const TU* __restrict__ U, int64_t ldu,
                                              const T* __restrict__ r, double* __restrict__ part,
                                              int64_t rows_per_chunk, const int* __restrict__ alldone) {
  typedef typename UVec<TU>::type VT;
  typedef typename UVec<TU>::acc TA;
  constexpr int E = UVec<TU>::E;
  const int skip_all = alldone ? *alldone : 0;  // tested once the first loads are issued
  __shared__ double red[4][64 * E];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j0 = ((int64_t)blockIdx.x * 64 + lane) * E;
  const bool ok = j0 < l;
  const int64_t jc = ok ? j0 : 0;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t i1 = i0 + rows_per_chunk < n ? i0 + rows_per_chunk : n;
  TA acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = TA(0);
  for (int64_t ib = i0 + wave; ib < i1; ib += 4 * RU) {
    VT uv[RU];
    TA rv[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = ib + 4 * u;
      const int64_t ic = i < i1 ? i : i1 - 1;
      uv[u] = *reinterpret_cast<const VT*>(U + ic * ldu + jc);
      rv[u] = i < i1 ? TA(r[ic]) : TA(0);
    }
    if (skip_all) return;
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += TA(UVec<TU>::get(uv[u], e)) * rv[u];
  }
  if (skip_all) return;
#pragma unroll
  for (int e = 0; e < E; ++e) red[wave][lane * E + e] = double(acc[e]);
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * E; q += NT) {
    const int64_t j = (int64_t)blockIdx.x * 64 * E + q;
    if (j < l) part[(int64_t)blockIdx.y * l + j] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
  (void)ok;
}

// k = 1, after a product that also gave pvq (see op_matvec_partials: X^T X,
// or a square RBF operator): p^T (A + mu I) p = scale sum_{g < npvq} pvq[g] +
// mu sum_{g < npp} pvq[npvq + g], summed by every workgroup in the same fixed
// order, so each knows alpha at once and no workgroup hands it to another.
// Workgroup b owns entries 32 b .. 32 b + 31 (n <= 32 gridDim.x): v_j from
// the ng partials (8 slices of 32 columns, as cg_finish_mv), x_j += alpha p_j,
// r_j -= alpha v_j, a part of ||r||^2, and this workgroup's part of U^T r over
// its 32 rows of U in float64.  With nvec = l / E 16-byte vectors per row, G
// groups of nvec threads (G nvec <= NT) share the rows (group g takes rows g,
// g + G, ...; their sums are added in a fixed order through LDS); with G = 1
// thread t owns vectors t and t + NT (CG = 2).  Every load that does not need
// alpha (the first rows of U, the partials, p, x, r) is issued before alpha is
// formed.  Workgroup 0 records alpha and a breakdown.
template <typename T, typename TU, int CG>
__global__ __launch_bounds__(NT) void cg_finish_pvq(int64_t n, const T* __restrict__ part, int ng,
                                                    const double* __restrict__ pvq, int npvq, int npp,
                                                    double scale, double mu, const T* __restrict__ P,
                                                    T* __restrict__ V, T* __restrict__ X, T* __restrict__ R,
                                                    const TU* __restrict__ U, int64_t l, int64_t ldu, int G,
                                                    double* __restrict__ apart, double* __restrict__ prr,
                                                    CgScalars sc, int par) {
  typedef typename UVec<TU>::type VT;
  constexpr int E = UVec<TU>::E;
  constexpr int RB = CG == 1 ? 16 : 8;  // rows of U in flight per thread
  __shared__ T shp[8][33];
  __shared__ double sh[NT / 64], sh2[NT / 64];
  __shared__ double rs[32];
  __shared__ double red[NT * E];  // the groups' sums when G > 1
  const int skip_all = *sc.alldone;
  const int c = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int64_t tile = blockIdx.x;
  const int64_t j = tile * 32 + c;
  const int64_t jc = j < n ? j : n - 1;
  const int64_t rows = n - tile * 32 < 32 ? n - tile * 32 : 32;
  const int nvec = (int)(l / E);
  const int grp = G > 1 ? (int)threadIdx.x / nvec : 0;
  const int rpt = 32 / G;  // rows per thread
  int64_t uo[CG];
  bool uok[CG];
#pragma unroll
  for (int v = 0; v < CG; ++v) {
    const int vi = G > 1 ? (int)threadIdx.x % nvec : v * NT + (int)threadIdx.x;
    uok[v] = vi < nvec && grp < G;
    uo[v] = uok[v] ? (int64_t)vi * E : 0;
  }
  const TU* ub = U + tile * 32 * ldu;
  VT uv[RB][CG];
  auto load_u = [&](int k0) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int k = k0 + rr, r = grp + G * k;
      const int64_t row = r < rows ? r : 0;  // rows past n re-read the tile's first (rs = 0)
#pragma unroll
      for (int v = 0; v < CG; ++v)
        if (uok[v] && k < rpt) uv[rr][v] = *reinterpret_cast<const VT*>(ub + row * ldu + uo[v]);
    }
  };
  load_u(0);
  T a0 = T(0);
  for (int g0 = sl; g0 < ng; g0 += 256) {
    T w[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int g = g0 + 8 * u;
      w[u] = g < ng ? part[(int64_t)g * n + jc] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) a0 += w[u];
  }
  T pj = T(0), xj = T(0), rj = T(0);
  if (sl == 0 && j < n) {
    pj = P[j];
    xj = X[j];
    rj = R[j];
  }
  double q = 0.0, qp = 0.0;
  for (int g = threadIdx.x; g < npvq; g += NT) q += pvq[g];
  for (int g = threadIdx.x; g < npp; g += NT) qp += pvq[npvq + g];
  const double pv = block_sum1(scale * q + mu * qp, sh);
  if (skip_all) return;  // the same value for every thread
  const int done = sc.done[0];
  const double a_d = (done || !(pv > 0.0)) ? 0.0 : sc.rz[par] / pv;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc.alpha[0] = a_d;
    if (!done && !(pv > 0.0)) {
      sc.status[0] = NYS_ERR_BREAKDOWN;
      sc.done[0] = 1;
    }
  }
  const T a = T(a_d);
  shp[sl][c] = a0;
  __syncthreads();
  double rrp = 0.0;
  if (sl == 0) {
    double rj_d = 0.0;
    if (j < n) {
      const T sum = ((shp[0][c] + shp[1][c]) + (shp[2][c] + shp[3][c])) +
                    ((shp[4][c] + shp[5][c]) + (shp[6][c] + shp[7][c]));
      const T vj = T(scale) * sum + T(mu) * pj;
      V[j] = vj;
      X[j] = xj + a * pj;
      rj = rj - a * vj;
      R[j] = rj;
      rrp = double(rj) * double(rj);
      rj_d = double(rj);
    }
    rs[c] = rj_d;  // 0 past n
  }
  __syncthreads();
  double acc[CG][E];
#pragma unroll
  for (int v = 0; v < CG; ++v)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[v][e] = 0.0;
  for (int k0 = 0; k0 < rpt; k0 += RB) {
    if (k0 > 0) load_u(k0);
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int k = k0 + rr;
      if (k < rpt) {
        const double rv = rs[grp + G * k < 32 ? grp + G * k : 0];
#pragma unroll
        for (int v = 0; v < CG; ++v)
          if (uok[v])
#pragma unroll
            for (int e = 0; e < E; ++e) acc[v][e] += double(UVec<TU>::get(uv[rr][v], e)) * rv;
      }
    }
  }
  if (G == 1) {
#pragma unroll
    for (int v = 0; v < CG; ++v)
      if (uok[v])
#pragma unroll
        for (int e = 0; e < E; ++e) apart[(int64_t)blockIdx.x * l + uo[v] + e] = acc[v][e];
  } else {
    if (uok[0])
#pragma unroll
      for (int e = 0; e < E; ++e) red[grp * nvec * E + uo[0] + e] = acc[0][e];
    __syncthreads();
    for (int i = threadIdx.x; i < nvec * E; i += NT) {
      double tot = 0.0;
      for (int g = 0; g < G; ++g) tot += red[g * nvec * E + i];
      apart[(int64_t)blockIdx.x * l + i] = tot;
    }
  }
  const double rr = block_sum1(rrp, sh2);
  if (threadIdx.x == 0) prr[blockIdx.x] = rr;
}

// utr_final plus, in workgroup 0, the stopping test of the update that
// cg_finish_pvq made: ||r||^2 from its per-workgroup parts (fixed order).
// rzq[b] (b < gridDim.x) receives workgroup b's part of w^T D w and
// rzq[gridDim.x] = ||r||^2, from which uc_vec's mode 4 forms r^T z.
__global__ __launch_bounds__(NT) void utr_final_rr(int64_t l, int nch, const double* __restrict__ part,
                                                   const double* __restrict__ lam, const double* __restrict__ mu,
                                                   double* __restrict__ Cs, const double* __restrict__ prr, int nprr,
                                                   CgScalars sc, double tol, double* __restrict__ rzq) {
  const int skip_all = *sc.alldone;
  __shared__ double red[4][64];
  __shared__ double sh[NT];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + tx;
  const int64_t jc = j < l ? j : l - 1;
  // loads that need nothing from this launch, issued first
  const double m = mu[0], lam_l = lam[l - 1], lam_j = lam[jc];
  double s = 0.0;
  int done0 = 1;
  double bn2 = 0.0;
  if (blockIdx.x == 0) {
    for (int q = threadIdx.x; q < nprr; q += NT) s += prr[q];
    done0 = sc.done[0];
    bn2 = sc.bnorm2[0];
  }
  double acc = 0.0;
  for (int q0 = ty; q0 < nch; q0 += 4 * 16) {  // 16 loads in flight per thread
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + 4 * u;
      v[u] = q < nch ? part[(int64_t)q * l + jc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += v[u];
  }
  if (skip_all) return;
  red[ty][tx] = acc;
  __syncthreads();
  double wdw = 0.0;  // this column's w_j d_j w_j, w = U^T r (unscaled), d_j the apply's diagonal
  if (ty == 0 && j < l) {
    const double tot = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
    const double cj = ((lam_l + m) / (lam_j + m) - 1.0) * tot;
    Cs[j] = cj;
    wdw = cj * tot;
  }
  // r^T z = ||r||^2 + w^T D w (z = r + U D w): this workgroup's part of the
  // second term, and ||r||^2 from workgroup 0, for the apply that follows
  if (ty == 0) {  // only wave 0 holds columns
    wdw = wave_sum(wdw);
    if (tx == 0) rzq[blockIdx.x] = wdw;
  }
  if (blockIdx.x != 0) return;
  const double rr = block_sum1(s, sh);
  if (threadIdx.x == 0) rzq[gridDim.x] = rr;
  if (threadIdx.x == 0 && !done0) {
    sc.rnorm2[0] = rr;
    sc.iters[0] += 1;
    const bool conv = rr <= tol * tol * bn2;
    sc.conv[0] = conv ? 1 : 0;
    if (conv) sc.status[0] = NYS_OK;
  }
}

// z_i = r_i + sum_j U[i][j] C'[j] with 16-byte loads: lane owns vectors
// lane + 64 g (g < NG) of every row, four rows per pass.  Modes as uc_rz.
template <typename TU, typename T, int NG>
__global__ __launch_bounds__(NT) void uc_vec(int64_t n, int64_t l, const TU* __restrict__ U, int64_t ldu,
                                             const double* __restrict__ Cs, const T* __restrict__ r,
                                             T* __restrict__ z, int64_t rows_per_wave,
                                             double* __restrict__ prz, CgScalars sc, int par, int mode,
                                             T* __restrict__ Pd) {
  typedef typename UVec<TU>::type VT;
  constexpr int E = UVec<TU>::E;
  const int skip_all = mode >= 2 ? *sc.alldone : 0;
  T bz = T(0);
  int dn = 0;
  __shared__ double sh[NT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T cs[NG][E];
  int64_t off[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int64_t j0 = ((int64_t)g * 64 + lane) * E;
    off[g] = j0 < l ? j0 : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) cs[g][e] = j0 < l ? T(Cs[j0 + e]) : T(0);
  }
  const int64_t w0 = ((int64_t)blockIdx.x * 4 + wave) * rows_per_wave;
  const int64_t w1 = w0 + rows_per_wave < n ? w0 + rows_per_wave : n;
  double rzp = 0.0;
  // four rows per pass; the next pass's rows are loaded while this one is
  // reduced (ping-pong buffers; a pass past the range re-reads row w0)
  VT ua[4][NG], ub[4][NG];
  T ra[4], rb[4];
  auto load = [&](VT(&u)[4][NG], T(&rv)[4], int64_t ib) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = ib + q < w1 ? ib + q : w0;
      rv[q] = r[row];
#pragma unroll
      for (int g = 0; g < NG; ++g) u[q][g] = *reinterpret_cast<const VT*>(U + row * ldu + off[g]);
    }
  };
  // lane l finishes row q = (l >> 4) & 3 of the pass: the four per-lane sums
  // are halved across lanes l ^ 32, then l ^ 16 (seven shuffles for the four
  // rows instead of 24), then summed over the 16 lanes of the group
  const int myq = (lane >> 4) & 3;
  const bool hi32 = (lane & 32) != 0, hi16 = (lane & 16) != 0;
  auto finish = [&](VT(&u)[4][NG], T(&rv)[4], int64_t ib) {
    const int64_t nr = (w1 - ib) < 4 ? (w1 - ib) : 4;
    T a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T acc = T(0);
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) acc += T(UVec<TU>::get(u[q][g], e)) * cs[g][e];  // cs = 0 past l
      a[q] = acc;
    }
    const T b0 = (hi32 ? a[2] : a[0]) + __shfl_xor(hi32 ? a[0] : a[2], 32, 64);
    const T b1 = (hi32 ? a[3] : a[1]) + __shfl_xor(hi32 ? a[1] : a[3], 32, 64);
    T c = (hi16 ? b1 : b0) + __shfl_xor(hi16 ? b0 : b1, 16, 64);
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if (myq < nr && (lane & 15) == 0) {
      const T zi = rv[myq] + c;
      z[ib + myq] = zi;
      rzp += double(rv[myq]) * double(zi);
      if (mode == 4 && !dn) Pd[ib + myq] = zi + bz * Pd[ib + myq];
    }
  };
  int64_t ib = w0;
  if (ib < w1) load(ua, ra, ib);
  // mode 4 (after utr_final_rr, whose cdiv(l, 64) workgroups left their parts
  // of w^T D w in prz, then ||r||^2): r^T z and so beta are known before the
  // apply, and each wave sets p = z + beta p on its own rows (formed after the
  // first rows of U are on their way)
  if (mode == 4) {
    __shared__ double shq[NT / 64];
    const int nq = (int)cdiv(l, 64);
    const int done_old = sc.done[0];
    const int conv = sc.conv[0];
    const double rz_old = sc.rz[par];
    double q = 0.0;
    for (int i = threadIdx.x; i <= nq; i += NT) q += prz[i];
    const double rzn = block_sum1(q, shq);
    dn = done_old || conv;
    const double beta = done_old ? 0.0 : rzn / rz_old;
    bz = T(beta);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (!done_old) {
        sc.beta[0] = beta;
        sc.rz[1 - par] = rzn;
        sc.done[0] = dn;
      }
      *sc.alldone = dn;  // also after a breakdown flagged earlier in the iteration
    }
  }
  if (skip_all) return;
  for (; ib + 4 < w1; ib += 8) {
    load(ub, rb, ib + 4);
    finish(ua, ra, ib);
    if (ib + 8 < w1) load(ua, ra, ib + 8);
    finish(ub, rb, ib + 4);
  }
  if (ib < w1) finish(ua, ra, ib);
  if (mode == 0 || mode == 4 || skip_all) return;
  // lanes 0, 16, 32 and 48 hold the rows' parts of r^T z
  const double tot = block_sum(rzp, sh);
  if (threadIdx.x == 0) prz[blockIdx.x] = tot;
  if (mode == 3) return;
  if (!last_block(sc.ctr, gridDim.x)) return;
  rz_tail(prz, gridDim.x, 1, sh, sc, par, mode == 1);
  if (Pd == nullptr) return;
  __syncthreads();
  const T b = mode == 1 ? T(0) : T(sc.beta[0]);
  if (mode == 1 || !sc.done[0]) {
    if (n <= 16 * NT) update_dir<T, 16>(n, b, mode == 1, z, Pd);
    else update_dir<T, 4>(n, b, mode == 1, z, Pd);
  }
}

template <typename TU>
bool uvec_ok(const PrecDesc& P) {
  constexpr int E = UVec<TU>::E;
  return P.ell % E == 0 && P.ldu % E == 0 && (reinterpret_cast<uintptr_t>(P.U) % 16) == 0 &&
         P.ell <= 64 * E * 8;
}

// ---------------------------------------------------------------- apply, k > 1

// C'[j][c] = ((lam_l + mu_c)/(lam_j + mu_c) - 1) C[j][c]
__global__ void apply_scale_blk(int64_t l, int64_t k, const double* __restrict__ C,
                                const double* __restrict__ lam, const double* __restrict__ mu,
                                int64_t nrhs, double* __restrict__ Cs, const int* __restrict__ done,
                                const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * k) return;
  const int64_t j = idx / k, c = idx % k;
  const double m = mu[c / nrhs];
  const double f = (lam[l - 1] + m) / (lam[j] + m) - 1.0;
  Cs[idx] = (done && done[c]) ? 0.0 : f * C[idx];
}

template <typename T>
__global__ void copy_vec(int64_t count, const T* __restrict__ src, T* __restrict__ dst,
                         const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

int64_t groups_for(int64_t n, int64_t k) {
  int64_t g = cdiv(n * k, 1024);
  if (g < 1) g = 1;
  if (g > 512) g = 512;
  return g;
}

// k = 1: Cs = scaled U^T r.
nys_status utr_launch(const PrecDesc& P, const double* mu_dev, const void* R, bool f32, double* part,
                      double* Cs, unsigned* ctr, const int* alldone, hipStream_t s) {
  (void)ctr;
  const int64_t n = P.n, l = P.ell;
  const bool vec = P.dtype == NYS_F64 ? uvec_ok<double>(P) : uvec_ok<float>(P);
  if (vec) {
    // 16-byte U loads: column groups of 64 vectors, row chunks sized for about
    // four workgroups per compute unit (at most 512 chunks, >= 32 rows each)
    const int E = P.dtype == NYS_F64 ? 2 : 4;
    const int64_t cg = cdiv(l, (int64_t)64 * E);
    int64_t want = cdiv((int64_t)4 * num_cus(), cg);
    want = want < 1 ? 1 : want > 512 ? 512 : want;
    int64_t rpc = cdiv(n, want);
    rpc = cdiv(rpc < 32 ? 32 : rpc, 32) * 32;
    const int64_t rc = cdiv(n, rpc);
    dim3 grid((unsigned)cg, (unsigned)rc);
#define LV(TU_, T_)                                                                                  \
  hipLaunchKernelGGL((utr_vec<TU_, T_, 8>), grid, dim3(NT), 0, s, n, l, static_cast<const TU_*>(P.U), \
                     P.ldu, static_cast<const T_*>(R), part, rpc, alldone)
    if (P.dtype == NYS_F64 && !f32) LV(double, double);
    else if (P.dtype == NYS_F64 && f32) LV(double, float);
    else if (P.dtype == NYS_F32 && !f32) LV(float, double);
    else LV(float, float);
#undef LV
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(utr_final, dim3((unsigned)cdiv(l, 64)), dim3(NT), 0, s, l, (int)rc, part, P.lam, mu_dev,
                       Cs, alldone);
    NYS_CHECK_LAUNCH();
    return NYS_OK;
  }
  const int64_t cb = cdiv(l, 64);
  // chunks of 32 rows (8 loads per thread, all in flight), at most 512 chunks
  int64_t rpc = cdiv(n, 512);
  rpc = cdiv(rpc < 32 ? 32 : rpc, 32) * 32;
  const int64_t rc = cdiv(n, rpc);
  dim3 grid((unsigned)cb, (unsigned)rc);
#define LU(TU_, T_)                                                                                  \
  hipLaunchKernelGGL((utr_part<TU_, T_, 8>), grid, dim3(NT), 0, s, n, l, static_cast<const TU_*>(P.U), \
                     P.ldu, static_cast<const T_*>(R), part, rpc, alldone)
  if (P.dtype == NYS_F64 && !f32) LU(double, double);
  else if (P.dtype == NYS_F64 && f32) LU(double, float);
  else if (P.dtype == NYS_F32 && !f32) LU(float, double);
  else LU(float, float);
#undef LU
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(utr_final, dim3((unsigned)cdiv(l, 64)), dim3(NT), 0, s, l, (int)rc, part, P.lam, mu_dev, Cs,
                     alldone);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename TU, typename T>
void uc_dispatch(int64_t n, int64_t l, const TU* U, int64_t ldu, const double* Cs, const T* R, T* Z,
                 int64_t rpw, double* prz, const CgScalars& sc, int par, int mode, T* Pd, unsigned nb,
                 hipStream_t s, bool vec) {
  if (vec) {
    constexpr int W = 64 * UVec<TU>::E;  // columns per vector group
#define LG(NG) hipLaunchKernelGGL((uc_vec<TU, T, NG>), dim3(nb), dim3(NT), 0, s, n, l, U, ldu, Cs, R, Z, rpw, prz, sc, par, mode, Pd)
    if (l <= W) LG(1);
    else if (l <= 2 * W) LG(2);
    else if (l <= 4 * W) LG(4);
    else LG(8);
#undef LG
    return;
  }
#define LC(NJ) hipLaunchKernelGGL((uc_rz<TU, T, NJ>), dim3(nb), dim3(NT), 0, s, n, l, U, ldu, Cs, R, Z, rpw, prz, sc, par, mode, Pd)
  if (l <= 128) LC(2);
  else if (l <= 256) LC(4);
  else if (l <= 512) LC(8);
  else if (l <= 1024) LC(16);
  else LC(32);
#undef LC
}

// rows per wave of the k = 1 apply: at most 512 workgroups (partial buffer
// size) and at least NYS_UC_MIN_RPW rows per wave
int64_t uc_rows_per_wave(int64_t n) {
  const int64_t rpw = cdiv(n, 4 * 512);
  return cdiv(rpw < NYS_UC_MIN_RPW ? NYS_UC_MIN_RPW : rpw, 4) * 4;
}
unsigned uc_blocks(int64_t n) { return (unsigned)cdiv(cdiv(n, uc_rows_per_wave(n)), 4); }

nys_status uc_launch(const PrecDesc& P, const double* Cs, const void* R, void* Z, bool f32, double* prz,
                     const CgScalars& sc, int par, int mode, hipStream_t s, void* Pd = nullptr) {
  const int64_t n = P.n, l = P.ell;
  if (l > 2048) {
    set_error("preconditioner apply: l = %lld > 2048 not supported", (long long)l);
    return NYS_ERR_ARG;
  }
  const int64_t rpw = uc_rows_per_wave(n);
  const unsigned nb = (unsigned)cdiv(cdiv(n, rpw), 4);
  const bool vec = P.dtype == NYS_F64 ? uvec_ok<double>(P) : uvec_ok<float>(P);
  if (P.dtype == NYS_F64 && !f32)
    uc_dispatch<double, double>(n, l, static_cast<const double*>(P.U), P.ldu, Cs, static_cast<const double*>(R),
                                static_cast<double*>(Z), rpw, prz, sc, par, mode, static_cast<double*>(Pd), nb, s, vec);
  else if (P.dtype == NYS_F64 && f32)
    uc_dispatch<double, float>(n, l, static_cast<const double*>(P.U), P.ldu, Cs, static_cast<const float*>(R),
                               static_cast<float*>(Z), rpw, prz, sc, par, mode, static_cast<float*>(Pd), nb, s, vec);
  else if (P.dtype == NYS_F32 && !f32)
    uc_dispatch<float, double>(n, l, static_cast<const float*>(P.U), P.ldu, Cs, static_cast<const double*>(R),
                               static_cast<double*>(Z), rpw, prz, sc, par, mode, static_cast<double*>(Pd), nb, s, vec);
  else
    uc_dispatch<float, float>(n, l, static_cast<const float*>(P.U), P.ldu, Cs, static_cast<const float*>(R),
                              static_cast<float*>(Z), rpw, prz, sc, par, mode, static_cast<float*>(Pd), nb, s, vec);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Block apply Z = R + U (f .* (U^T R)) through the MFMA GEMM.  float64
// vectors take U in either precision; float32 vectors need a float32 U.
template <typename T>
__global__ void apply_scale_blk_t(int64_t l, int64_t k, const T* __restrict__ C, const double* __restrict__ lam,
                                  const double* __restrict__ mu, int64_t nrhs, T* __restrict__ Cs,
                                  const int* __restrict__ done, const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * k) return;
  const int64_t j = idx / k, c = idx % k;
  const double m = mu[c / nrhs];
  const double f = (lam[l - 1] + m) / (lam[j] + m) - 1.0;
  Cs[idx] = (done && done[c]) ? T(0) : T(f * double(C[idx]));
}

nys_status apply_block(const PrecDesc& P, const double* mu_dev, int64_t nrhs, const double* R, double* Z,
                       int64_t k, const int* done, const int* alldone, double* part, size_t part_elems,
                       double* C, double* Cs, hipStream_t s) {
  const int64_t n = P.n, l = P.ell;
  if (P.dtype == NYS_F64)
    NYS_TRY((gemm<double, double, double>(true, false, l, k, n, 1.0, static_cast<const double*>(P.U), P.ldu, R,
                                          k, 0.0, C, k, part, part_elems, s, alldone)));
  else
    NYS_TRY((gemm<double, float, double>(true, false, l, k, n, 1.0, static_cast<const float*>(P.U), P.ldu, R,
                                         k, 0.0, C, k, part, part_elems, s, alldone)));
  hipLaunchKernelGGL(apply_scale_blk, dim3((unsigned)cdiv(l * k, 256)), dim3(256), 0, s, l, k, C, P.lam,
                     mu_dev, nrhs, Cs, done, alldone);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(copy_vec<double>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n * k, R, Z,
                     alldone);
  NYS_CHECK_LAUNCH();
  if (P.dtype == NYS_F64)
    NYS_TRY((gemm<double, double, double>(false, false, n, k, l, 1.0, static_cast<const double*>(P.U), P.ldu,
                                          Cs, k, 1.0, Z, k, part, part_elems, s, alldone)));
  else
    NYS_TRY((gemm<double, float, double>(false, false, n, k, l, 1.0, static_cast<const float*>(P.U), P.ldu,
                                         Cs, k, 1.0, Z, k, part, part_elems, s, alldone)));
  return NYS_OK;
}

nys_status apply_block_f32(const PrecDesc& P, const double* mu_dev, int64_t nrhs, const float* R, float* Z,
                           int64_t k, const int* done, const int* alldone, double* part, size_t part_elems,
                           double* Cbuf, double* Csbuf, hipStream_t s) {
  const int64_t n = P.n, l = P.ell;
  if (P.dtype != NYS_F32) {
    set_error("float32 block preconditioner apply needs a float32 U");
    return NYS_ERR_ARG;
  }
  const float* U = static_cast<const float*>(P.U);
  float* C = reinterpret_cast<float*>(Cbuf);
  float* Cs = reinterpret_cast<float*>(Csbuf);
  float* fpart = reinterpret_cast<float*>(part);
  NYS_TRY((gemm<float, float, float>(true, false, l, k, n, 1.0f, U, P.ldu, R, k, 0.0f, C, k, fpart, part_elems, s,
                                     alldone)));
  hipLaunchKernelGGL(apply_scale_blk_t<float>, dim3((unsigned)cdiv(l * k, 256)), dim3(256), 0, s, l, k, C, P.lam,
                     mu_dev, nrhs, Cs, done, alldone);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(copy_vec<float>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n * k, R, Z, alldone);
  NYS_CHECK_LAUNCH();
  NYS_TRY((gemm<float, float, float>(false, false, n, k, l, 1.0f, U, P.ldu, Cs, k, 1.0f, Z, k, fpart, part_elems, s,
                                     alldone)));
  return NYS_OK;
}

template <typename T>
nys_status apply_block_t(const PrecDesc& P, const double* mu_dev, int64_t nrhs, const T* R, T* Z, int64_t k,
                         const int* done, const int* alldone, PcgWork& w, hipStream_t s) {
  if (sizeof(T) == 8)
    return apply_block(P, mu_dev, nrhs, reinterpret_cast<const double*>(R), reinterpret_cast<double*>(Z), k, done,
                       alldone, w.apart, w.apart_elems, w.Ct, w.Cs, s);
  return apply_block_f32(P, mu_dev, nrhs, reinterpret_cast<const float*>(R), reinterpret_cast<float*>(Z), k, done,
                         alldone, w.apart, w.apart_elems, w.Ct, w.Cs, s);
}

}  // namespace

// ---------------------------------------------------------------- host API

size_t precond_part_elems(int64_t n, int64_t l, int64_t k) {
  const size_t a = (size_t)512 * (size_t)l * (size_t)k;
  const size_t b = gemm_scratch_elems(l, k);
  const size_t c = gemm_scratch_elems(n, k);
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

nys_status precond_apply_standalone(const PrecDesc& P, const double* mu_dev, const double* R, double* Z,
                                    int64_t k, double* part, size_t part_elems, double* Cs, double* Ct,
                                    unsigned* ctr, hipStream_t s) {
  if (k == 1) {
    NYS_TRY(utr_launch(P, mu_dev, R, false, part, Cs, ctr, nullptr, s));
    CgScalars none{};
    return uc_launch(P, Cs, R, Z, false, nullptr, none, 0, 0, s);
  }
  return apply_block(P, mu_dev, k, R, Z, k, nullptr, nullptr, part, part_elems, Ct, Cs, s);
}

template <typename T>
nys_status pcg_setup(int64_t n, int64_t k, const PrecDesc& P, const double* mu_dev, int64_t nrhs,
                     const T* B, const T* V, T* R, T* Z, T* Pd, PcgWork& w, const CgScalars& sc, double tol,
                     hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  const int64_t ng = groups_for(n, k);
  const int64_t rpw = cdiv(n, ng);
  hipLaunchKernelGGL(cg_init_residual<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, B, V, R, w.pb, w.prr, rpw,
                     tol, sc);
  NYS_CHECK_LAUNCH();
  if (k == 1) {
    NYS_TRY(utr_launch(P, mu_dev, R, f32, w.apart, w.Cs, sc.ctr + 1, nullptr, s));
    NYS_TRY(uc_launch(P, w.Cs, R, Z, f32, w.prz, sc, 0, 1, s));
  } else {
    NYS_TRY(apply_block_t<T>(P, mu_dev, nrhs, R, Z, k, nullptr, nullptr, w, s));
    hipLaunchKernelGGL(cg_rz<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, R, Z, w.prz, rpw, sc, 0, 1);
    NYS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(cg_direction<T>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, Z, Pd, sc, 1);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// k = 1: beta and P = Z + beta P after a mode-3 apply
template <typename T>
nys_status beta_direction_launch(int64_t n, const T* Z, T* Pd, PcgWork& w, const CgScalars& sc, int par,
                                 hipStream_t s) {
  int64_t g = cdiv(n, 4 * NT);  // four entries per thread
  g = g < 1 ? 1 : g > 1024 ? 1024 : g;
  hipLaunchKernelGGL(cg_beta_direction<T>, dim3((unsigned)g), dim3(NT), 0, s, n, Z, Pd, w.prz, (int)uc_blocks(n),
                     sc, par);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status pcg_iteration(int64_t n, int64_t k, const PrecDesc& P, const double* mu_dev, int64_t nrhs,
                         const T* V, T* X, int64_t ldx, T* R, T* Z, T* Pd, PcgWork& w, const CgScalars& sc,
                         int par, double tol, hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  const int64_t ng = groups_for(n, k);
  const int64_t rpw = cdiv(n, ng);
  hipLaunchKernelGGL(cg_pv_alpha<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, Pd, V, w.ppv, rpw, sc, par);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_update<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, Pd, V, X, ldx, R, w.prr, rpw, tol,
                     sc);
  NYS_CHECK_LAUNCH();
  if (k == 1) {
    NYS_TRY(utr_launch(P, mu_dev, R, f32, w.apart, w.Cs, sc.ctr + 1, sc.alldone, s));
    NYS_TRY(uc_launch(P, w.Cs, R, Z, f32, w.prz, sc, par, 3, s));
    return beta_direction_launch<T>(n, Z, Pd, w, sc, par, s);
  }
  NYS_TRY(apply_block_t<T>(P, mu_dev, nrhs, R, Z, k, sc.done, sc.alldone, w, s));
  hipLaunchKernelGGL(cg_rz<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, R, Z, w.prz, rpw, sc, par, 0);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_direction<T>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, Z, Pd, sc, 0);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

__global__ void pcg_snapshot_kernel(CgScalars sc, PcgSnap* out, int seq) {
  volatile PcgSnap* o = out;
  o->alldone = *sc.alldone;
  o->iters = sc.iters[0];
  o->status = sc.status[0];
  o->rnorm2 = sc.rnorm2[0];
  o->bnorm2 = sc.bnorm2[0];
  __threadfence_system();
  o->seq = seq;
}

constexpr int64_t kFuseMaxN = 16384;
#ifndef NYS_FINX_BLOCKS
#define NYS_FINX_BLOCKS 512
#endif
#ifndef NYS_FIN_FUSED_BLOCKS
#define NYS_FIN_FUSED_BLOCKS 64  // matvec finish when it also updates x and r (n <= kFuseMaxN)
#endif

nys_status pcg_snapshot(const CgScalars& sc, PcgSnap* out, int seq, hipStream_t s) {
  hipLaunchKernelGGL(pcg_snapshot_kernel, dim3(1), dim3(1), 0, s, sc, out, seq);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status pcg_iteration_fused(int64_t n, const PrecDesc& P, const double* mu_dev, double mu, const T* part,
                               int ng, double scale, T* V, T* X, T* R, T* Z, T* Pd, PcgWork& w,
                               const CgScalars& sc, int par, double tol, hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  const bool fuse = n <= kFuseMaxN;
  const int64_t fmax = fuse ? NYS_FIN_FUSED_BLOCKS : 512;
  const int64_t nfb = cdiv(n, 32) < fmax ? cdiv(n, 32) : fmax;
  hipLaunchKernelGGL(cg_finish_mv<T>, dim3((unsigned)nfb), dim3(NT), 0, s, n, part, ng, scale, mu, Pd,
                     V, w.ppv, sc, par, fuse ? 1 : 0, X, R, w.prr, tol);
  NYS_CHECK_LAUNCH();
  if (!fuse) {
    const int64_t g = groups_for(n, 1);
    hipLaunchKernelGGL(cg_update<T>, dim3((unsigned)g), dim3(NT), 0, s, n, (int64_t)1, Pd, V, X, (int64_t)1, R,
                       w.prr, cdiv(n, g), tol, sc);
    NYS_CHECK_LAUNCH();
  }
  NYS_TRY(utr_launch(P, mu_dev, R, f32, w.apart, w.Cs, sc.ctr + 1, sc.alldone, s));
  if (fuse) return uc_launch(P, w.Cs, R, Z, f32, w.prz, sc, par, 2, s, Pd);
  NYS_TRY(uc_launch(P, w.Cs, R, Z, f32, w.prz, sc, par, 3, s));
  return beta_direction_launch<T>(n, Z, Pd, w, sc, par, s);
}

bool pcg_pvq_ok(const PrecDesc& P, int64_t n) {
  return n <= kFuseMaxN && (P.dtype == NYS_F64 ? uvec_ok<double>(P) : uvec_ok<float>(P));
}

template <typename T>
nys_status pcg_iteration_pvq(int64_t n, const PrecDesc& P, const double* mu_dev, double mu, const T* part, int ng,
                             const double* pvq, int npvq, int npp, double scale, T* V, T* X, T* R, T* Z, T* Pd,
                             PcgWork& w, const CgScalars& sc, int par, double tol, hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  if (!pcg_pvq_ok(P, n)) {
    set_error("pcg_iteration_pvq: needs n <= %lld and a 16-byte U layout", (long long)kFuseMaxN);
    return NYS_ERR_ARG;
  }
  const int64_t l = P.ell;
  // one tile of 32 entries per workgroup (n <= kFuseMaxN keeps it within the
  // partial-sum slots); each also reads its rows of U for U^T r, and nothing
  // here waits on another workgroup
  const int64_t nfb = cdiv(n, 32);
  if (nfb > NYS_FINX_BLOCKS) {
    set_error("pcg_iteration_pvq: n = %lld needs %lld > %d tiles", (long long)n, (long long)nfb, NYS_FINX_BLOCKS);
    return NYS_ERR_ARG;
  }
  const int E = P.dtype == NYS_F64 ? 2 : 4;
  const int nvec = (int)(l / E);
  int G = 1;  // groups of nvec threads sharing the tile's rows
  while (G < 32 && 2 * G * nvec <= NT) G *= 2;
  const bool cg2 = nvec > NT;  // G = 1 and two vectors per thread
#define NYS_FINX(TU, CGV)                                                                                            hipLaunchKernelGGL((cg_finish_pvq<T, TU, CGV>), dim3((unsigned)nfb), dim3(NT), 0, s, n, part, ng, pvq, npvq, npp,                      scale, mu, Pd, V, X, R, static_cast<const TU*>(P.U), l, P.ldu, G, w.apart, w.prr, sc, par)
  if (P.dtype == NYS_F64) {
    if (cg2) NYS_FINX(double, 2);
    else NYS_FINX(double, 1);
  } else {
    if (cg2) NYS_FINX(float, 2);
    else NYS_FINX(float, 1);
  }
#undef NYS_FINX
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(utr_final_rr, dim3((unsigned)cdiv(l, 64)), dim3(NT), 0, s, l, (int)nfb, w.apart, P.lam, mu_dev,
                     w.Cs, w.prr, (int)nfb, sc, tol, w.prz);
  NYS_CHECK_LAUNCH();
  // r^T z from utr_final_rr's parts: the apply also sets the direction, with
  // no workgroup waiting for another
  return uc_launch(P, w.Cs, R, Z, f32, w.prz, sc, par, 4, s, Pd);
}

template <typename T>
nys_status cg_block_init(int64_t n, int64_t k, const T* B, const T* V, T* R, PcgWork& w, const CgScalars& sc,
                         double tol, hipStream_t s) {
  const int64_t ng = groups_for(n, k);
  hipLaunchKernelGGL(cg_init_residual<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, B, V, R, w.pb, w.prr,
                     cdiv(n, ng), tol, sc);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status cg_block_update(int64_t n, int64_t k, const T* V, T* X, T* R, const T* Pd, PcgWork& w,
                           const CgScalars& sc, int par, double tol, hipStream_t s) {
  const int64_t ng = groups_for(n, k);
  const int64_t rpw = cdiv(n, ng);
  hipLaunchKernelGGL(cg_pv_alpha<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, Pd, V, w.ppv, rpw, sc, par);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_update<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, Pd, V, X, k, R, w.prr, rpw, tol,
                     sc);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status cg_block_direction(int64_t n, int64_t k, const T* R, const T* Z, T* Pd, PcgWork& w,
                              const CgScalars& sc, int par, bool init, hipStream_t s) {
  const int64_t ng = groups_for(n, k);
  hipLaunchKernelGGL(cg_rz<T>, dim3((unsigned)ng), dim3(NT), 0, s, n, k, R, Z, w.prz, cdiv(n, ng), sc, par,
                     init ? 1 : 0);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(cg_direction<T>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, Z, Pd, sc,
                     init ? 1 : 0);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template nys_status cg_block_init<float>(int64_t, int64_t, const float*, const float*, float*, PcgWork&,
                                         const CgScalars&, double, hipStream_t);
template nys_status cg_block_init<double>(int64_t, int64_t, const double*, const double*, double*, PcgWork&,
                                          const CgScalars&, double, hipStream_t);
template nys_status cg_block_update<float>(int64_t, int64_t, const float*, float*, float*, const float*, PcgWork&,
                                           const CgScalars&, int, double, hipStream_t);
template nys_status cg_block_update<double>(int64_t, int64_t, const double*, double*, double*, const double*,
                                            PcgWork&, const CgScalars&, int, double, hipStream_t);
template nys_status cg_block_direction<float>(int64_t, int64_t, const float*, const float*, float*, PcgWork&,
                                              const CgScalars&, int, bool, hipStream_t);
template nys_status cg_block_direction<double>(int64_t, int64_t, const double*, const double*, double*,
                                               PcgWork&, const CgScalars&, int, bool, hipStream_t);

template nys_status pcg_iteration_pvq<double>(int64_t, const PrecDesc&, const double*, double, const double*, int,
                                              const double*, int, int, double, double*, double*, double*, double*,
                                              double*, PcgWork&, const CgScalars&, int, double, hipStream_t);
template nys_status pcg_iteration_pvq<float>(int64_t, const PrecDesc&, const double*, double, const float*, int,
                                             const double*, int, int, double, float*, float*, float*, float*, float*,
                                             PcgWork&, const CgScalars&, int, double, hipStream_t);
template nys_status pcg_iteration_fused<double>(int64_t, const PrecDesc&, const double*, double, const double*, int,
                                                double, double*, double*, double*, double*, double*, PcgWork&,
                                                const CgScalars&, int, double, hipStream_t);
template nys_status pcg_iteration_fused<float>(int64_t, const PrecDesc&, const double*, double, const float*, int,
                                               double, float*, float*, float*, float*, float*, PcgWork&,
                                               const CgScalars&, int, double, hipStream_t);

template nys_status pcg_setup<double>(int64_t, int64_t, const PrecDesc&, const double*, int64_t, const double*,
                                      const double*, double*, double*, double*, PcgWork&, const CgScalars&,
                                      double, hipStream_t);
template nys_status pcg_setup<float>(int64_t, int64_t, const PrecDesc&, const double*, int64_t, const float*,
                                     const float*, float*, float*, float*, PcgWork&, const CgScalars&, double,
                                     hipStream_t);
template nys_status pcg_iteration<double>(int64_t, int64_t, const PrecDesc&, const double*, int64_t,
                                          const double*, double*, int64_t, double*, double*, double*, PcgWork&,
                                          const CgScalars&, int, double, hipStream_t);
template nys_status pcg_iteration<float>(int64_t, int64_t, const PrecDesc&, const double*, int64_t, const float*,
                                         float*, int64_t, float*, float*, float*, PcgWork&, const CgScalars&, int,
                                         double, hipStream_t);

}  // namespace nys
