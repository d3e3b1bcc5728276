// Ragged batch of ridge problems (Section 1.3, eq. (RidgeRegression), one
// operator A_c = scale_c X_c^T X_c and one Nystrom preconditioner, eq.
// (NysPre), per problem) solved together by the PCG of Section 5.2.
//
// Problem c is column c of padded n_max x nprob blocks (rows >= n_c stay
// zero), so the CG vector kernels of pcg.hip serve every problem in one
// launch, each column with its own alpha, beta and stopping test.  The two
// problem-specific steps read a device table:
//   * the product v_c = A_c p_c + mu_c p_c: one pass over each X_c (the
//     workgroups are shared out over the problems in proportion to m_c n_c,
//     so one launch streams every X_c once), then a fixed-order sum of the
//     per-workgroup partials;
//   * the apply z_c = r_c + U_c diag((lam_l + mu_c)/(lam + mu_c) - 1) U_c^T r_c.
// Finished problems return at once from both, so an iteration costs only the
// bytes of the problems still iterating.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ragged.hpp"

namespace nys {

namespace {

constexpr int NT = 256;
constexpr int kMaxProb = 256;
constexpr int kMaxN = 8192;
constexpr int kMaxEll = 2048;
constexpr int kGroups = 512;  // partial-sum groups of the CG kernels (matches the block solver)

struct RagProb {
  const void* X;        // m x n, row-major, ld
  int64_t m, n, ld;
  double scale;
  const void* U;        // n x ell, ldu
  int64_t ldu, ell;
  const double* lam;    // ell, descending
  int64_t g0, ng, rpw, poff;           // product: groups [g0, g0 + ng), rows per group, partial offset
  int64_t u0, ncb, nch, rpc, uoff;     // U^T r: groups [u0, u0 + ncb * nch), row chunks, partial offset
  int64_t w0, nw, rpwv, coff;          // U c: groups [w0, w0 + nw), rows per wave, offset of c in Cs
};

// index of the last table entry whose start (field `start`) is <= g
template <int64_t RagProb::*START>
__device__ __forceinline__ int find_prob(const RagProb* tab, int np, int64_t g) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].*START <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// part[poff + gl * n + j] = sum over rows r of this group of (x_r^T p) x_r[j].
// Thread t owns columns v * 256 + t.  Loads use clamped addresses and a mask
// (no divergent branches); R rows are reduced across the 4 waves at a time.
template <typename TD, typename TA, int NV, int R>
__global__ __launch_bounds__(NT) void rag_mv_part(const RagProb* __restrict__ tab, int np, int64_t k,
                                                  const TA* __restrict__ P, TA* __restrict__ part,
                                                  const int* __restrict__ done, const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int c = find_prob<&RagProb::g0>(tab, np, blockIdx.x);
  if (done && done[c]) return;
  const RagProb pb = tab[c];
  const TD* __restrict__ X = static_cast<const TD*>(pb.X);
  const int64_t n = pb.n, ld = pb.ld;
  const int64_t gl = (int64_t)blockIdx.x - pb.g0;
  const int64_t r0 = gl * pb.rpw;
  const int64_t r1 = r0 + pb.rpw < pb.m ? r0 + pb.rpw : pb.m;
  __shared__ TA red[2][4][R];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  TA pr[NV], acc[NV];
  int64_t col[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t j = (int64_t)v * NT + t;
    col[v] = j < n ? j : n - 1;
    pr[v] = j < n ? P[j * k + c] : TA(0);
    acc[v] = TA(0);
  }
  int buf = 0;
  for (int64_t rb = r0; rb < r1; rb += R) {
    TA xr[R][NV];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = rb + r < r1 ? rb + r : r1 - 1;
      const TA rm = rb + r < r1 ? TA(1) : TA(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) xr[r][v] = rm * TA(X[row * ld + col[v]]);
    }
    TA d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      TA s = TA(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) s += xr[r][v] * pr[v];  // pr = 0 on padded columns
      d[r] = wave_sum(s);
    }
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) red[buf][wave][r] = d[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const TA tr = red[buf][0][r] + red[buf][1][r] + red[buf][2][r] + red[buf][3][r];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += tr * xr[r][v];
    }
    buf ^= 1;
  }
  TA* out = part + pb.poff + gl * n;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t j = (int64_t)v * NT + t;
    if (j < n) out[j] = acc[v];
  }
}

// V[i][c] = scale_c sum_g part_c[g][i] + mu_c P[i][c], i < n_c (fixed order over g).
template <typename T, typename TA>
__global__ __launch_bounds__(NT) void rag_mv_finish(const RagProb* __restrict__ tab, int64_t k,
                                                    const TA* __restrict__ part, const T* __restrict__ P,
                                                    const double* __restrict__ mu, T* __restrict__ V,
                                                    const int* __restrict__ done, const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int c = blockIdx.y;
  if (done && done[c]) return;
  const int64_t n = tab[c].n;
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const TA* pp = part + tab[c].poff + i;
  const int64_t ng = tab[c].ng;
  TA a0 = TA(0), a1 = TA(0);
  int64_t g = 0;
  for (; g + 1 < ng; g += 2) {
    a0 += pp[g * n];
    a1 += pp[(g + 1) * n];
  }
  if (g < ng) a0 += pp[g * n];
  const double v = tab[c].scale * double(a0 + a1) + mu[c] * double(P[i * k + c]);
  V[i * k + c] = T(v);
}

// partu[uoff + ch * ell + j] = sum over rows of chunk ch of U[i][j] r_c[i].
// Group = (column block of 64, row chunk); thread (tx, ty): column tx, rows ty (mod 4).
template <typename TU, typename T>
__global__ __launch_bounds__(NT) void rag_utr_part(const RagProb* __restrict__ tab, int np, int64_t k,
                                                   const T* __restrict__ Rv, double* __restrict__ partu,
                                                   const int* __restrict__ done, const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int c = find_prob<&RagProb::u0>(tab, np, blockIdx.x);
  if (done && done[c]) return;
  const RagProb pb = tab[c];
  const TU* __restrict__ U = static_cast<const TU*>(pb.U);
  const int64_t gl = (int64_t)blockIdx.x - pb.u0;
  const int64_t cb = gl % pb.ncb, ch = gl / pb.ncb;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j = cb * 64 + tx;
  const int64_t i0 = ch * pb.rpc;
  const int64_t i1 = i0 + pb.rpc < pb.n ? i0 + pb.rpc : pb.n;
  __shared__ double red[4][64];
  double a0 = 0.0, a1 = 0.0;
  if (j < pb.ell) {
    int64_t i = i0 + ty;
    for (; i + 4 < i1; i += 8) {
      a0 += double(U[i * pb.ldu + j]) * double(Rv[i * k + c]);
      a1 += double(U[(i + 4) * pb.ldu + j]) * double(Rv[(i + 4) * k + c]);
    }
    if (i < i1) a0 += double(U[i * pb.ldu + j]) * double(Rv[i * k + c]);
  }
  red[ty][tx] = a0 + a1;
  __syncthreads();
  if (ty == 0 && j < pb.ell)
    partu[pb.uoff + ch * pb.ell + j] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// Cs[coff + j] = ((lam_l + mu_c)/(lam_j + mu_c) - 1) sum_ch partu[ch][j]  (fixed order)
__global__ __launch_bounds__(NT) void rag_utr_finish(const RagProb* __restrict__ tab,
                                                     const double* __restrict__ partu, const double* __restrict__ mu,
                                                     double* __restrict__ Cs, const int* __restrict__ done,
                                                     const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int c = blockIdx.y;
  if (done && done[c]) return;
  const int64_t ell = tab[c].ell;
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= ell) return;
  const double* pp = partu + tab[c].uoff + j;
  double a0 = 0.0, a1 = 0.0;
  int64_t q = 0;
  const int64_t nch = tab[c].nch;
  for (; q + 1 < nch; q += 2) {
    a0 += pp[q * ell];
    a1 += pp[(q + 1) * ell];
  }
  if (q < nch) a0 += pp[q * ell];
  const double* lam = tab[c].lam;
  const double m = mu[c];
  Cs[tab[c].coff + j] = ((lam[ell - 1] + m) / (lam[j] + m) - 1.0) * (a0 + a1);
}

// Z[i][c] = R[i][c] + sum_j U_c[i][j] Cs_c[j]; one wave per row, four rows at once.
template <typename TU, typename T>
__global__ __launch_bounds__(NT) void rag_uc(const RagProb* __restrict__ tab, int np, int64_t k,
                                             const double* __restrict__ Cs, const T* __restrict__ Rv,
                                             T* __restrict__ Z, const int* __restrict__ done,
                                             const int* __restrict__ alldone) {
  if (alldone && *alldone) return;
  const int c = find_prob<&RagProb::w0>(tab, np, blockIdx.x);
  if (done && done[c]) return;
  const RagProb pb = tab[c];
  const TU* __restrict__ U = static_cast<const TU*>(pb.U);
  __shared__ T cs[kMaxEll];
  for (int64_t j = threadIdx.x; j < pb.ell; j += NT) cs[j] = T(Cs[pb.coff + j]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t w = ((int64_t)blockIdx.x - pb.w0) * 4 + wave;
  const int64_t i0 = w * pb.rpwv;
  const int64_t i1 = i0 + pb.rpwv < pb.n ? i0 + pb.rpwv : pb.n;
  for (int64_t ib = i0; ib < i1; ib += 4) {
    const int64_t nr = (i1 - ib) < 4 ? (i1 - ib) : 4;
    T s[4] = {T(0), T(0), T(0), T(0)};
    for (int64_t j = lane; j < pb.ell; j += 64) {
      const T cj = cs[j];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nr) s[q] += T(U[(ib + q) * pb.ldu + j]) * cj;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = wave_sum(s[q]);
    if (lane < nr) {
      const int64_t i = ib + lane;
      const T sq = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
      Z[i * k + c] = Rv[i * k + c] + sq;
    }
  }
}

// dst[i][c] = src_c[i] (i < n_c), zero on the padded rows
template <typename TS, typename TD>
__global__ void rag_pack(const RagProb* __restrict__ tab, int64_t k, int64_t nmax, const TS* const* __restrict__ src,
                         TD* __restrict__ dst) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= nmax) return;
  dst[i * k + c] = i < tab[c].n ? TD(src[c][i]) : TD(0);
}

// dst_c[i] = src[i][c] for i < n_c
__global__ void rag_unpack(const RagProb* __restrict__ tab, int64_t k, const double* __restrict__ src,
                           double* const* __restrict__ dst) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= tab[c].n) return;
  dst[c][i] = src[i * k + c];
}

// per-column ||R||^2 and ||B||^2 partials over row groups (k <= 256 columns):
// part[g][c] and part[G + g][c]; R = B - V
__global__ __launch_bounds__(NT) void rag_residual(int64_t n, int64_t k, const double* __restrict__ B,
                                                   const double* __restrict__ V, double* __restrict__ R,
                                                   double* __restrict__ part) {
  const int c = threadIdx.x;
  const int64_t rows = cdiv(n, (int64_t)gridDim.x);
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  if (c >= k) return;
  double sr = 0.0, sb = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double b = B[i * k + c];
    const double r = b - V[i * k + c];
    R[i * k + c] = r;
    sr += r * r;
    sb += b * b;
  }
  part[(int64_t)blockIdx.x * k + c] = sr;
  part[((int64_t)gridDim.x + blockIdx.x) * k + c] = sb;
}

// f32/f64 copy of R into B with the columns that are already converged zeroed
template <typename T>
__global__ void rag_masked_copy(int64_t count, int64_t k, const double* __restrict__ R,
                                const int* __restrict__ active, T* __restrict__ dst) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= count) return;
  dst[idx] = active[idx % k] ? T(R[idx]) : T(0);
}

template <typename TS>
__global__ void rag_add(int64_t count, double* __restrict__ dst, const TS* __restrict__ src) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx < count) dst[idx] += double(src[idx]);
}

template <typename T>
__global__ void rag_zero(int64_t count, T* __restrict__ p) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx < count) p[idx] = T(0);
}

struct IntList {
  int v[kMaxProb];
};

__global__ void rag_set_ints(int* __restrict__ dst, int64_t count, IntList l) {
  if ((int64_t)threadIdx.x < count) dst[threadIdx.x] = l.v[threadIdx.x];
}

// ---- device-info form: tables set by value, every decision on the device

constexpr int kTabChunk = 8;  // problems per table upload (kernel argument size, ~1.6 KB)

struct TabChunk {
  RagProb tab[kTabChunk];
  double mu[kTabChunk];
  const double* bsrc[kTabChunk];
  double* xdst[kTabChunk];
};

__global__ void rag_set_tab(TabChunk c, int first, int count, RagProb* __restrict__ tab, double* __restrict__ mu,
                            const double** __restrict__ bsrc, double** __restrict__ xdst) {
  const int i = threadIdx.x;
  if (i >= count) return;
  tab[first + i] = c.tab[i];
  mu[first + i] = c.mu[i];
  bsrc[first + i] = c.bsrc[i];
  xdst[first + i] = c.xdst[i];
}

// relres[c] from the rag_residual partials (groups summed in order)
__global__ void rag_relres(int64_t k, int ng, const double* __restrict__ part, double* __restrict__ relres) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double rr = 0.0, bb = 0.0;
  for (int q = 0; q < ng; ++q) {
    rr += part[(int64_t)q * k + c];
    bb += part[(int64_t)(ng + q) * k + c];
  }
  relres[c] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

__global__ void rag_state_init(int64_t k, double* __restrict__ prev, int* __restrict__ iters, int* __restrict__ brk) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  prev[c] = __builtin_huge_val();
  iters[c] = 0;
  brk[c] = 0;
}

// a problem is refined while its true residual exceeds tol, it has not
// broken down and the last step at least halved its residual; prev <- relres
__global__ void rag_select(int64_t k, const double* __restrict__ relres, double* __restrict__ prev,
                           const int* __restrict__ brk, int* __restrict__ active, double tol) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const double r = relres[c];
  active[c] = (!brk[c] && !(r <= tol) && r <= 0.5 * prev[c]) ? 1 : 0;
  prev[c] = r;
}

// inner iterations and breakdowns of the active problems added to the totals
__global__ void rag_count(int64_t k, CgScalars sc, const int* __restrict__ active, int* __restrict__ iters,
                          int* __restrict__ brk) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k || !active[c]) return;
  iters[c] += sc.iters[c];
  if (sc.status[c] == NYS_ERR_BREAKDOWN) brk[c] = 1;
}

// float64 form: the inner solve on r = b - A x0 stops at ||r_inner|| <= tol ||b||
// (the outer test), so its reference norm is ||b||^2 from the residual partials
__global__ void rag_bnorm_from_parts(int64_t k, int ng, const double* __restrict__ part, CgScalars sc, double tol) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double bb = 0.0;
  for (int q = 0; q < ng; ++q) bb += part[(int64_t)(ng + q) * k + c];
  sc.bnorm2[c] = bb;
  const bool conv = sc.rnorm2[c] <= tol * tol * bb;
  sc.done[c] = conv ? 1 : 0;
  sc.conv[c] = conv ? 1 : 0;
  sc.status[c] = conv ? NYS_OK : NYS_NOT_CONVERGED;
}

// all-done flag after the flags above changed
__global__ void rag_alldone(int64_t k, CgScalars sc) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int64_t c = threadIdx.x; c < k; c += blockDim.x)
    if (!sc.done[c]) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) *sc.alldone = any ? 0 : 1;
}

__global__ void rag_write_info(int64_t k, const int* __restrict__ iters, const int* __restrict__ brk,
                               const double* __restrict__ relres, double tol, int32_t* __restrict__ o_iters,
                               double* __restrict__ o_relres, int32_t* __restrict__ o_status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const double r = relres[c];
  if (o_iters) o_iters[c] = iters[c];
  if (o_relres) o_relres[c] = r;
  if (o_status) o_status[c] = brk[c] ? NYS_ERR_BREAKDOWN : (r <= tol ? NYS_OK : NYS_NOT_CONVERGED);
}

unsigned nb256(int64_t count) { return (unsigned)(count > 0 ? cdiv(count, (int64_t)NT) : 1); }

// ---------------------------------------------------------------- host side

struct Plan {
  std::vector<RagProb> tab;
  int np = 0;
  int64_t nmax = 0, ellmax = 0;
  int64_t g_mv = 0, g_utr = 0, g_uc = 0;
  size_t part_elems = 0, partu_elems = 0, cs_elems = 0;
  bool f64_data = false, f64_u = false;
};

Plan make_plan(const OpDesc* ops, const PrecDesc* pds, int np, const int cus) {
  Plan p;
  p.np = np;
  p.f64_data = ops[0].dtype == NYS_F64;
  p.f64_u = pds[0].dtype == NYS_F64;
  double wmv = 0.0, wu = 0.0;
  for (int c = 0; c < np; ++c) {
    p.nmax = std::max(p.nmax, ops[c].n);
    p.ellmax = std::max(p.ellmax, pds[c].ell);
    wmv += double(ops[c].rows) * double(ops[c].n);
    wu += double(ops[c].n) * double(pds[c].ell);
  }
  const double target = 4.0 * cus;  // about four groups per compute unit per launch
  int64_t g = 0, u = 0, w = 0;
  size_t po = 0, uo = 0, co = 0;
  p.tab.resize(np);
  for (int c = 0; c < np; ++c) {
    RagProb& t = p.tab[c];
    const OpDesc& op = ops[c];
    const PrecDesc& pd = pds[c];
    t.X = op.data;
    t.m = op.rows;
    t.n = op.n;
    t.ld = op.ld;
    t.scale = op.scale;
    t.U = pd.U;
    t.ldu = pd.ldu;
    t.ell = pd.ell;
    t.lam = pd.lam;
    // product groups in proportion to m n (rows per group a multiple of 4)
    int64_t ng = (int64_t)std::llround(target * double(op.rows) * double(op.n) / wmv);
    ng = std::max<int64_t>(1, std::min<int64_t>(ng, cdiv(op.rows, (int64_t)4)));
    t.rpw = cdiv(cdiv(op.rows, ng), (int64_t)4) * 4;
    t.ng = cdiv(op.rows, t.rpw);
    t.g0 = g;
    t.poff = (int64_t)po;
    g += t.ng;
    po += (size_t)t.ng * (size_t)op.n;
    // U^T r groups: 64 columns x row chunks of >= 64 rows
    t.ncb = cdiv(pd.ell, (int64_t)64);
    int64_t nch = (int64_t)std::llround(target * double(op.n) * double(pd.ell) / wu / double(t.ncb));
    nch = std::max<int64_t>(1, std::min<int64_t>(nch, cdiv(op.n, (int64_t)64)));
    t.rpc = cdiv(op.n, nch);
    t.nch = cdiv(op.n, t.rpc);
    t.u0 = u;
    t.uoff = (int64_t)uo;
    u += t.ncb * t.nch;
    uo += (size_t)t.nch * (size_t)pd.ell;
    // U c groups: 4 waves each, rows per wave a multiple of 4
    int64_t waves = (int64_t)std::llround(4.0 * target * double(op.n) * double(pd.ell) / wu);
    waves = std::max<int64_t>(4, std::min<int64_t>(waves, cdiv(op.n, (int64_t)4)));
    t.rpwv = cdiv(cdiv(op.n, waves), (int64_t)4) * 4;
    t.nw = cdiv(cdiv(op.n, t.rpwv), (int64_t)4);
    t.w0 = w;
    w += t.nw;
    t.coff = (int64_t)co;
    co += (size_t)pd.ell;
  }
  p.g_mv = g;
  p.g_utr = u;
  p.g_uc = w;
  p.part_elems = po;
  p.partu_elems = uo;
  p.cs_elems = co;
  return p;
}

template <typename T>
struct RagBufs {
  T *V, *R, *Z, *P, *X, *B;
  PcgWork w;
  CgScalars sc;
};

struct RagWs {
  RagProb* tab;
  double* mu;
  int* active;
  double *relres_d, *prev_d;  // device-info form
  int *iters_d, *brk_d;
  double *B64, *X64, *R64, *V64, *dots;
  double *part, *partu, *Cs;
  const double** bsrc;
  double** xdst;
  RagBufs<double> d;
  RagBufs<float> f;
  bool has_f;
};

template <typename T>
void carve_rag_bufs(Arena& a, int64_t nk, int64_t k, RagBufs<T>& b) {
  b.V = a.take<T>(nk);
  b.R = a.take<T>(nk);
  b.Z = a.take<T>(nk);
  b.P = a.take<T>(nk);
  b.X = a.take<T>(nk);
  b.B = a.take<T>(nk);
  b.w.pb = a.take<double>(kGroups * k);
  b.w.prr = a.take<double>(kGroups * k);
  b.w.ppv = a.take<double>(kGroups * k);
  b.w.prz = a.take<double>(kGroups * k);
  b.w.apart = nullptr;
  b.w.apart_elems = 0;
  b.w.Cs = b.w.Ct = nullptr;
  b.sc.rz = a.take<double>(2 * k);
  b.sc.bnorm2 = a.take<double>(k);
  b.sc.rnorm2 = a.take<double>(k);
  b.sc.alpha = a.take<double>(k);
  b.sc.beta = a.take<double>(k);
  b.sc.done = a.take<int>(k);
  b.sc.conv = a.take<int>(k);
  b.sc.iters = a.take<int>(k);
  b.sc.status = a.take<int>(k);
  b.sc.alldone = a.take<int>(1);
  b.sc.ctr = a.take<unsigned>(64);
}

void carve_rag(Arena& a, const Plan& p, int prec, RagWs& w) {
  const int64_t k = p.np, nk = p.nmax * k;
  w.tab = a.take<RagProb>(k);
  w.mu = a.take<double>(k);
  w.active = a.take<int>(k);
  w.relres_d = a.take<double>(k);
  w.prev_d = a.take<double>(k);
  w.iters_d = a.take<int>(k);
  w.brk_d = a.take<int>(k);
  w.bsrc = a.take<const double*>(k);
  w.xdst = a.take<double*>(k);
  w.B64 = a.take<double>(nk);
  w.X64 = a.take<double>(nk);
  w.R64 = a.take<double>(nk);
  w.V64 = a.take<double>(nk);
  w.dots = a.take<double>(2 * 64 * k);
  w.part = a.take<double>(p.part_elems);
  w.partu = a.take<double>(p.partu_elems);
  w.Cs = a.take<double>(p.cs_elems);
  carve_rag_bufs<double>(a, nk, k, w.d);
  w.has_f = prec != NYS_PREC_FP64;
  if (w.has_f) carve_rag_bufs<float>(a, nk, k, w.f);
}

template <typename TD, typename TA>
nys_status launch_mv_part(const Plan& p, const RagProb* tab, const TA* P, TA* part, const int* done,
                          const int* alldone, hipStream_t s) {
  const int64_t k = p.np;
  const int nv = (int)cdiv(p.nmax, (int64_t)NT);
#define RMV(NV, R) hipLaunchKernelGGL((rag_mv_part<TD, TA, NV, R>), dim3((unsigned)p.g_mv), dim3(NT), 0, s, tab, p.np, k, P, part, done, alldone)
  if (nv <= 4) RMV(4, 4);
  else if (nv <= 8) RMV(8, 4);
  else if (nv <= 16) RMV(16, 2);
  else if (nv <= 24) RMV(24, 2);
  else RMV(32, 1);
#undef RMV
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// V = A P + mu P for every problem (TA: accumulation type of the product)
template <typename T, typename TA>
nys_status rag_matvec(const Plan& p, RagWs& w, const T* P, T* V, const int* done, const int* alldone,
                      hipStream_t s) {
  TA* part = reinterpret_cast<TA*>(w.part);
  if (p.f64_data) NYS_TRY((launch_mv_part<double, TA>(p, w.tab, P, part, done, alldone, s)));
  else NYS_TRY((launch_mv_part<float, TA>(p, w.tab, P, part, done, alldone, s)));
  hipLaunchKernelGGL((rag_mv_finish<T, TA>), dim3(nb256(p.nmax), (unsigned)p.np), dim3(NT), 0, s, w.tab,
                     (int64_t)p.np, part, P, w.mu, V, done, alldone);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status rag_apply(const Plan& p, RagWs& w, const T* Rv, T* Z, const int* done, const int* alldone,
                     hipStream_t s) {
  const int64_t k = p.np;
  if (p.f64_u)
    hipLaunchKernelGGL((rag_utr_part<double, T>), dim3((unsigned)p.g_utr), dim3(NT), 0, s, w.tab, p.np, k, Rv,
                       w.partu, done, alldone);
  else
    hipLaunchKernelGGL((rag_utr_part<float, T>), dim3((unsigned)p.g_utr), dim3(NT), 0, s, w.tab, p.np, k, Rv,
                       w.partu, done, alldone);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(rag_utr_finish, dim3(nb256(p.ellmax), (unsigned)p.np), dim3(NT), 0, s, w.tab, w.partu, w.mu,
                     w.Cs, done, alldone);
  NYS_CHECK_LAUNCH();
  if (p.f64_u)
    hipLaunchKernelGGL((rag_uc<double, T>), dim3((unsigned)p.g_uc), dim3(NT), 0, s, w.tab, p.np, k, w.Cs, Rv, Z,
                       done, alldone);
  else
    hipLaunchKernelGGL((rag_uc<float, T>), dim3((unsigned)p.g_uc), dim3(NT), 0, s, w.tab, p.np, k, w.Cs, Rv, Z,
                       done, alldone);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

struct RagResult {
  std::vector<int> iters, status;
  int sweeps = 0;
};

// PCG on every column of the padded block B (x0 = 0), result in b.X.
template <typename T>
nys_status rag_pcg(const Plan& p, RagWs& w, RagBufs<T>& b, double tol, int maxit, int check_every,
                   RagResult& res, hipStream_t s) {
  const int64_t k = p.np, n = p.nmax, nk = n * k;
  NYS_HIP(hipMemsetAsync(b.sc.ctr, 0, sizeof(unsigned) * 64, s));
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.X);
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.V);
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.Z);
  NYS_CHECK_LAUNCH();
  NYS_TRY(cg_block_init<T>(n, k, b.B, b.V, b.R, b.w, b.sc, tol, s));
  NYS_TRY(rag_apply<T>(p, w, b.R, b.Z, nullptr, nullptr, s));
  NYS_TRY(cg_block_direction<T>(n, k, b.R, b.Z, b.P, b.w, b.sc, 0, true, s));
  int alldone_h = 0;
  NYS_HIP(hipMemcpyAsync(&alldone_h, b.sc.alldone, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  const int interval = check_every > 0 ? check_every : 8;
  int it = 0;
  while (!alldone_h && it < maxit) {
    const int par = it & 1;
    NYS_TRY((rag_matvec<T, T>(p, w, b.P, b.V, b.sc.done, b.sc.alldone, s)));
    NYS_TRY(cg_block_update<T>(n, k, b.V, b.X, b.R, b.P, b.w, b.sc, par, tol, s));
    NYS_TRY(rag_apply<T>(p, w, b.R, b.Z, b.sc.done, b.sc.alldone, s));
    NYS_TRY(cg_block_direction<T>(n, k, b.R, b.Z, b.P, b.w, b.sc, par, false, s));
    ++it;
    if (it % interval == 0 || it == maxit) {
      NYS_HIP(hipMemcpyAsync(&alldone_h, b.sc.alldone, sizeof(int), hipMemcpyDeviceToHost, s));
      NYS_HIP(hipStreamSynchronize(s));
    }
  }
  res.iters.assign(k, 0);
  res.status.assign(k, 0);
  NYS_HIP(hipMemcpyAsync(res.iters.data(), b.sc.iters, sizeof(int) * k, hipMemcpyDeviceToHost, s));
  NYS_HIP(hipMemcpyAsync(res.status.data(), b.sc.status, sizeof(int) * k, hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  res.sweeps = it;
  return NYS_OK;
}

// R64 = B64 - (A + mu I) X64 in float64; relative residual per problem
nys_status rag_true_residual(const Plan& p, RagWs& w, std::vector<double>& relres, hipStream_t s) {
  const int64_t k = p.np, n = p.nmax;
  NYS_TRY((rag_matvec<double, double>(p, w, w.X64, w.V64, nullptr, nullptr, s)));
  const int g = 64;
  hipLaunchKernelGGL(rag_residual, dim3(g), dim3(NT), 0, s, n, k, w.B64, w.V64, w.R64, w.dots);
  NYS_CHECK_LAUNCH();
  std::vector<double> h(2 * g * k);
  NYS_HIP(hipMemcpyAsync(h.data(), w.dots, sizeof(double) * 2 * g * k, hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  relres.assign(k, 0.0);
  for (int64_t c = 0; c < k; ++c) {
    double rr = 0.0, bb = 0.0;
    for (int q = 0; q < g; ++q) {
      rr += h[q * k + c];
      bb += h[(g + q) * k + c];
    }
    relres[c] = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  }
  return NYS_OK;
}

// One correction step on the columns with active[c] != 0: solve (A + mu I) d = r
// (r from R64) to the relative tolerance itol in arithmetic T, then X64 += d.
template <typename T>
nys_status rag_correct(const Plan& p, RagWs& w, RagBufs<T>& b, const std::vector<int>& active, double itol,
                       int maxit, int check, RagResult& r, hipStream_t s) {
  const int64_t k = p.np, nk = p.nmax * k;
  IntList l{};
  for (int64_t c = 0; c < k; ++c) l.v[c] = active[c];
  hipLaunchKernelGGL(rag_set_ints, dim3(1), dim3(kMaxProb), 0, s, w.active, k, l);
  hipLaunchKernelGGL((rag_masked_copy<T>), dim3(nb256(nk)), dim3(NT), 0, s, nk, k, w.R64, w.active, b.B);
  NYS_CHECK_LAUNCH();
  NYS_TRY(rag_pcg<T>(p, w, b, itol, maxit, check, r, s));
  hipLaunchKernelGGL((rag_add<T>), dim3(nb256(nk)), dim3(NT), 0, s, nk, w.X64, b.X);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Device-info PCG: exactly maxit iterations on every column (stopped
// columns are frozen by their flags, finished problems skip the products).
// bnorm_parts (float64 form): stopping test against ||b|| instead of the
// inner right-hand side.
template <typename T>
nys_status rag_pcg_dev(const Plan& p, RagWs& w, RagBufs<T>& b, double tol, int maxit, const double* bnorm_parts,
                       int ng, hipStream_t s) {
  const int64_t k = p.np, n = p.nmax, nk = n * k;
  hipLaunchKernelGGL(rag_zero<unsigned>, dim3(1), dim3(NT), 0, s, (int64_t)64, b.sc.ctr);
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.X);
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.V);
  hipLaunchKernelGGL(rag_zero<T>, dim3(nb256(nk)), dim3(NT), 0, s, nk, b.Z);
  NYS_CHECK_LAUNCH();
  NYS_TRY(cg_block_init<T>(n, k, b.B, b.V, b.R, b.w, b.sc, tol, s));
  if (bnorm_parts) {
    hipLaunchKernelGGL(rag_bnorm_from_parts, dim3(nb256(k)), dim3(NT), 0, s, k, ng, bnorm_parts, b.sc, tol);
    hipLaunchKernelGGL(rag_alldone, dim3(1), dim3(NT), 0, s, k, b.sc);
    NYS_CHECK_LAUNCH();
  }
  NYS_TRY(rag_apply<T>(p, w, b.R, b.Z, nullptr, nullptr, s));
  NYS_TRY(cg_block_direction<T>(n, k, b.R, b.Z, b.P, b.w, b.sc, 0, true, s));
  for (int it = 0; it < maxit; ++it) {
    const int par = it & 1;
    NYS_TRY((rag_matvec<T, T>(p, w, b.P, b.V, b.sc.done, b.sc.alldone, s)));
    NYS_TRY(cg_block_update<T>(n, k, b.V, b.X, b.R, b.P, b.w, b.sc, par, tol, s));
    NYS_TRY(rag_apply<T>(p, w, b.R, b.Z, b.sc.done, b.sc.alldone, s));
    NYS_TRY(cg_block_direction<T>(n, k, b.R, b.Z, b.P, b.w, b.sc, par, false, s));
  }
  return NYS_OK;
}

// R64 = B64 - (A + mu I) X64 and relres_d on the device
nys_status rag_true_residual_dev(const Plan& p, RagWs& w, hipStream_t s) {
  const int64_t k = p.np, n = p.nmax;
  NYS_TRY((rag_matvec<double, double>(p, w, w.X64, w.V64, nullptr, nullptr, s)));
  const int g = 64;
  hipLaunchKernelGGL(rag_residual, dim3(g), dim3(NT), 0, s, n, k, w.B64, w.V64, w.R64, w.dots);
  hipLaunchKernelGGL(rag_relres, dim3(nb256(k)), dim3(NT), 0, s, k, g, w.dots, w.relres_d);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

nys_status ragged_solve_device(const Plan& p, const double* mu, const double* const* B, double* const* X,
                               const nys_solve_opts* o, nys_solve_info* info, RagWs& w, hipStream_t s) {
  const int64_t k = p.np, nk = p.nmax * k;
  const double tol = o->tol;
  const int maxit = o->maxit > 0 ? o->maxit : 500;
  // problem table, mu and vector pointers by value (no host-to-device copy)
  for (int64_t c0 = 0; c0 < k; c0 += kTabChunk) {
    TabChunk ch{};
    const int cnt = (int)std::min<int64_t>(kTabChunk, k - c0);
    for (int i = 0; i < cnt; ++i) {
      ch.tab[i] = p.tab[c0 + i];
      ch.mu[i] = mu[c0 + i];
      ch.bsrc[i] = B[c0 + i];
      ch.xdst[i] = X[c0 + i];
    }
    hipLaunchKernelGGL(rag_set_tab, dim3(1), dim3(kTabChunk), 0, s, ch, (int)c0, cnt, w.tab, w.mu, w.bsrc, w.xdst);
    NYS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(rag_zero<double>, dim3(nb256(nk)), dim3(NT), 0, s, nk, w.V64);
  hipLaunchKernelGGL(rag_zero<double>, dim3(nb256(nk)), dim3(NT), 0, s, nk, w.R64);
  hipLaunchKernelGGL((rag_pack<double, double>), dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, p.nmax,
                     w.bsrc, w.B64);
  hipLaunchKernelGGL((rag_pack<double, double>), dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, p.nmax,
                     (const double* const*)w.xdst, w.X64);
  hipLaunchKernelGGL(rag_state_init, dim3(nb256(k)), dim3(NT), 0, s, k, w.prev_d, w.iters_d, w.brk_d);
  NYS_CHECK_LAUNCH();
  NYS_TRY(rag_true_residual_dev(p, w, s));
  const bool f64 = o->prec == NYS_PREC_FP64;
  const int steps = f64 ? 1 : (o->max_refine > 0 ? o->max_refine : 10);
  const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
  for (int step = 0; step < steps; ++step) {
    hipLaunchKernelGGL(rag_select, dim3(nb256(k)), dim3(NT), 0, s, k, w.relres_d, w.prev_d, w.brk_d, w.active, tol);
    NYS_CHECK_LAUNCH();
    if (f64) {
      hipLaunchKernelGGL((rag_masked_copy<double>), dim3(nb256(nk)), dim3(NT), 0, s, nk, k, w.R64, w.active, w.d.B);
      NYS_CHECK_LAUNCH();
      NYS_TRY(rag_pcg_dev<double>(p, w, w.d, tol, maxit, w.dots, 64, s));
      hipLaunchKernelGGL((rag_add<double>), dim3(nb256(nk)), dim3(NT), 0, s, nk, w.X64, w.d.X);
      hipLaunchKernelGGL(rag_count, dim3(nb256(k)), dim3(NT), 0, s, k, w.d.sc, w.active, w.iters_d, w.brk_d);
    } else {
      hipLaunchKernelGGL((rag_masked_copy<float>), dim3(nb256(nk)), dim3(NT), 0, s, nk, k, w.R64, w.active, w.f.B);
      NYS_CHECK_LAUNCH();
      NYS_TRY(rag_pcg_dev<float>(p, w, w.f, itol, maxit, nullptr, 0, s));
      hipLaunchKernelGGL((rag_add<float>), dim3(nb256(nk)), dim3(NT), 0, s, nk, w.X64, w.f.X);
      hipLaunchKernelGGL(rag_count, dim3(nb256(k)), dim3(NT), 0, s, k, w.f.sc, w.active, w.iters_d, w.brk_d);
    }
    NYS_CHECK_LAUNCH();
    NYS_TRY(rag_true_residual_dev(p, w, s));
  }
  hipLaunchKernelGGL(rag_write_info, dim3(nb256(k)), dim3(NT), 0, s, k, w.iters_d, w.brk_d, w.relres_d, tol,
                     info ? info->iters : nullptr, info ? info->relres : nullptr, info ? info->status : nullptr);
  hipLaunchKernelGGL(rag_unpack, dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, w.X64, w.xdst);
  NYS_CHECK_LAUNCH();
  if (info) {
    info->refine_steps = f64 ? 0 : steps;
    info->total_iters = steps * maxit;
  }
  return NYS_OK;
}

}  // namespace

bool ragged_supported(const OpDesc* ops, const PrecDesc* pds, int nprob) {
  if (nprob < 1 || nprob > kMaxProb) return false;
  for (int c = 0; c < nprob; ++c) {
    if (ops[c].kind != NYS_OP_XTX || ops[c].dtype != ops[0].dtype || pds[c].dtype != pds[0].dtype) return false;
    if (ops[c].w != nullptr) return false;  // weighted operators: one solve after the other
    if (ops[c].n > kMaxN || pds[c].ell > kMaxEll || pds[c].n != ops[c].n) return false;
  }
  return true;
}

size_t ragged_workspace(const OpDesc* ops, const PrecDesc* pds, int nprob, int prec) {
  const Plan p = make_plan(ops, pds, nprob, num_cus());
  Arena a(nullptr, 0);
  RagWs w;
  carve_rag(a, p, prec, w);
  return a.off + 256;
}

nys_status ragged_solve(const OpDesc* ops, const PrecDesc* pds, const double* mu, const double* const* B,
                        double* const* X, int nprob, const nys_solve_opts* o, nys_solve_info* info, void* ws,
                        size_t ws_bytes, hipStream_t s) {
  const Plan p = make_plan(ops, pds, nprob, num_cus());
  Arena a(ws, ws_bytes);
  RagWs w;
  carve_rag(a, p, o->prec, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  if (o->device_info) return ragged_solve_device(p, mu, B, X, o, info, w, s);
  const int64_t k = nprob, nk = p.nmax * k;
  const double tol = o->tol;
  const int maxit = o->maxit > 0 ? o->maxit : 500;
  const int check = o->check_every;
  // problem table, mu and the vector pointers (synchronised once: host staging is released after)
  NYS_HIP(hipMemcpyAsync(w.tab, p.tab.data(), sizeof(RagProb) * k, hipMemcpyHostToDevice, s));
  NYS_HIP(hipMemcpyAsync(w.mu, mu, sizeof(double) * k, hipMemcpyHostToDevice, s));
  NYS_HIP(hipMemcpyAsync(w.bsrc, B, sizeof(double*) * k, hipMemcpyHostToDevice, s));
  NYS_HIP(hipMemcpyAsync(w.xdst, X, sizeof(double*) * k, hipMemcpyHostToDevice, s));
  NYS_HIP(hipStreamSynchronize(s));
  // the product kernels write rows < n_c only: the padded rows of V64 (and so
  // of every residual) must start, and stay, at zero
  hipLaunchKernelGGL(rag_zero<double>, dim3(nb256(nk)), dim3(NT), 0, s, nk, w.V64);
  hipLaunchKernelGGL(rag_zero<double>, dim3(nb256(nk)), dim3(NT), 0, s, nk, w.R64);
  hipLaunchKernelGGL((rag_pack<double, double>), dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, p.nmax,
                     w.bsrc, w.B64);
  hipLaunchKernelGGL((rag_pack<double, double>), dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, p.nmax,
                     (const double* const*)w.xdst, w.X64);
  NYS_CHECK_LAUNCH();
  std::vector<int> iters(k, 0), status(k, NYS_NOT_CONVERGED);
  std::vector<double> relres;
  int total = 0, refine = 0;
  NYS_TRY(rag_true_residual(p, w, relres, s));
  const bool f64 = o->prec == NYS_PREC_FP64;
  const int max_steps = f64 ? 4 : (o->max_refine > 0 ? o->max_refine : 10);
  const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
  std::vector<double> prev(relres);
  for (int step = 0; step < max_steps; ++step) {
    std::vector<int> act(k, 0);
    double worst = 0.0;
    int nact = 0;
    for (int64_t c = 0; c < k; ++c)
      // as in the single solve: stop refining a problem whose residual grew or stalled
      if (!(relres[c] <= tol) && status[c] != NYS_ERR_BREAKDOWN && (step == 0 || relres[c] <= 0.5 * prev[c])) {
        act[c] = 1;
        ++nact;
        worst = std::max(worst, relres[c]);
      }
    if (nact == 0 || !std::isfinite(worst)) break;
    prev = relres;
    RagResult r;
    if (f64) {
      // first pass: the solve itself (tol relative to b, as the residual is b
      // while X = x0 = 0); later passes correct residual drift
      const double t = step == 0 ? tol / std::max(worst, 1e-300) : 0.5 * tol / worst;
      NYS_TRY(rag_correct<double>(p, w, w.d, act, std::min(t, 0.5), maxit, check, r, s));
    } else {
      NYS_TRY(rag_correct<float>(p, w, w.f, act, itol, maxit, check, r, s));
    }
    for (int64_t c = 0; c < k; ++c)
      if (act[c]) {
        iters[c] += r.iters[c];
        if (r.status[c] == NYS_ERR_BREAKDOWN) status[c] = NYS_ERR_BREAKDOWN;
      }
    total += r.sweeps;
    ++refine;
    NYS_TRY(rag_true_residual(p, w, relres, s));
  }
  for (int64_t c = 0; c < k; ++c)
    if (status[c] != NYS_ERR_BREAKDOWN) status[c] = relres[c] <= tol ? NYS_OK : NYS_NOT_CONVERGED;
  hipLaunchKernelGGL(rag_unpack, dim3(nb256(p.nmax), (unsigned)k), dim3(NT), 0, s, w.tab, k, w.X64, w.xdst);
  NYS_CHECK_LAUNCH();
  NYS_HIP(hipStreamSynchronize(s));
  nys_status worst = NYS_OK;
  for (int64_t c = 0; c < k; ++c) {
    if (status[c] == NYS_ERR_BREAKDOWN) worst = NYS_ERR_BREAKDOWN;
    else if (status[c] != NYS_OK && worst == NYS_OK) worst = NYS_NOT_CONVERGED;
  }
  if (info) {
    for (int64_t c = 0; c < k; ++c) {
      if (info->iters) info->iters[c] = iters[c];
      if (info->relres) info->relres[c] = relres[c];
      if (info->status) info->status[c] = status[c];
    }
    info->refine_steps = f64 ? 0 : refine;
    info->total_iters = total;
  }
  if (worst == NYS_ERR_BREAKDOWN) set_error("PCG breakdown: p^T (A + mu I) p <= 0");
  else if (worst == NYS_NOT_CONVERGED) set_error("PCG did not reach the tolerance within maxit");
  return worst;
}

}  // namespace nys
