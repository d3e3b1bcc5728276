// Operator products V = A P for the three operator forms (Section 1.1: A is
// touched only through products), gfx950.
//
//  * dense    : row-per-wave GEMV (k = 1) or the MFMA GEMM (k > 1)
//  * X^T X    : one pass over X per single-vector product (xtx.hip); MFMA
//               GEMMs X^T (X P) for blocks of columns
//  * RBF      : K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) evaluated tile by
//               tile and never stored (Section 6.5 kernel ridge regression).
//               float64 forms, both with the Gram on v_mfma_f64_16x16x4f64:
//               one vector (exp and compensated sum on the vector units;
//               for n >= 16384 each pair of point super-blocks once, K being
//               symmetric), and blocks of columns (the sketch A Omega, block
//               PCG).
#include "operators.hpp"
#include "xtx.hpp"
#include "gemm.hpp"
#include "rbf_lowp.hpp"

namespace nys {

namespace {

// ------------------------------------------------------------- dense GEMV

template <typename TD, typename T>
__global__ __launch_bounds__(256) void dense_gemv(const TD* __restrict__ A, int64_t n, int64_t ld,
                                                  T scale, const T* __restrict__ p, T mu,
                                                  T* __restrict__ v, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const TD* a = A + row * ld;
  T s = T(0);
  for (int64_t j = lane; j < n; j += 64) s += T(a[j]) * p[j];
  s = wave_sum(s);
  if (lane == 0) v[row] = scale * s + mu * p[row];
}

// V[i][c] += mu_c P[i][c]
template <typename T>
__global__ void add_mu(T* __restrict__ V, int64_t ldv, const T* __restrict__ P, int64_t ldp,
                       int64_t n, int64_t k, const double* __restrict__ mu, int64_t nrhs,
                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  V[i * ldv + c] += T(mu[c / nrhs]) * P[i * ldp + c];
}

// V[i][c] = scale V[i][c] + mu_c P[i][c] (mu from the device array when given,
// else the value mu_h): the shift of a caller-supplied product
template <typename T>
__global__ void scale_shift(T* __restrict__ V, int64_t ldv, const T* __restrict__ P, int64_t ldp, int64_t n,
                            int64_t k, double scale, const double* __restrict__ mu, double mu_h,
                            int64_t nrhs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  const double m = mu ? mu[c / nrhs] : mu_h;
  V[i * ldv + c] = T(scale) * V[i * ldv + c] + T(m) * P[i * ldp + c];
}

// ------------------------------------------------------------- RBF, float64

constexpr int RB_ROWS = 64;   // rows per workgroup
constexpr int RB_PTS = 64;    // points per staged tile
constexpr int KV_PTS = 16;    // points per staged tile of the block product

typedef double d4 __attribute__((ext_vector_type(4)));

// One vector, rectangular, float64, Gram on the matrix cores (d <= 4 KS):
// part[s][i] = sum_{j in split s} W_ij p_j with W = K(Xr, Xc) (MODE 0) or
// dK/dsigma (MODE 1).  Wave w of the block owns rows i0 + 16 w .. + 15 and
// forms x_i^T y_j for 16 points at a time with KS v_mfma_f64_16x16x4f64
// (operand lane l: row / point l % 16, coordinate 4 ks + l / 16; result lane l,
// element q: row 4 q + l / 16, point l % 16), so the vector units only do
// the exponential and the compensated accumulation.
template <typename TD, int KS, int MODE>
__global__ __launch_bounds__(256) void rbf_mv_f64m(const TD* __restrict__ Xr, int64_t nr, int64_t ldr,
                                                   const TD* __restrict__ Xc, int64_t nc, int64_t ldc, int d,
                                                   double c2, double inv_s3, const double* __restrict__ p,
                                                   double* __restrict__ part, int64_t pts_per_split,
                                                   const int* __restrict__ skip, double* __restrict__ pvq) {
  if (skip && *skip) return;
  constexpr int DW = 4 * KS;
  __shared__ double Xs[RB_PTS][DW + 1];
  __shared__ double Ns[RB_PTS];
  __shared__ double Ps[RB_PTS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * RB_ROWS + wave * 16;
  // row operand and the norms of this lane's four output rows
  double a[KS];
  double nrm = 0.0;
  {
    const int64_t r = i0 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      a[ks] = (r < nr && kk < d) ? double(Xr[r * ldr + kk]) : 0.0;
      nrm += a[ks] * a[ks];
    }
  }
  nrm += __shfl_xor(nrm, 16, 64);
  nrm += __shfl_xor(nrm, 32, 64);  // every lane: ||x||^2 of row l % 16
  double ni[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ni[q] = __shfl(nrm, 4 * q + (lane >> 4), 64);
  const int64_t j0 = (int64_t)blockIdx.y * pts_per_split;
  const int64_t j1 = (j0 + pts_per_split < nc) ? j0 + pts_per_split : nc;
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, cmp[4] = {0.0, 0.0, 0.0, 0.0};
  // with pvq (square operator): p on this lane's output rows, loaded now
  double pr[4] = {0.0, 0.0, 0.0, 0.0};
  if (pvq) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = i0 + 4 * q + (lane >> 4);
      pr[q] = row < nr ? p[row] : 0.0;
    }
  }
  for (int64_t jt = j0; jt < j1; jt += RB_PTS) {
    __syncthreads();
    {
      double v[RB_PTS * DW / 256];
#pragma unroll
      for (int u = 0; u < RB_PTS * DW / 256; ++u) {
        const int e = t + 256 * u, jj = e / DW, kk = e % DW;
        const int64_t j = jt + jj;
        v[u] = (j < j1 && kk < d) ? double(Xc[j * ldc + kk]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RB_PTS * DW / 256; ++u) {
        const int e = t + 256 * u;
        Xs[e / DW][e % DW] = v[u];
      }
    }
    if (t < RB_PTS) Ps[t] = (jt + t < j1) ? p[jt + t] : 0.0;
    __syncthreads();
    if (t < RB_PTS) {
      double sn = 0.0;
#pragma unroll
      for (int kk = 0; kk < DW; ++kk) sn += Xs[t][kk] * Xs[t][kk];
      Ns[t] = sn;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < RB_PTS / 16; ++st) {
      const int pt = st * 16 + (lane & 15);
      d4 g = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) g = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], Xs[pt][4 * ks + (lane >> 4)], g, 0, 0, 0);
      const double nj = Ns[pt], pj = Ps[pt];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double d2 = fmax(ni[q] + nj - 2.0 * g[q], 0.0);
        const double kv = exp(-d2 * c2);
        const double y = (MODE == 0 ? kv : kv * d2 * inv_s3) * pj - cmp[q];
        const double ts = acc[q] + y;
        cmp[q] = (ts - acc[q]) - y;
        acc[q] = ts;
      }
    }
  }
  // rows 4 q + l / 16: add the 16 lanes (points) of each group in a fixed tree
  double pq = 0.0, pp = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = acc[q] - cmp[q];
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    const int64_t row = i0 + 4 * q + (lane >> 4);
    if ((lane & 15) == 0 && row < nr) {
      part[(int64_t)blockIdx.y * nr + row] = v;
      pq += pr[q] * v;
      pp += pr[q] * pr[q];
    }
  }
  if (pvq) {
    // square operator (Xr = Xc): this workgroup's part of p^T W p at
    // pvq[y gx + x], and the split-0 workgroups' parts of ||p||^2 over their
    // rows at pvq[gx gy + x], so that a CG step knows p^T A p before the
    // partials are summed
    __shared__ double shq[4];
    pq = block_sum(pq, shq);
    if (t == 0) pvq[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = pq;
    if (blockIdx.y == 0) {
      pp = block_sum(pp, shq);
      if (t == 0) pvq[(int64_t)gridDim.x * gridDim.y + blockIdx.x] = pp;
    }
  }
}

// Pair b of the upper triangle (I <= J) of an nsb x nsb block grid, row by
// row: I = the largest with I nsb - I (I - 1) / 2 <= b.
__device__ __forceinline__ void tri_pair(int64_t b, int nsb, int& I, int& J) {
  const double w = 2.0 * nsb + 1.0;
  int64_t i = (int64_t)((w - sqrt(w * w - 8.0 * (double)b)) * 0.5);
  auto off = [&](int64_t x) { return x * nsb - x * (x - 1) / 2; };
  if (i < 0) i = 0;
  while (i > 0 && off(i) > b) --i;
  while (off(i + 1) <= b) ++i;
  I = (int)i;
  J = (int)(i + (b - off(i)));
}

// One vector, square, float64, using the symmetry of K: the points are cut
// into super-blocks of SP and workgroup (I, J), I <= J, evaluates K_IJ once.
// Its rows give part[J][i] = sum_{j in J} K_ij p_j (i in I) and, for I < J,
// its columns give part[I][j] = sum_{i in I} K_ij p_i (j in J): every slot is
// written by one workgroup and (K p)[x] = sum_{Y < nsb} part[Y][x], with half
// the exponentials of rbf_mv_f64m.  J's points are staged in LDS once; the
// rows of I pass in sub-blocks of 64 (wave w: 16 rows, lane layout as in
// rbf_mv_f64m, compensated row sums); column sums go to per-wave LDS rows
// added in a fixed order at the end.
template <typename TD, int KS>
__global__ __launch_bounds__(256) void rbf_mv_f64_sym(const TD* __restrict__ X, int64_t n, int64_t ld, int d,
                                                      double c2, const double* __restrict__ p,
                                                      double* __restrict__ part, int nsb,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int DW = 4 * KS;
  constexpr int SP = KS <= 8 ? 256 : 128;
  __shared__ double Xs[SP][DW + 1];
  __shared__ double Ns[SP], Ps[SP];
  __shared__ double colsum[4][SP];
  int I, J;
  tri_pair(blockIdx.x, nsb, I, J);
  const bool offd = I != J;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)I * SP, j0 = (int64_t)J * SP;
  for (int e = t; e < SP * DW; e += 256) {
    const int jj = e / DW, kk = e % DW;
    const int64_t j = j0 + jj;
    Xs[jj][kk] = (j < n && kk < d) ? double(X[j * ld + kk]) : 0.0;
  }
  __syncthreads();
  for (int x = t; x < SP; x += 256) {
    double sn = 0.0;
#pragma unroll
    for (int kk = 0; kk < DW; ++kk) sn += Xs[x][kk] * Xs[x][kk];
    Ns[x] = sn;
    Ps[x] = (j0 + x < n) ? p[j0 + x] : 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) colsum[w][x] = 0.0;
  }
  __syncthreads();
  for (int sb = 0; sb < SP / 64; ++sb) {
    const int64_t ib = i0 + sb * 64 + wave * 16;  // this wave's 16 rows
    double a[KS];
    double nrm = 0.0;
    {
      const int64_t r = ib + (lane & 15);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kk = 4 * ks + (lane >> 4);
        a[ks] = (r < n && kk < d) ? double(X[r * ld + kk]) : 0.0;
        nrm += a[ks] * a[ks];
      }
    }
    nrm += __shfl_xor(nrm, 16, 64);
    nrm += __shfl_xor(nrm, 32, 64);  // every lane: ||x||^2 of row l % 16
    double ni[4], prow[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, cmp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ni[q] = __shfl(nrm, 4 * q + (lane >> 4), 64);
      const int64_t row = ib + 4 * q + (lane >> 4);
      prow[q] = row < n ? p[row] : 0.0;
    }
    for (int st = 0; st < SP / 16; ++st) {
      const int pt = st * 16 + (lane & 15);
      d4 g = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) g = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], Xs[pt][4 * ks + (lane >> 4)], g, 0, 0, 0);
      const double nj = Ns[pt], pj = Ps[pt];
      double cs = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double d2 = fmax(ni[q] + nj - 2.0 * g[q], 0.0);
        const double kv = exp(-d2 * c2);
        const double y = kv * pj - cmp[q];
        const double ts = acc[q] + y;
        cmp[q] = (ts - acc[q]) - y;
        acc[q] = ts;
        cs = fma(kv, prow[q], cs);
      }
      if (offd) {
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        if (lane < 16) colsum[wave][st * 16 + lane] += cs;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = acc[q] - cmp[q];
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
      const int64_t row = ib + 4 * q + (lane >> 4);
      if ((lane & 15) == 0 && row < n) part[(int64_t)J * n + row] = v;
    }
  }
  if (offd) {
    __syncthreads();
    for (int x = t; x < SP; x += 256)
      if (j0 + x < n) part[(int64_t)I * n + j0 + x] = (colsum[0][x] + colsum[1][x]) + (colsum[2][x] + colsum[3][x]);
  }
}

// Points per super-block of rbf_mv_f64_sym for d coordinates.
int rbf_sym_sp(int d) { return d <= 32 ? 256 : 128; }

// Launches rbf_mv_f64m with the fewest coordinate steps that cover d (<= 64).
template <typename TD, int MODE>
void launch_rbf_mv_f64(dim3 grid, hipStream_t s, const TD* Xr, int64_t nr, int64_t ldr, const TD* Xc,
                       int64_t nc, int64_t ldc, int d, double c2, double is3, const double* p,
                       double* part, int64_t pps, const int* skip, double* pvq = nullptr) {
#define LM(KS) hipLaunchKernelGGL((rbf_mv_f64m<TD, KS, MODE>), grid, dim3(256), 0, s, Xr, nr, ldr, Xc, nc, ldc, d, c2, is3, p, part, pps, skip, pvq)
  if (d <= 4) LM(1);
  else if (d <= 8) LM(2);
  else if (d <= 16) LM(4);
  else if (d <= 32) LM(8);
  else LM(16);
#undef LM
}

// Block of columns: V[I, c0:c0+64] (+)= K_IJ P[J, c0:c0+64] with MFMA f64.
// Grid: (row blocks, column chunks of 64, point splits).  Output partials
// part[split][i][c] (ld = k) when splits > 1, else V directly.
template <typename TD, int DMAX>
__global__ __launch_bounds__(256) void rbf_kv_f64(const TD* __restrict__ X, int64_t n, int d,
                                                  int64_t ld, double c2, const double* __restrict__ P,
                                                  int64_t ldp, int64_t k, double* __restrict__ out,
                                                  int64_t ldo, int64_t pts_per_split, double scale,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double Xi[RB_ROWS][DMAX + 1];
  __shared__ double Xj[KV_PTS][DMAX + 1];
  __shared__ double Ni[RB_ROWS], Nj[KV_PTS];
  __shared__ double Ks[KV_PTS][RB_ROWS + 2];  // Ks[j][i]
  __shared__ double Ps[KV_PTS][64 + 2];       // Ps[j][c]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t i0 = (int64_t)blockIdx.x * RB_ROWS;
  const int64_t cb = (int64_t)blockIdx.y * 64;
  const int64_t j0 = (int64_t)blockIdx.z * pts_per_split;
  const int64_t j1 = (j0 + pts_per_split < n) ? j0 + pts_per_split : n;
  for (int e = t; e < RB_ROWS * DMAX; e += 256) {
    const int ii = e / DMAX, kk = e % DMAX;
    Xi[ii][kk] = (i0 + ii < n && kk < d) ? double(X[(i0 + ii) * ld + kk]) : 0.0;
  }
  __syncthreads();
  if (t < RB_ROWS) {
    double s = 0.0;
    for (int kk = 0; kk < DMAX; ++kk) s += Xi[t][kk] * Xi[t][kk];
    Ni[t] = s;
  }
  // the per-tile MFMA products are summed over tiles with a compensation term
  // (TwoSum), so long point ranges keep float64 accuracy
  d4 acc[2][2], cmp[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = d4{0, 0, 0, 0};
      cmp[a][b] = d4{0, 0, 0, 0};
    }
  for (int64_t jt = j0; jt < j1; jt += KV_PTS) {
    __syncthreads();
    for (int e = t; e < KV_PTS * DMAX; e += 256) {
      const int jj = e / DMAX, kk = e % DMAX;
      Xj[jj][kk] = (jt + jj < j1 && kk < d) ? double(X[(jt + jj) * ld + kk]) : 0.0;
    }
    for (int e = t; e < KV_PTS * 64; e += 256) {
      const int jj = e / 64, cc = e % 64;
      Ps[jj][cc] = (jt + jj < j1 && cb + cc < k) ? P[(jt + jj) * ldp + cb + cc] : 0.0;
    }
    __syncthreads();
    if (t < KV_PTS) {
      double s = 0.0;
      for (int kk = 0; kk < DMAX; ++kk) s += Xj[t][kk] * Xj[t][kk];
      Nj[t] = s;
    }
    __syncthreads();
    // kernel tile: wave w forms rows w*16 .. +15 against the 64 points, the
    // Gram entries on f64 MFMA (row operand from Xi, point operand from Xj;
    // accumulator element q of lane l: row 4 q + l/16, point l % 16)
#pragma unroll
    for (int st = 0; st < KV_PTS / 16; ++st) {
      const int pt = st * 16 + (lane & 15);
      d4 g = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < DMAX / 4; ++ks)
        g = __builtin_amdgcn_mfma_f64_16x16x4f64(Xi[wave * 16 + (lane & 15)][4 * ks + (lane >> 4)],
                                                 Xj[pt][4 * ks + (lane >> 4)], g, 0, 0, 0);
      const double nj = Nj[pt];
      const bool in = jt + pt < j1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ii = wave * 16 + 4 * q + (lane >> 4);
        const double d2 = fmax(Ni[ii] + nj - 2.0 * g[q], 0.0);
        Ks[pt][ii] = in ? exp(-d2 * c2) : 0.0;
      }
    }
    __syncthreads();
    // tile(64 rows x 64 cols) = K(64 x 64 pts) * P(64 pts x 64 cols), then acc += tile
    d4 tl[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) tl[a][b] = d4{0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < KV_PTS; kk += 4) {
      const int kq = kk + (lane >> 4);
      const double a0 = Ks[kq][wm * 32 + (lane & 15)];
      const double a1 = Ks[kq][wm * 32 + 16 + (lane & 15)];
      const double b0 = Ps[kq][wn * 32 + (lane & 15)];
      const double b1 = Ps[kq][wn * 32 + 16 + (lane & 15)];
      tl[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, tl[0][0], 0, 0, 0);
      tl[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, tl[0][1], 0, 0, 0);
      tl[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, tl[1][0], 0, 0, 0);
      tl[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, tl[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const double x = acc[a][b][qq], y = tl[a][b][qq];
          const double sm = x + y, bb = sm - x;
          cmp[a][b][qq] += (x - (sm - bb)) + (y - bb);
          acc[a][b][qq] = sm;
        }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) acc[a][b][qq] += cmp[a][b][qq];
  double* o = out + (int64_t)blockIdx.z * n * ldo;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        // f64 MFMA accumulator element qq of lane l holds row 4 qq + l/16
        const int64_t gi = i0 + wm * 32 + a * 16 + 4 * qq + (lane >> 4);
        const int64_t gc = cb + wn * 32 + b * 16 + (lane & 15);
        if (gi < n && gc < k) o[gi * ldo + gc] = scale * acc[a][b][qq];
      }
}

// out[i][c] = sum_s part[s][i][c] (+ mu_c P[i][c]) for n x k
__global__ void reduce_splits_mu(const double* __restrict__ part, int ns, int64_t n, int64_t k,
                                 double scale, const double* __restrict__ P, int64_t ldp,
                                 const double* __restrict__ mu, int64_t nrhs,
                                 double* __restrict__ out, int64_t ldo,
                                 const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  double s = 0.0;
  for (int q = 0; q < ns; ++q) s += part[((int64_t)q * n + i) * k + c];
  s *= scale;
  if (mu) s += mu[c / nrhs] * P[i * ldp + c];
  out[i * ldo + c] = s;
}

int rbf_dmax(int64_t d) { return d <= 8 ? 8 : d <= 16 ? 16 : d <= 32 ? 32 : d <= 64 ? 64 : -1; }

template <typename TD>
nys_status rbf_apply_f64_t(const OpDesc& op, const double* P, int64_t k, int64_t ldp,
                           const double* mu_dev, int64_t nrhs, double* V, int64_t ldv,
                           double* scratch, size_t scratch_elems, hipStream_t s) {
  const TD* X = static_cast<const TD*>(op.data);
  const int64_t n = op.n;
  const int d = (int)op.cols;
  const double c2 = 1.0 / (2.0 * op.sigma * op.sigma);
  const int dm = rbf_dmax(d);
  if (dm < 0) {
    set_error("RBF operator: d = %d > 64 not supported", d);
    return NYS_ERR_ARG;
  }
  const int64_t nrb = cdiv(n, RB_ROWS);
  const int cus = num_cus() < 256 ? num_cus() : 256;
  if (k == 1 && ldp == 1) {
    // large n: the symmetric form (half the exponentials; n / SP partial slots)
    const int sp = rbf_sym_sp(d);
    const int64_t nsb = cdiv(n, sp);
    if (n >= 16384 && (size_t)(nsb * n) <= scratch_elems) {
      const unsigned pairs = (unsigned)(nsb * (nsb + 1) / 2);
#define LS(KS) hipLaunchKernelGGL((rbf_mv_f64_sym<TD, KS>), dim3(pairs), dim3(256), 0, s, X, n, op.ld, d, c2, P, scratch, (int)nsb, op.skip)
      if (d <= 4) LS(1);
      else if (d <= 8) LS(2);
      else if (d <= 16) LS(4);
      else if (d <= 32) LS(8);
      else LS(16);
#undef LS
      NYS_CHECK_LAUNCH();
      hipLaunchKernelGGL(reduce_splits_mu, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, scratch,
                         (int)nsb, n, (int64_t)1, op.scale, P, ldp, mu_dev, nrhs, V, ldv, op.skip);
      NYS_CHECK_LAUNCH();
      return NYS_OK;
    }
    int64_t ns = cdiv(4 * cus, nrb);
    if (ns < 1) ns = 1;
    while (ns > 1 && (size_t)(ns * n) > scratch_elems) --ns;
    const int64_t pps = cdiv(cdiv(n, ns), RB_PTS) * RB_PTS;
    ns = cdiv(n, pps);
    dim3 grid((unsigned)nrb, (unsigned)ns);
    launch_rbf_mv_f64<TD, 0>(grid, s, X, n, op.ld, X, n, op.ld, d, c2, 0.0, P, scratch, pps, op.skip);
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(reduce_splits_mu, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, scratch,
                       (int)ns, n, (int64_t)1, op.scale, P, ldp, mu_dev, nrhs, V, ldv, op.skip);
    NYS_CHECK_LAUNCH();
    return NYS_OK;
  }
  const int64_t ncb = cdiv(k, 64);
  int64_t ns = cdiv(2 * cus, nrb * ncb);
  if (ns < 1) ns = 1;
  while (ns > 1 && (size_t)(ns * n * k) > scratch_elems) --ns;
  const int64_t pps = cdiv(cdiv(n, ns), RB_PTS) * RB_PTS;
  ns = cdiv(n, pps);
  dim3 grid((unsigned)nrb, (unsigned)ncb, (unsigned)ns);
  double* o = ns > 1 ? scratch : V;
  const int64_t ldo = ns > 1 ? k : ldv;
#define L2(DM) hipLaunchKernelGGL((rbf_kv_f64<TD, DM>), grid, dim3(256), 0, s, X, n, d, op.ld, c2, P, ldp, k, o, ldo, pps, ns > 1 ? 1.0 : op.scale, op.skip)
  if (dm == 8) L2(8); else if (dm == 16) L2(16); else if (dm == 32) L2(32); else L2(64);
#undef L2
  NYS_CHECK_LAUNCH();
  if (ns > 1 || mu_dev) {
    if (ns == 1) {
      // V holds K P; add mu P in place
      hipLaunchKernelGGL(add_mu<double>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, V, ldv,
                         P, ldp, n, k, mu_dev, nrhs, op.skip);
    } else {
      hipLaunchKernelGGL(reduce_splits_mu, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s,
                         scratch, (int)ns, n, k, op.scale, P, ldp, mu_dev, nrhs, V, ldv, op.skip);
    }
    NYS_CHECK_LAUNCH();
  }
  return NYS_OK;
}

template <typename TD>
nys_status rbf_rect_t(const TD* Xr, int64_t nr, int64_t ldr, const TD* Xc, int64_t nc, int64_t ldc,
                      int d, double sigma, int mode, const double* p, double* out, double* scratch,
                      size_t scratch_elems, hipStream_t s) {
  const int dm = rbf_dmax(d);
  if (dm < 0) {
    set_error("RBF operator: d = %d > 64 not supported", d);
    return NYS_ERR_ARG;
  }
  const double c2 = 1.0 / (2.0 * sigma * sigma);
  const double is3 = 1.0 / (sigma * sigma * sigma);
  const int64_t nrb = cdiv(nr, RB_ROWS);
  int64_t ns = cdiv(4 * (num_cus() < 256 ? num_cus() : 256), nrb);
  if (ns < 1) ns = 1;
  while (ns > 1 && (size_t)(ns * nr) > scratch_elems) --ns;
  const int64_t pps = cdiv(cdiv(nc, ns), RB_PTS) * RB_PTS;
  ns = cdiv(nc, pps);
  dim3 grid((unsigned)nrb, (unsigned)ns);
  if (mode == 0)
    launch_rbf_mv_f64<TD, 0>(grid, s, Xr, nr, ldr, Xc, nc, ldc, d, c2, is3, p, scratch, pps, nullptr);
  else
    launch_rbf_mv_f64<TD, 1>(grid, s, Xr, nr, ldr, Xc, nc, ldc, d, c2, is3, p, scratch, pps, nullptr);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_splits_mu, dim3((unsigned)cdiv(nr, 256)), dim3(256), 0, s, scratch,
                     (int)ns, nr, (int64_t)1, 1.0, (const double*)nullptr, (int64_t)1,
                     (const double*)nullptr, (int64_t)1, out, (int64_t)1, (const int*)nullptr);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

}  // namespace

template <typename T>
nys_status callback_apply(const OpDesc& op, const T* P, int64_t k, int64_t ldp, const double* mu_dev,
                          int64_t nrhs, double mu_host, T* V, int64_t ldv, hipStream_t s) {
  const int32_t dt = sizeof(T) == 8 ? NYS_F64 : NYS_F32;
  const int32_t rc = op.apply(op.ctx, k, dt, P, ldp, V, ldv, s);
  if (rc != 0) {
    set_error("operator product routine returned %d (k = %lld, dtype %s)", rc, (long long)k,
              dt == NYS_F64 ? "NYS_F64" : "NYS_F32");
    return NYS_ERR_DEVICE;
  }
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL(scale_shift<T>, dim3((unsigned)cdiv(op.n * k, 256)), dim3(256), 0, s, V, ldv, P, ldp, op.n,
                     k, op.scale, mu_dev, mu_host, nrhs > 0 ? nrhs : 1);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template nys_status callback_apply<double>(const OpDesc&, const double*, int64_t, int64_t, const double*, int64_t,
                                           double, double*, int64_t, hipStream_t);
template nys_status callback_apply<float>(const OpDesc&, const float*, int64_t, int64_t, const double*, int64_t,
                                          double, float*, int64_t, hipStream_t);

namespace {
template <typename T>
__global__ void scale_rows_kernel(T* __restrict__ t, int64_t m, int64_t k, const double* __restrict__ w) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * k) return;
  t[idx] = T(double(t[idx]) * w[idx / k]);
}
}  // namespace

template <typename T>
nys_status scale_rows(T* t, int64_t m, int64_t k, const double* w, hipStream_t s) {
  hipLaunchKernelGGL(scale_rows_kernel<T>, dim3((unsigned)cdiv(m * k, 256)), dim3(256), 0, s, t, m, k, w);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}
template nys_status scale_rows<double>(double*, int64_t, int64_t, const double*, hipStream_t);
template nys_status scale_rows<float>(float*, int64_t, int64_t, const double*, hipStream_t);

size_t op_scratch_elems(const OpDesc& op, int64_t k) {
  if (op.kind == NYS_OP_CALLBACK) return 1;
  if (op.kind == NYS_OP_XTX) {
    const size_t t = (size_t)(op.rows * k);
    return (size_t)(2 * 256 * op.n) + t + gemm_scratch_elems(op.rows, k) + gemm_scratch_elems(op.n, k);
  }
  if (op.kind == NYS_OP_RBF) {
    const size_t one = (size_t)(4 * 256) * (size_t)op.n;
    const int64_t tiles = cdiv(op.n, RB_ROWS) * cdiv(k, 64);
    const int64_t ns = cdiv(2 * 256, tiles);
    size_t blk = ns > 1 ? (size_t)ns * (size_t)op.n * (size_t)k : 0;
    const size_t lowp = rbf_lowp_kv_scratch(op.n, k);  // float elements: fits in as many doubles
    blk = blk > lowp ? blk : lowp;
    return one > blk ? one : blk;
  }
  return gemm_scratch_elems(op.n, k);
}

// V = A P + mu_c P_c (mu_dev == nullptr: no shift).  float64 arithmetic.
nys_status op_apply_f64(const OpDesc& op, const double* P, int64_t k, int64_t ldp,
                        const double* mu_dev, int64_t nrhs, double* V, int64_t ldv,
                        double* scratch, size_t scratch_elems, hipStream_t s) {
  const int64_t n = op.n;
  if (op.kind == NYS_OP_CALLBACK) return callback_apply<double>(op, P, k, ldp, mu_dev, nrhs, 0.0, V, ldv, s);
  if (op.kind == NYS_OP_DENSE) {
    if (k == 1 && ldp == 1 && ldv == 1) {
      // mu is applied by the caller-visible convention: handled by add_mu below
      if (op.dtype == NYS_F64)
        hipLaunchKernelGGL((dense_gemv<double, double>), dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s,
                           static_cast<const double*>(op.data), n, op.ld, op.scale, P, 0.0, V, op.skip);
      else
        hipLaunchKernelGGL((dense_gemv<float, double>), dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s,
                           static_cast<const float*>(op.data), n, op.ld, op.scale, P, 0.0, V, op.skip);
      NYS_CHECK_LAUNCH();
    } else {
      if (op.dtype == NYS_F64)
        NYS_TRY((gemm<double, double, double>(false, false, n, k, n, op.scale,
                                              static_cast<const double*>(op.data), op.ld, P, ldp,
                                              0.0, V, ldv, scratch, scratch_elems, s, op.skip)));
      else
        NYS_TRY((gemm<double, float, double>(false, false, n, k, n, op.scale,
                                             static_cast<const float*>(op.data), op.ld, P, ldp, 0.0,
                                             V, ldv, scratch, scratch_elems, s, op.skip)));
    }
    if (mu_dev) {
      hipLaunchKernelGGL(add_mu<double>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, V, ldv,
                         P, ldp, n, k, mu_dev, nrhs, op.skip);
      NYS_CHECK_LAUNCH();
    }
    return NYS_OK;
  }
  if (op.kind == NYS_OP_XTX) {
    if (k == 1 && ldp == 1 && ldv == 1 && !mu_dev) {
      if (op.dtype == NYS_F64)
        return xtx_apply<double, double>(op, P, 0.0, V, scratch, scratch_elems, s);
      return xtx_apply<float, double>(op, P, 0.0, V, scratch, scratch_elems, s);
    }
    // T = X P (m x k) then V = scale X^T T
    double* T = scratch;
    double* rest = scratch + op.rows * k;
    const size_t rest_elems = scratch_elems - (size_t)(op.rows * k);
    if (op.dtype == NYS_F64) {
      const double* X = static_cast<const double*>(op.data);
      NYS_TRY((gemm<double, double, double>(false, false, op.rows, k, n, 1.0, X, op.ld, P, ldp, 0.0,
                                            T, k, rest, rest_elems, s, op.skip)));
      if (op.w) NYS_TRY(scale_rows<double>(T, op.rows, k, op.w, s));
      NYS_TRY((gemm<double, double, double>(true, false, n, k, op.rows, op.scale, X, op.ld, T, k,
                                            0.0, V, ldv, rest, rest_elems, s, op.skip)));
    } else {
      const float* X = static_cast<const float*>(op.data);
      NYS_TRY((gemm<double, float, double>(false, false, op.rows, k, n, 1.0, X, op.ld, P, ldp, 0.0,
                                           T, k, rest, rest_elems, s, op.skip)));
      if (op.w) NYS_TRY(scale_rows<double>(T, op.rows, k, op.w, s));
      NYS_TRY((gemm<double, float, double>(true, false, n, k, op.rows, op.scale, X, op.ld, T, k, 0.0,
                                           V, ldv, rest, rest_elems, s, op.skip)));
    }
    if (mu_dev) {
      hipLaunchKernelGGL(add_mu<double>, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, V, ldv,
                         P, ldp, n, k, mu_dev, nrhs, op.skip);
      NYS_CHECK_LAUNCH();
    }
    return NYS_OK;
  }
  if (op.kind == NYS_OP_RBF) {
    if (op.dtype == NYS_F64)
      return rbf_apply_f64_t<double>(op, P, k, ldp, mu_dev, nrhs, V, ldv, scratch, scratch_elems, s);
    return rbf_apply_f64_t<float>(op, P, k, ldp, mu_dev, nrhs, V, ldv, scratch, scratch_elems, s);
  }
  set_error("unknown operator kind %d", op.kind);
  return NYS_ERR_ARG;
}

// Single vector, fused shift: v = A p + mu p, arithmetic in TA.
template <typename TA>
nys_status op_matvec(const OpDesc& op, const TA* p, TA mu, TA* v, TA* scratch, size_t scratch_elems,
                     hipStream_t s) {
  const int64_t n = op.n;
  if (op.kind == NYS_OP_CALLBACK) return callback_apply<TA>(op, p, 1, 1, nullptr, 1, double(mu), v, 1, s);
  if (op.kind == NYS_OP_XTX) {
    if (op.dtype == NYS_F64) return xtx_apply<double, TA>(op, p, mu, v, scratch, scratch_elems, s);
    return xtx_apply<float, TA>(op, p, mu, v, scratch, scratch_elems, s);
  }
  if (op.kind == NYS_OP_DENSE) {
    if (op.dtype == NYS_F64)
      hipLaunchKernelGGL((dense_gemv<double, TA>), dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s,
                         static_cast<const double*>(op.data), n, op.ld, TA(op.scale), p, mu, v, op.skip);
    else
      hipLaunchKernelGGL((dense_gemv<float, TA>), dim3((unsigned)cdiv(n, 4)), dim3(256), 0, s,
                         static_cast<const float*>(op.data), n, op.ld, TA(op.scale), p, mu, v, op.skip);
    NYS_CHECK_LAUNCH();
    return NYS_OK;
  }
  set_error("op_matvec: unsupported operator for this precision");
  return NYS_ERR_ARG;
}

// Single vector in partial-sum form: (A p)[j] = scale * sum_{g < ng} part[g][j].
template <typename TA>
nys_status op_matvec_partials(const OpDesc& op, const TA* p, TA* part, size_t part_elems, int* ng_out,
                              hipStream_t s, double* pvq, int* npvq, int* npp);

template <>
nys_status op_matvec_partials<double>(const OpDesc& op, const double* p, double* part, size_t part_elems,
                                      int* ng_out, hipStream_t s, double* pvq, int* npvq, int* npp) {
  const int64_t n = op.n;
  if (npvq) *npvq = 0;
  if (npp) *npp = 0;
  if (!npvq || !npp) pvq = nullptr;
  if (op.kind == NYS_OP_XTX) {
    bool filled = false;
    nys_status st = op.dtype == NYS_F64
                        ? xtx_partials<double, double>(op, p, part, part_elems, ng_out, s, pvq, pvq ? &filled : nullptr)
                        : xtx_partials<float, double>(op, p, part, part_elems, ng_out, s, pvq, pvq ? &filled : nullptr);
    if (st == NYS_OK && filled) {
      *npvq = *ng_out;
      *npp = 1;
    }
    return st;
  }
  if (op.kind == NYS_OP_RBF) {
    const int d = (int)op.cols;
    const int dm = rbf_dmax(d);
    if (dm < 0) {
      set_error("RBF operator: d = %d > 64 not supported", d);
      return NYS_ERR_ARG;
    }
    const double c2 = 1.0 / (2.0 * op.sigma * op.sigma);
    const int64_t nrb = cdiv(n, RB_ROWS);
    int64_t ns = cdiv(4 * (num_cus() < 256 ? num_cus() : 256), nrb);
    if (ns < 1) ns = 1;
    while (ns > 1 && (size_t)(ns * n) > part_elems) --ns;
    // p^T K p parts, one per workgroup, and ||p||^2 parts, one per row block,
    // when they fit the caller's kPvqMax slots
    const bool want_pvq = pvq && 2 * nrb <= kPvqMax;
    if (want_pvq)
      while (ns > 1 && nrb * (ns + 1) > kPvqMax) --ns;
    const int64_t pps = cdiv(cdiv(n, ns), RB_PTS) * RB_PTS;
    ns = cdiv(n, pps);
    dim3 grid((unsigned)nrb, (unsigned)ns);
    double* pq = want_pvq ? pvq : nullptr;
    if (op.dtype == NYS_F64) {
      const double* X = static_cast<const double*>(op.data);
      launch_rbf_mv_f64<double, 0>(grid, s, X, n, op.ld, X, n, op.ld, d, c2, 0.0, p, part, pps, op.skip, pq);
    } else {
      const float* X = static_cast<const float*>(op.data);
      launch_rbf_mv_f64<float, 0>(grid, s, X, n, op.ld, X, n, op.ld, d, c2, 0.0, p, part, pps, op.skip, pq);
    }
    NYS_CHECK_LAUNCH();
    *ng_out = (int)ns;
    if (want_pvq) {
      *npvq = (int)(nrb * ns);
      *npp = (int)nrb;
    }
    return NYS_OK;
  }
  set_error("op_matvec_partials: operator has no partial form");
  return NYS_ERR_ARG;
}

template <>
nys_status op_matvec_partials<float>(const OpDesc& op, const float* p, float* part, size_t part_elems,
                                     int* ng_out, hipStream_t s, double* pvq, int* npvq, int* npp) {
  if (npvq) *npvq = 0;
  if (npp) *npp = 0;
  if (!npvq || !npp) pvq = nullptr;
  if (op.kind == NYS_OP_RBF && op.lowp)
    return rbf_lowp_mv_partials(*op.lowp, op.gram, p, part, part_elems, ng_out, op.skip, s);
  if (op.kind == NYS_OP_XTX) {
    bool filled = false;
    nys_status st = op.dtype == NYS_F64
                        ? xtx_partials<double, float>(op, p, part, part_elems, ng_out, s, pvq, pvq ? &filled : nullptr)
                        : xtx_partials<float, float>(op, p, part, part_elems, ng_out, s, pvq, pvq ? &filled : nullptr);
    if (st == NYS_OK && filled) {
      *npvq = *ng_out;
      *npp = 1;
    }
    return st;
  }
  set_error("op_matvec_partials: float32 form needs X^T X or a prepared RBF operator");
  return NYS_ERR_ARG;
}

template nys_status op_matvec<double>(const OpDesc&, const double*, double, double*, double*, size_t,
                                      hipStream_t);
template nys_status op_matvec<float>(const OpDesc&, const float*, float, float*, float*, size_t,
                                     hipStream_t);

}  // namespace nys

namespace nys {
nys_status rbf_rect_mv(const void* Xr, int64_t nr, int64_t ldr, const void* Xc, int64_t nc,
                       int64_t ldc, int d, int dtype, double sigma, int mode, const double* p,
                       double* out, double* scratch, size_t scratch_elems, hipStream_t s) {
  if (dtype == NYS_F64)
    return rbf_rect_t<double>(static_cast<const double*>(Xr), nr, ldr, static_cast<const double*>(Xc),
                              nc, ldc, d, sigma, mode, p, out, scratch, scratch_elems, s);
  return rbf_rect_t<float>(static_cast<const float*>(Xr), nr, ldr, static_cast<const float*>(Xc), nc,
                           ldc, d, sigma, mode, p, out, scratch, scratch_elems, s);
}
}  // namespace nys
