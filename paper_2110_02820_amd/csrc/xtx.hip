// X^T X products for the ridge normal equations (Section 1.3, eq.
// (RidgeRegression)), one contiguous vector, gfx950.
//
// One pass over X per product (X up to 8192 columns; wider X takes two
// passes, a row-dot kernel and a column-partial kernel): each workgroup owns a contiguous range of rows
// of X, keeps R rows in registers (16-byte vector loads), forms t_r = x_r^T p
// with a block reduction and at once accumulates t_r x_r into a per-workgroup
// partial of X^T t held in registers.  X is read from HBM exactly once; a
// second kernel sums the partials in a fixed order (deterministic) and adds
// mu p.  The PCG loop uses the partial form and folds the final sum into its
// own update kernel.
#include "xtx.hpp"

namespace nys {

namespace {

// ------------------------------------------------------------- X^T X
// (with row weights d, X^T D X: t_r = d_r x_r^T p)

template <typename TD>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int E = 4;
  // X is streamed once per product (no reuse within it): non-temporal loads
  // keep it from displacing other data in the caches (measured 54.4 us per
  // 320 MB product against 58.9 us with ordinary loads)
  static __device__ __forceinline__ float4 load(const float* p) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return float4(v[0], v[1], v[2], v[3]);
  }
  static __device__ __forceinline__ float get(const float4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
  }
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int E = 2;
  static __device__ __forceinline__ double2 load(const double* p) { return *reinterpret_cast<const double2*>(p); }
  static __device__ __forceinline__ double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
};
// one element per load: rows that are not 16-byte aligned
template <typename TD>
struct Vec1 {
  typedef TD type;
  static constexpr int E = 1;
  static __device__ __forceinline__ TD load(const TD* p) { return *p; }
  static __device__ __forceinline__ TD get(const TD& v, int) { return v; }
};

// part[g][j] = sum over rows r of this workgroup of (x_r^T p) x_r[j]
// (accumulated in TA).  Requires n <= 256 * NV * E; with E > 1 the rows must
// be 16-byte aligned and n a multiple of E.  Thread t owns the vectors
// v * 256 + t of every row.  Rows are processed in groups of R; the loads of
// the next group are issued before the current group is reduced, so HBM
// reads stay in flight across the cross-wave reduction.
template <typename TD, typename TA, typename VP, int NV, int R>
__global__ __launch_bounds__(256) void xtx_fused(const TD* __restrict__ X, int64_t m, int64_t n,
                                                 int64_t ld, const TA* __restrict__ p,
                                                 TA* __restrict__ part, int64_t rows_per_wg,
                                                 const int* __restrict__ skip, const double* __restrict__ wts,
                                                 double* __restrict__ pvq) {
  const int sk = skip ? *skip : 0;  // tested once the first loads are issued
  typedef typename VP::type VT;
  constexpr int E = VP::E;
  __shared__ TA red[2][4][R];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t nvec = n / E;
  TA pr[NV][E];
  TA acc[NV][E];
  int64_t off[NV];
  bool ok[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t vi = (int64_t)v * 256 + t;
    ok[v] = vi < nvec;
    off[v] = ok[v] ? vi * E : 0;  // out-of-range vectors read the row start and are masked
#pragma unroll
    for (int e = 0; e < E; ++e) {
      pr[v][e] = ok[v] ? p[vi * E + e] : TA(0);
      acc[v][e] = TA(0);
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < m) ? r0 + rows_per_wg : m;
  int buf = 0;
  double tq = 0.0;  // thread 0, when pvq is given: sum over this workgroup's rows of w_r (x_r^T p)^2
  // one group of RR rows held in registers: t_r = x_r^T p, acc += t_r x_r
  auto process = [&](VT(&xr)[R][NV], int rr, int64_t row0) {
    TA d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      TA s = TA(0);
      if (r < rr) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (!ok[v]) continue;
#pragma unroll
          for (int e = 0; e < E; ++e) s += TA(VP::get(xr[r][v], e)) * pr[v][e];
        }
      }
      d[r] = wave_sum(s);
    }
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) red[buf][wave][r] = d[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= rr) break;
      const TA tu = red[buf][0][r] + red[buf][1][r] + red[buf][2][r] + red[buf][3][r];
      TA tr = tu;
      if (wts) tr *= TA(wts[row0 + r]);  // weighted operator: d_r x_r^T p
      if (pvq && t == 0) tq += double(tu) * double(tr);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!ok[v]) continue;
#pragma unroll
        for (int e = 0; e < E; ++e) acc[v][e] += tr * TA(VP::get(xr[r][v], e));
      }
    }
    buf ^= 1;  // the other buffer is free: its readers passed this barrier
  };
  VT cur[R][NV], nxt[R][NV];
  auto load = [&](VT(&dst)[R][NV], int64_t row) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < NV; ++v) dst[r][v] = VP::load(X + (row + r) * ld + off[v]);
  };
  int64_t rb = r0;
  if (rb + R <= r1) load(cur, rb);
  if (sk) return;
  // two groups per trip (ping-pong buffers, no register copies); each load is
  // issued one group ahead and the last prefetch of a range re-reads valid rows
  for (; rb + 2 * R <= r1; rb += 2 * R) {
    load(nxt, rb + R);
    process(cur, R, rb);
    load(cur, (rb + 3 * R <= r1) ? rb + 2 * R : rb + R);
    process(nxt, R, rb + R);
  }
  if (rb + R <= r1) {  // cur holds rows rb .. rb + R - 1
    process(cur, R, rb);
    rb += R;
  }
  if (rb < r1) {  // fewer than R rows left
    const int rr = (int)(r1 - rb);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < NV; ++v)
        cur[r][v] = *reinterpret_cast<const VT*>(X + (rb + (r < rr ? r : 0)) * ld + off[v]);
    process(cur, rr, rb);
  }
  TA* out = part + (int64_t)blockIdx.x * n;
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (ok[v]) {
      const int64_t vi = (int64_t)v * 256 + t;
#pragma unroll
      for (int e = 0; e < E; ++e) out[vi * E + e] = acc[v][e];
    }
  if (pvq) {
    // pvq[g] = sum over workgroup g's rows of w_r (x_r^T p)^2, so p^T X^T D X p
    // is known without summing the partials; workgroup 0 also writes ||p||^2
    if (t == 0) pvq[blockIdx.x] = tq;
    if (blockIdx.x == 0) {
      __shared__ double shq[4];
      double q = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) q += double(pr[v][e]) * double(pr[v][e]);  // 0 past n
      q = block_sum(q, shq);
      if (t == 0) pvq[gridDim.x] = q;
    }
  }
}

// out[j] = alpha * sum_g part[g][j] + beta * y[j].  Block = 32 columns x 8
// slices of g; each thread sums its slice with two accumulators, then the
// slices are combined in order in LDS (fixed order: deterministic).
template <typename TA, typename TO>
__global__ __launch_bounds__(256) void reduce_cols(const TA* __restrict__ part, int ng, int64_t n, TA alpha,
                                                   const TO* __restrict__ y, TA beta, TO* __restrict__ out,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ TA sh[8][33];
  const int c = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int64_t j = (int64_t)blockIdx.x * 32 + c;
  TA a0 = TA(0), a1 = TA(0);
  if (j < n) {
    int g = sl;
    for (; g + 8 < ng; g += 16) {
      a0 += part[(int64_t)g * n + j];
      a1 += part[(int64_t)(g + 8) * n + j];
    }
    if (g < ng) a0 += part[(int64_t)g * n + j];
  }
  sh[sl][c] = a0 + a1;
  __syncthreads();
  if (sl == 0 && j < n) {
    TA s = ((sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c])) + ((sh[4][c] + sh[5][c]) + (sh[6][c] + sh[7][c]));
    TA o = alpha * s;
    if (y) o += beta * TA(y[j]);
    out[j] = TO(o);
  }
}

// ---- two passes for wide X (more columns than the one-pass kernel keeps
// in registers): t = D X p (one wave per row), then per-group partials of
// X^T t in the same layout as the one-pass kernel.  X is read twice.

// t[r] = w_r x_r^T p, one wave per row (w_r = 1 without weights)
template <typename TD, typename TA, typename VP>
__global__ __launch_bounds__(256) void xtx_rowdot(const TD* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                                                  const TA* __restrict__ p, TA* __restrict__ t,
                                                  const int* __restrict__ skip, const double* __restrict__ wts) {
  if (skip && *skip) return;
  typedef typename VP::type VT;
  constexpr int E = VP::E;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  const TD* x = X + r * ld;
  TA s = TA(0);
  for (int64_t j = (int64_t)lane * E; j < n; j += 64 * E) {
    const VT v = VP::load(x + j);
#pragma unroll
    for (int e = 0; e < E; ++e) s += TA(VP::get(v, e)) * p[j + e];
  }
  s = wave_sum(s);
  if (lane == 0) t[r] = wts ? s * TA(wts[r]) : s;
}

// part[g][j] = sum over rows r of group g of t[r] x_r[j]: thread owns E
// consecutive columns of a block of 256 E, groups of rows_per_group rows
template <typename TD, typename TA, typename VP>
__global__ __launch_bounds__(256) void xtx_colpart(const TD* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                                                   const TA* __restrict__ t, TA* __restrict__ part,
                                                   int64_t rows_per_group, const int* __restrict__ skip) {
  if (skip && *skip) return;
  typedef typename VP::type VT;
  constexpr int E = VP::E;
  const int64_t j0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * E;
  if (j0 >= n) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_group;
  const int64_t r1 = r0 + rows_per_group < m ? r0 + rows_per_group : m;
  TA acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = TA(0);
  int64_t r = r0;
  for (; r + 4 <= r1; r += 4) {  // four rows' loads in flight
    VT v[4];
    TA tr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = VP::load(X + (r + q) * ld + j0);
      tr[q] = t[r + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += tr[q] * TA(VP::get(v[q], e));
  }
  for (; r < r1; ++r) {
    const VT v = VP::load(X + r * ld + j0);
    const TA tr = t[r];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] += tr * TA(VP::get(v, e));
  }
  TA* out = part + (int64_t)blockIdx.y * n + j0;
#pragma unroll
  for (int e = 0; e < E; ++e) out[e] = acc[e];
}

}  // namespace

template <typename TD, typename TA>
nys_status xtx_partials(const OpDesc& op, const TA* p, TA* scratch, size_t scratch_elems, int* ng_out,
                          hipStream_t s, double* pvq, bool* pvq_filled) {
  if (pvq_filled) *pvq_filled = false;
  const TD* X = static_cast<const TD*>(op.data);
  const int64_t m = op.rows, n = op.n;
  constexpr int E = Vec16<TD>::E;
  const bool aligned = (op.ld % E == 0) && (n % E == 0) && ((uintptr_t)X % 16 == 0);
  const int64_t need_nv = aligned ? cdiv(n, 256 * E) : cdiv(n, 256);
  // one workgroup per compute unit (2, 3 or 4 per CU measured no faster)
  int64_t ng = (num_cus() < 256 ? num_cus() : 256);
  const int64_t R = 4;
  if (ng > cdiv(m, R)) ng = cdiv(m, R);
  if (ng < 1) ng = 1;
  while (ng > 1 && (size_t)(ng * n) > scratch_elems) ng /= 2;
  int64_t rpw = cdiv(cdiv(m, ng), R) * R;
  ng = cdiv(m, rpw);
  const bool vec = aligned && need_nv <= 8;
  const int64_t nv1 = cdiv(n, (int64_t)256);
  if (!vec && nv1 > 32) {
    // wide X: two passes (row dots, then column partials); t takes the last
    // m entries of the scratch, the partials the front
    if (scratch_elems < (size_t)(m + n)) {
      set_error("X^T X operator: scratch too small for the two-pass product");
      return NYS_ERR_WORKSPACE;
    }
    TA* t = scratch + (scratch_elems - (size_t)m);
    int64_t ng2 = (num_cus() < 256 ? num_cus() : 256) * 2 / (int64_t)cdiv(n, (int64_t)256 * E);
    if (ng2 < 1) ng2 = 1;
    if (ng2 > cdiv(m, (int64_t)4)) ng2 = cdiv(m, (int64_t)4);
    while (ng2 > 1 && (size_t)(ng2 * n) > scratch_elems - (size_t)m) ng2 /= 2;
    const int64_t rpg = cdiv(m, ng2);
    ng2 = cdiv(m, rpg);
    timing_mark_begin(s);
    if (aligned) {
      hipLaunchKernelGGL((xtx_rowdot<TD, TA, Vec16<TD>>), dim3((unsigned)cdiv(m, (int64_t)4)), dim3(256), 0, s, X,
                         m, n, op.ld, p, t, op.skip, op.w);
      hipLaunchKernelGGL((xtx_colpart<TD, TA, Vec16<TD>>), dim3((unsigned)cdiv(n, (int64_t)256 * E), (unsigned)ng2),
                         dim3(256), 0, s, X, m, n, op.ld, t, scratch, rpg, op.skip);
    } else {
      hipLaunchKernelGGL((xtx_rowdot<TD, TA, Vec1<TD>>), dim3((unsigned)cdiv(m, (int64_t)4)), dim3(256), 0, s, X, m,
                         n, op.ld, p, t, op.skip, op.w);
      hipLaunchKernelGGL((xtx_colpart<TD, TA, Vec1<TD>>), dim3((unsigned)cdiv(n, (int64_t)256), (unsigned)ng2),
                         dim3(256), 0, s, X, m, n, op.ld, t, scratch, rpg, op.skip);
    }
    NYS_CHECK_LAUNCH();
    timing_mark_end(s);
    *ng_out = (int)ng2;
    // the two-pass form does not produce the p^T A p parts (*pvq_filled stays false)
    return NYS_OK;
  }
  if (pvq && pvq_filled) *pvq_filled = true;
#define LX(VP_, NV, RR) hipLaunchKernelGGL((xtx_fused<TD, TA, VP_, NV, RR>), dim3((unsigned)ng), dim3(256), 0, s, X, m, n, op.ld, p, scratch, rpw, op.skip, op.w, pvq_filled ? pvq : nullptr)
  timing_mark_begin(s);
  if (vec) {
    if (need_nv <= 1) LX(Vec16<TD>, 1, 4);
    else if (need_nv <= 2) LX(Vec16<TD>, 2, 4);
    else if (need_nv <= 4) LX(Vec16<TD>, 4, 4);
    else LX(Vec16<TD>, 8, 2);
  } else {  // scalar loads: rows not 16-byte aligned, or too many 16-byte vectors per thread
    if (nv1 <= 4) LX(Vec1<TD>, 4, 4);
    else if (nv1 <= 8) LX(Vec1<TD>, 8, 4);
    else if (nv1 <= 16) LX(Vec1<TD>, 16, 4);
    else LX(Vec1<TD>, 32, 2);
  }
#undef LX
  NYS_CHECK_LAUNCH();
  timing_mark_end(s);
  *ng_out = (int)ng;
  return NYS_OK;
}

template <typename TD, typename TA>
nys_status xtx_apply(const OpDesc& op, const TA* p, TA mu, TA* v, TA* scratch,
                       size_t scratch_elems, hipStream_t s) {
  int ng = 0;
  NYS_TRY((xtx_partials<TD, TA>(op, p, scratch, scratch_elems, &ng, s)));
  const int64_t n = op.n;
  hipLaunchKernelGGL((reduce_cols<TA, TA>), dim3((unsigned)cdiv(n, 32)), dim3(256), 0, s, scratch,
                     ng, n, TA(op.scale), p, mu, v, op.skip);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}


template nys_status xtx_partials<float, float>(const OpDesc&, const float*, float*, size_t, int*, hipStream_t,
                                               double*, bool*);
template nys_status xtx_partials<float, double>(const OpDesc&, const double*, double*, size_t, int*, hipStream_t,
                                                double*, bool*);
template nys_status xtx_partials<double, float>(const OpDesc&, const float*, float*, size_t, int*, hipStream_t,
                                                double*, bool*);
template nys_status xtx_partials<double, double>(const OpDesc&, const double*, double*, size_t, int*, hipStream_t,
                                                 double*, bool*);
template nys_status xtx_apply<float, float>(const OpDesc&, const float*, float, float*, float*, size_t, hipStream_t);
template nys_status xtx_apply<float, double>(const OpDesc&, const double*, double, double*, double*, size_t,
                                             hipStream_t);
template nys_status xtx_apply<double, float>(const OpDesc&, const float*, float, float*, float*, size_t,
                                             hipStream_t);
template nys_status xtx_apply<double, double>(const OpDesc&, const double*, double, double*, double*, size_t,
                                              hipStream_t);

}  // namespace nys
