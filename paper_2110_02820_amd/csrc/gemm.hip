// Tiled MFMA GEMM for the sketch and factorisation steps (gfx950).
//
//   C = alpha * op(A) * op(B) + beta * C      (row-major, leading dimensions)
//
// float64 uses v_mfma_f64_16x16x4f64, float32 uses v_mfma_f32_16x16x4f32.
// Storage types of A and B may be narrower than the compute type (float32
// data promoted exactly to float64).  A 256-thread workgroup computes a
// 64 x 64 tile as a 2 x 2 arrangement of waves, each wave a 32 x 32 block of
// four 16 x 16 MFMA tiles; the K loop stages 16-deep slabs of A and B through
// LDS.  When the output has too few tiles to fill 256 CUs, K is split across
// workgroups (grid z) and a second kernel sums the partial tiles in a fixed
// order, so results are deterministic.  Large products with 16-byte aligned
// operands use 128 x 128 tiles instead (gemm_large).
#include "gemm.hpp"

namespace nys {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element q of lane l holds D[4 q + l/16][l % 16]
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * q + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element q of lane l holds D[4 (l/16) + q][l % 16]
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// Lane layout of the 16x16x4 MFMA (one wave): operand a holds A[l%16][l/16],
// operand b holds B[l/16][l%16]; the accumulator rows differ between the f32
// and f64 forms (Mfma<T>::row, checked on the device).
template <typename TC, typename TAs, typename TBs, bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                  TC alpha, const TAs* __restrict__ A, int64_t lda,
                                                  const TBs* __restrict__ B, int64_t ldb, TC beta,
                                                  TC* __restrict__ C, int64_t ldc,
                                                  TC* __restrict__ part, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ TC As[BK][BM + 4];
  __shared__ TC Bs[BK][BN + 4];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;

  typename Mfma<TC>::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<TC>::acc_t{0, 0, 0, 0};

  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    // stage A slab (BM x BK) as As[k][m]
#pragma unroll
    for (int r = 0; r < (BM * BK) / NT; ++r) {
      const int e = t + r * NT;
      int mm, kk;
      if (!TA) { mm = e / BK; kk = e % BK; } else { kk = e / BM; mm = e % BM; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      TC v = TC(0);
      if (gm < M && gk < ke) v = TC(TA ? A[gk * lda + gm] : A[gm * lda + gk]);
      As[kk][mm] = v;
    }
    // stage B slab (BK x BN) as Bs[k][n]
#pragma unroll
    for (int r = 0; r < (BN * BK) / NT; ++r) {
      const int e = t + r * NT;
      int nn, kk;
      if (!TB) { kk = e / BN; nn = e % BN; } else { nn = e / BK; kk = e % BK; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      TC v = TC(0);
      if (gn < N && gk < ke) v = TC(TB ? B[gn * ldb + gk] : B[gk * ldb + gn]);
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      TC a0 = As[kk][wm * 32 + (lane & 15)];
      TC a1 = As[kk][wm * 32 + 16 + (lane & 15)];
      TC b0 = Bs[kk][wn * 32 + (lane & 15)];
      TC b1 = Bs[kk][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = Mfma<TC>::op(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<TC>::op(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<TC>::op(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<TC>::op(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gm = m0 + wm * 32 + i * 16 + Mfma<TC>::row(lane, q);
        const int64_t gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const TC v = acc[i][j][q];
          if (part) {
            part[((int64_t)blockIdx.z * M + gm) * N + gn] = v;
          } else {
            TC o = alpha * v;
            if (beta != TC(0)) o += beta * C[gm * ldc + gn];
            C[gm * ldc + gn] = o;
          }
        }
      }
}

// 16-byte vector of storage elements.
template <typename TS>
struct Vec16B;
template <>
struct Vec16B<float> {
  typedef float4 type;
  static constexpr int E = 4;
};
template <>
struct Vec16B<double> {
  typedef double2 type;
  static constexpr int E = 2;
};
template <typename TS>
__device__ __forceinline__ TS vget(const typename Vec16B<TS>::type& v, int u);
template <>
__device__ __forceinline__ float vget<float>(const float4& v, int u) {
  return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w;
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int u) {
  return u == 0 ? v.x : v.y;
}

constexpr int LM = 128, LN = 128, LK = 16, LPAD = 16;

// Large tiles: a 256-thread workgroup computes a 128 x 128 tile, each wave a
// 64 x 64 block of 4 x 4 MFMA tiles, from 16-deep slabs of A and B loaded with
// 16-byte vector loads; the next slab is held in registers while the current
// one is multiplied out of LDS.  Requires the contiguous dimension of each
// operand to be a multiple of the vector width and 16-byte aligned rows
// (checked on the host).  Tiles are numbered so that the workgroups that
// share a row block of A run on the same XCD (blocks are dealt to the XCDs
// round-robin): grid = 8 * ceil(tiles / 8) in x, split-K in y.
template <typename TC, typename TAs, typename TBs, bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_large(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                 TC alpha, const TAs* __restrict__ A, int64_t lda,
                                                 const TBs* __restrict__ B, int64_t ldb, TC beta,
                                                 TC* __restrict__ C, int64_t ldc,
                                                 TC* __restrict__ part, const int* __restrict__ skip) {
  if (skip && *skip) return;
  typedef typename Vec16B<TAs>::type VA;
  typedef typename Vec16B<TBs>::type VB;
  constexpr int EA = Vec16B<TAs>::E, EB = Vec16B<TBs>::E;
  constexpr int NVA = LM * LK / EA / NT, NVB = LN * LK / EB / NT;
  __shared__ TC As[LK][LM + LPAD];
  __shared__ TC Bs[LK][LN + LPAD];
  const int64_t mt = (M + LM - 1) / LM, nt = (N + LN - 1) / LN, tiles = mt * nt;
  const int64_t per = (int64_t)gridDim.x / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= tiles) return;
  const int64_t m0 = (tile / nt) * LM, n0 = (tile % nt) * LN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;

  VA ra[NVA];
  VB rb[NVB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < NVA; ++r) {
      const int e = t + r * NT;
      int64_t gm, gk;
      if (!TA) { gm = m0 + e / (LK / EA); gk = k0 + (e % (LK / EA)) * EA; }
      else { gk = k0 + e / (LM / EA); gm = m0 + (e % (LM / EA)) * EA; }
      const bool ok = gm < M && gk < ke;
      ra[r] = ok ? *reinterpret_cast<const VA*>(TA ? A + gk * lda + gm : A + gm * lda + gk) : VA{};
    }
#pragma unroll
    for (int r = 0; r < NVB; ++r) {
      const int e = t + r * NT;
      int64_t gn, gk;
      if (TB) { gn = n0 + e / (LK / EB); gk = k0 + (e % (LK / EB)) * EB; }
      else { gk = k0 + e / (LN / EB); gn = n0 + (e % (LN / EB)) * EB; }
      const bool ok = gn < N && gk < ke;
      rb[r] = ok ? *reinterpret_cast<const VB*>(TB ? B + gn * ldb + gk : B + gk * ldb + gn) : VB{};
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < NVA; ++r) {
      const int e = t + r * NT;
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        if (!TA) As[(e % (LK / EA)) * EA + u][e / (LK / EA)] = TC(vget<TAs>(ra[r], u));
        else As[e / (LM / EA)][(e % (LM / EA)) * EA + u] = TC(vget<TAs>(ra[r], u));
      }
    }
#pragma unroll
    for (int r = 0; r < NVB; ++r) {
      const int e = t + r * NT;
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        if (TB) Bs[(e % (LK / EB)) * EB + u][e / (LK / EB)] = TC(vget<TBs>(rb[r], u));
        else Bs[e / (LN / EB)][(e % (LN / EB)) * EB + u] = TC(vget<TBs>(rb[r], u));
      }
    }
  };

  typename Mfma<TC>::acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = typename Mfma<TC>::acc_t{0, 0, 0, 0};

  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += LK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + LK < ke) load(k0 + LK);
#pragma unroll
    for (int ks = 0; ks < LK; ks += 4) {
      const int kk = ks + (lane >> 4);
      TC a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<TC>::op(a[i], b[j], acc[i][j]);
    }
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gm = m0 + wm * 64 + i * 16 + Mfma<TC>::row(lane, q);
        const int64_t gn = n0 + wn * 64 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const TC v = acc[i][j][q];
          if (part) {
            part[((int64_t)blockIdx.y * M + gm) * N + gn] = v;
          } else {
            TC o = alpha * v;
            if (beta != TC(0)) o += beta * C[gm * ldc + gn];
            C[gm * ldc + gn] = o;
          }
        }
      }
}

// float32 operands, products on bf16 MFMA with the three-product split:
// a = a_hi + a_lo, b = b_hi + b_lo (bf16, round to nearest even) and
// a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi, float32 accumulation (relative
// error ~2^-16 per product).  128 x 128 tiles, 4 waves of 64 x 64, 32-deep
// slabs (one v_mfma_f32_16x16x32_bf16 step), split in registers on the way
// into LDS as [row][k] (A) and [column][k] (B) so that each lane reads its
// 8 consecutive k with one 16-byte load; the next slab is loaded while the
// current one is multiplied.  Tile numbering and split-K as in gemm_large.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16x4(const float (&v)[4], bf4v& hi, bf4v& lo) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const __bf16 h = (__bf16)v[u];
    hi[u] = h;
    lo[u] = (__bf16)(v[u] - (float)h);
  }
}

#ifndef NYS_GEMM_XK
#define NYS_GEMM_XK 32
#endif
constexpr int XK = NYS_GEMM_XK, XPAD = XK + 8;  // k per staged slab (a multiple of 32)
constexpr int XR = XK / 8;                      // runs of 4 k per thread per operand and slab
constexpr int XQ = XK / 4;                      // runs of 4 k per row of a slab

// B split once into bf16 hi / lo, column-major by k: element (k, n) at
// [n * ldk + k], ldk a multiple of XK, zeros past K (split_b_bf16).
struct SplitB {
  const __bf16* hi;
  const __bf16* lo;
  int64_t ldk;
};

// PB: B comes pre-split (SplitB) and is copied into LDS as it stands, two
// 16-byte runs of 8 k per thread and piece; else B is split on the way in.
template <bool TA, bool TB, bool PB>
__global__ __launch_bounds__(NT) void gemm_bf16x3(int64_t M, int64_t N, int64_t K, int64_t kchunk, float alpha,
                                                  const float* __restrict__ A, int64_t lda,
                                                  const float* __restrict__ B, int64_t ldb, SplitB bs, float beta,
                                                  float* __restrict__ C, int64_t ldc, float* __restrict__ part,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[LM][XPAD], Al[LM][XPAD], Bh[LN][XPAD], Bl[LN][XPAD];
  const int64_t mt = (M + LM - 1) / LM, nt = (N + LN - 1) / LN, tiles = mt * nt;
  const int64_t per = (int64_t)gridDim.x / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= tiles) return;
  const int64_t m0 = (tile / nt) * LM, n0 = (tile % nt) * LN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  // each thread stages XR runs of 4 consecutive k for A and for B (128 x XK each)
  float ra[XR][4], rb[XR][4];
  constexpr int PR = LN * XK / 8 / NT;  // pre-split B: 16-byte runs of 8 k per thread and piece
  uint4 rbh[PR], rbl[PR];
  auto load = [&](int64_t k0) {
    if (PB) {
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int e = t + NT * r, col = e / (XK / 8), k8 = e % (XK / 8);
        const int64_t gn = n0 + col;
        if (gn < N) {
          const int64_t o = gn * bs.ldk + k0 + 8 * k8;  // k0 + XK <= ldk (zero padded)
          rbh[r] = *reinterpret_cast<const uint4*>(bs.hi + o);
          rbl[r] = *reinterpret_cast<const uint4*>(bs.lo + o);
        } else {
          rbh[r] = make_uint4(0u, 0u, 0u, 0u);
          rbl[r] = make_uint4(0u, 0u, 0u, 0u);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < XR; ++r) {
      const int e = t + NT * r;
      // A run: row (e % 128) when A is transposed, else row e / XQ; k offset 4 * (e / 128) or 4 * (e % XQ)
      const int row = TA ? (e & (LM - 1)) : (e / XQ);
      const int kq = TA ? (e >> 7) : (e % XQ);
      const int64_t gm = m0 + row, gk = k0 + 4 * kq;
      if (!TA && gm < M && gk + 3 < ke) {
        const float4 v = *reinterpret_cast<const float4*>(A + gm * lda + gk);
        ra[r][0] = v.x; ra[r][1] = v.y; ra[r][2] = v.z; ra[r][3] = v.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          ra[r][u] = (gm < M && gk + u < ke) ? (TA ? A[(gk + u) * lda + gm] : A[gm * lda + gk + u]) : 0.0f;
      }
      if (PB) continue;
      const int col = TB ? (e / XQ) : (e & (LN - 1));
      const int kqb = TB ? (e % XQ) : (e >> 7);
      const int64_t gn = n0 + col, gkb = k0 + 4 * kqb;
      if (TB && gn < N && gkb + 3 < ke) {
        const float4 v = *reinterpret_cast<const float4*>(B + gn * ldb + gkb);
        rb[r][0] = v.x; rb[r][1] = v.y; rb[r][2] = v.z; rb[r][3] = v.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          rb[r][u] = (gn < N && gkb + u < ke) ? (TB ? B[gn * ldb + gkb + u] : B[(gkb + u) * ldb + gn]) : 0.0f;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < XR; ++r) {
      const int e = t + NT * r;
      const int row = TA ? (e & (LM - 1)) : (e / XQ);
      const int kq = TA ? (e >> 7) : (e % XQ);
      bf4v h, l;
      split_bf16x4(ra[r], h, l);
      *reinterpret_cast<bf4v*>(&Ah[row][4 * kq]) = h;
      *reinterpret_cast<bf4v*>(&Al[row][4 * kq]) = l;
      if (PB) continue;
      const int col = TB ? (e / XQ) : (e & (LN - 1));
      const int kqb = TB ? (e % XQ) : (e >> 7);
      split_bf16x4(rb[r], h, l);
      *reinterpret_cast<bf4v*>(&Bh[col][4 * kqb]) = h;
      *reinterpret_cast<bf4v*>(&Bl[col][4 * kqb]) = l;
    }
    if (PB) {
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int e = t + NT * r, col = e / (XK / 8), k8 = e % (XK / 8);
        *reinterpret_cast<uint4*>(&Bh[col][8 * k8]) = rbh[r];
        *reinterpret_cast<uint4*>(&Bl[col][8 * k8]) = rbl[r];
      }
    }
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += XK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + XK < ke) load(k0 + XK);
#pragma unroll
    for (int kk = 0; kk < XK; kk += 32) {
      const int ks = kk + 8 * (lane >> 4);
      bf8v ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ah[i] = *reinterpret_cast<const bf8v*>(&Ah[wm * 64 + i * 16 + (lane & 15)][ks]);
        al[i] = *reinterpret_cast<const bf8v*>(&Al[wm * 64 + i * 16 + (lane & 15)][ks]);
        bh[i] = *reinterpret_cast<const bf8v*>(&Bh[wn * 64 + i * 16 + (lane & 15)][ks]);
        bl[i] = *reinterpret_cast<const bf8v*>(&Bl[wn * 64 + i * 16 + (lane & 15)][ks]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          f4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], c, 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], c, 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gm = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + q;
        const int64_t gn = n0 + wn * 64 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const float v = acc[i][j][q];
          if (part) {
            part[((int64_t)blockIdx.y * M + gm) * N + gn] = v;
          } else {
            float o = alpha * v;
            if (beta != 0.0f) o += beta * C[gm * ldc + gn];
            C[gm * ldc + gn] = o;
          }
        }
      }
}

// B (K x N, or N x K stored when tb) -> hi / lo bf16 pieces at [n * ldk + k]
// (round to nearest even, as split_bf16x4), zeros for K <= k < ldk.  32 x 32
// tiles through LDS so that both the reads of B and the writes are coalesced.
__global__ __launch_bounds__(256) void split_b_bf16(int64_t K, int64_t N, const float* __restrict__ B, int64_t ldb,
                                                    int tb, int64_t ldk, __bf16* __restrict__ hi,
                                                    __bf16* __restrict__ lo) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t k0 = (int64_t)blockIdx.x * 32, n0 = (int64_t)blockIdx.y * 32;
  // read: rows of B's storage run along its contiguous index
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    float v = 0.0f;
    if (tb) {  // B stored N x K: contiguous in k
      const int64_t n = n0 + r, k = k0 + tx;
      if (n < N && k < K) v = B[n * ldb + k];
      tile[r][tx] = v;  // [n][k]
    } else {   // B stored K x N: contiguous in n
      const int64_t k = k0 + r, n = n0 + tx;
      if (n < N && k < K) v = B[k * ldb + n];
      tile[tx][r] = v;  // [n][k]
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int64_t n = n0 + r, k = k0 + tx;
    if (n < N && k < ldk) {
      const float v = tile[r][tx];
      const __bf16 h = (__bf16)v;
      hi[n * ldk + k] = h;
      lo[n * ldk + k] = (__bf16)(v - (float)h);
    }
  }
}

template <typename TC>
__global__ void splitk_reduce(int64_t M, int64_t N, int nz, TC alpha, const TC* __restrict__ part,
                              TC beta, TC* __restrict__ C, int64_t ldc, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t m = idx / N, n = idx % N;
  TC s = TC(0);
  for (int z = 0; z < nz; ++z) s += part[(int64_t)z * M * N + idx];
  TC o = alpha * s;
  if (beta != TC(0)) o += beta * C[m * ldc + n];
  C[m * ldc + n] = o;
}

}  // namespace

template <typename TC, typename TAs, typename TBs>
nys_status gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, TC alpha, const TAs* A,
                int64_t lda, const TBs* B, int64_t ldb, TC beta, TC* C, int64_t ldc, TC* scratch,
                size_t scratch_elems, hipStream_t s, const int* skip) {
  if (M <= 0 || N <= 0) return NYS_OK;
  // large problems whose operands allow 16-byte loads: 128 x 128 tiles
  constexpr int EA = 16 / sizeof(TAs), EB = 16 / sizeof(TBs);
  const bool vec_a = (lda % EA == 0) && ((uintptr_t)A % 16 == 0) && ((ta ? M : K) % EA == 0);
  const bool vec_b = (ldb % EB == 0) && ((uintptr_t)B % 16 == 0) && ((tb ? K : N) % EB == 0);
  if (vec_a && vec_b && M >= LM && N >= 64 && K >= 4 * LK && (double)M * N * K >= 1.0e9) {
    const int64_t lt = cdiv(M, LM) * cdiv(N, LN);
    const int64_t target = 2 * (int64_t)(num_cus() < 256 ? num_cus() : 256);
    int64_t nz = 1;
    if (lt < target) {
      nz = cdiv(target, lt);
      nz = nz < cdiv(K, 16 * LK) ? nz : cdiv(K, 16 * LK);
      while (nz > 1 && (size_t)(nz * M * N) > scratch_elems) --nz;
      if (nz > 64) nz = 64;
    }
    const int64_t kchunk = cdiv(cdiv(K, nz), LK) * LK;
    nz = cdiv(K, kchunk);
    dim3 grid((unsigned)(8 * cdiv(lt, 8)), (unsigned)nz);
    TC* part = nz > 1 ? scratch : nullptr;
#define NYS_GEMM_LARGE(TA_, TB_)                                                              \
  hipLaunchKernelGGL((gemm_large<TC, TAs, TBs, TA_, TB_>), grid, dim3(NT), 0, s, M, N, K,    \
                     kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part, skip)
    if (!ta && !tb) NYS_GEMM_LARGE(false, false);
    else if (!ta && tb) NYS_GEMM_LARGE(false, true);
    else if (ta && !tb) NYS_GEMM_LARGE(true, false);
    else NYS_GEMM_LARGE(true, true);
#undef NYS_GEMM_LARGE
    NYS_CHECK_LAUNCH();
    if (nz > 1) {
      const int64_t tot = M * N;
      hipLaunchKernelGGL(splitk_reduce<TC>, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, M, N,
                         (int)nz, alpha, part, beta, C, ldc, skip);
      NYS_CHECK_LAUNCH();
    }
    return NYS_OK;
  }
  const int64_t tiles = cdiv(M, BM) * cdiv(N, BN);

  const int64_t target = 2 * (int64_t)(num_cus() < 256 ? num_cus() : 256);
  int64_t nz = 1;
  if (tiles < target && K > 4 * BK) {
    nz = cdiv(target, tiles);
    nz = nz < cdiv(K, 8 * BK) ? nz : cdiv(K, 8 * BK);
    while (nz > 1 && (size_t)(nz * M * N) > scratch_elems) --nz;
    if (nz > 64) nz = 64;
  }
  int64_t kchunk = cdiv(cdiv(K, nz), BK) * BK;
  if (K <= 0) kchunk = BK;
  nz = K > 0 ? cdiv(K, kchunk) : 1;
  dim3 grid((unsigned)cdiv(N, BN), (unsigned)cdiv(M, BM), (unsigned)nz);
  TC* part = nz > 1 ? scratch : nullptr;
#define NYS_GEMM_LAUNCH(TA_, TB_)                                                              \
  hipLaunchKernelGGL((gemm_kernel<TC, TAs, TBs, TA_, TB_>), grid, dim3(NT), 0, s, M, N, K,    \
                     kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part, skip)
  if (!ta && !tb) NYS_GEMM_LAUNCH(false, false);
  else if (!ta && tb) NYS_GEMM_LAUNCH(false, true);
  else if (ta && !tb) NYS_GEMM_LAUNCH(true, false);
  else NYS_GEMM_LAUNCH(true, true);
#undef NYS_GEMM_LAUNCH
  NYS_CHECK_LAUNCH();
  if (nz > 1) {
    const int64_t tot = M * N;
    hipLaunchKernelGGL(splitk_reduce<TC>, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, M, N,
                       (int)nz, alpha, part, beta, C, ldc, skip);
    NYS_CHECK_LAUNCH();
  }
  return NYS_OK;
}

template nys_status gemm<double, double, double>(bool, bool, int64_t, int64_t, int64_t, double,
                                                 const double*, int64_t, const double*, int64_t,
                                                 double, double*, int64_t, double*, size_t,
                                                 hipStream_t, const int*);
template nys_status gemm<double, float, double>(bool, bool, int64_t, int64_t, int64_t, double,
                                                const float*, int64_t, const double*, int64_t,
                                                double, double*, int64_t, double*, size_t,
                                                hipStream_t, const int*);
template nys_status gemm<double, double, float>(bool, bool, int64_t, int64_t, int64_t, double,
                                                const double*, int64_t, const float*, int64_t,
                                                double, double*, int64_t, double*, size_t,
                                                hipStream_t, const int*);
template nys_status gemm<double, float, float>(bool, bool, int64_t, int64_t, int64_t, double,
                                               const float*, int64_t, const float*, int64_t, double,
                                               double*, int64_t, double*, size_t, hipStream_t, const int*);
template nys_status gemm<float, float, float>(bool, bool, int64_t, int64_t, int64_t, float,
                                              const float*, int64_t, const float*, int64_t, float,
                                              float*, int64_t, float*, size_t, hipStream_t, const int*);
template nys_status gemm<float, float, double>(bool, bool, int64_t, int64_t, int64_t, float,
                                               const float*, int64_t, const double*, int64_t, float,
                                               float*, int64_t, float*, size_t, hipStream_t, const int*);

namespace {

// Launches of one bf16x3 product; bs.hi != nullptr: B pre-split.
nys_status gemm_bf16x3_run(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                           int64_t lda, const float* B, int64_t ldb, SplitB bs, float beta, float* C, int64_t ldc,
                           float* scratch, size_t scratch_elems, hipStream_t s) {
  const int64_t nt = cdiv(N, LN), lt = cdiv(M, LM) * nt;
  // two workgroups of this kernel fit on a compute unit: one round of tiles
  const int64_t target = 2 * (int64_t)(num_cus() < 256 ? num_cus() : 256);
  if (lt > target && lt < 2 * target) {
    // between one and two rounds: the rows of one full round first, then
    // the remaining rows on their own, split over k, instead of a second
    // round that leaves most compute units idle (the ridge sketch's
    // 20000 x 500 product: 628 tiles for 512 slots)
    const int64_t m1 = (target / nt) * LM;
    if (m1 > 0 && m1 < M) {
      NYS_TRY(gemm_bf16x3_run(ta, tb, m1, N, K, alpha, A, lda, B, ldb, bs, beta, C, ldc, scratch, scratch_elems,
                              s));
      const float* A2 = ta ? A + m1 : A + m1 * lda;
      return gemm_bf16x3_run(ta, tb, M - m1, N, K, alpha, A2, lda, B, ldb, bs, beta, C + m1 * ldc, ldc, scratch,
                             scratch_elems, s);
    }
  }
  int64_t nz = 1;
  if (lt < target) {
    nz = cdiv(target, lt);
    nz = nz < cdiv(K, 8 * XK) ? nz : cdiv(K, 8 * XK);
    while (nz > 1 && (size_t)(nz * M * N) > scratch_elems) --nz;
    if (nz > 64) nz = 64;
  }
  const int64_t kchunk = cdiv(cdiv(K, nz), XK) * XK;
  nz = cdiv(K, kchunk);
  dim3 grid((unsigned)(8 * cdiv(lt, 8)), (unsigned)nz);
  float* part = nz > 1 ? scratch : nullptr;
#define NYS_GEMM_B3(TA_, TB_, PB_)                                                                            \
  hipLaunchKernelGGL((gemm_bf16x3<TA_, TB_, PB_>), grid, dim3(NT), 0, s, M, N, K, kchunk, alpha, A, lda, B, ldb, \
                     bs, beta, C, ldc, part, (const int*)nullptr)
  if (bs.hi) {
    if (ta) NYS_GEMM_B3(true, false, true);
    else NYS_GEMM_B3(false, false, true);
  } else if (!ta && !tb) {
    NYS_GEMM_B3(false, false, false);
  } else if (!ta && tb) {
    NYS_GEMM_B3(false, true, false);
  } else if (ta && !tb) {
    NYS_GEMM_B3(true, false, false);
  } else {
    NYS_GEMM_B3(true, true, false);
  }
#undef NYS_GEMM_B3
  NYS_CHECK_LAUNCH();
  if (nz > 1) {
    hipLaunchKernelGGL(splitk_reduce<float>, dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s, M, N, (int)nz,
                       alpha, part, beta, C, ldc, (const int*)nullptr);
    NYS_CHECK_LAUNCH();
  }
  return NYS_OK;
}

}  // namespace

size_t gemm_bf16x3_split_elems(int64_t K, int64_t N) { return (size_t)(cdiv(K, XK) * XK) * (size_t)N; }

nys_status gemm_bf16x3(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float beta, float* C, int64_t ldc, float* scratch,
                       size_t scratch_elems, hipStream_t s) {
  if (M <= 0 || N <= 0) return NYS_OK;
  // float4 loads along k need 16-byte aligned rows
  const bool vec_a = ta || ((lda % 4 == 0) && ((uintptr_t)A % 16 == 0));
  const bool vec_b = !tb || ((ldb % 4 == 0) && ((uintptr_t)B % 16 == 0));
  if (!vec_a || !vec_b || K % 4 != 0)
    return gemm<float, float, float>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch, scratch_elems, s);
  // B split into bf16 pieces once (every row block of A reads it) when the
  // scratch's tail holds the pieces and its front the split-K partials the
  // product would take anyway
  SplitB bs{nullptr, nullptr, 0};
  const int64_t ldk = cdiv(K, XK) * XK;
  const size_t pieces = (size_t)ldk * (size_t)N;  // hi + lo bf16: one float's room each
  const int64_t lt = cdiv(M, LM) * cdiv(N, LN);
  const int64_t target = 2 * (int64_t)(num_cus() < 256 ? num_cus() : 256);
  int64_t nzw = lt < target ? cdiv(target, lt) : 1;
  if (nzw > 64) nzw = 64;
  const size_t want = pieces + (nzw > 1 ? (size_t)nzw * (size_t)M * (size_t)N : 0) + 4;
  if (scratch && want <= scratch_elems) {
    const size_t off = (scratch_elems - pieces) & ~(size_t)3;  // 16-byte aligned pieces
    __bf16* hi = reinterpret_cast<__bf16*>(scratch + off);
    __bf16* lo = hi + (size_t)ldk * (size_t)N;
    hipLaunchKernelGGL(split_b_bf16, dim3((unsigned)cdiv(ldk, 32), (unsigned)cdiv(N, 32)), dim3(256), 0, s, K, N,
                       B, ldb, tb ? 1 : 0, ldk, hi, lo);
    NYS_CHECK_LAUNCH();
    bs = SplitB{hi, lo, ldk};
    scratch_elems = off;
  }
  return gemm_bf16x3_run(ta, tb, M, N, K, alpha, A, lda, B, ldb, bs, beta, C, ldc, scratch, scratch_elems, s);
}

}  // namespace nys
