// Reduced-precision Gaussian-kernel products on MFMA (gfx950).
//
// K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) is evaluated tile by tile and
// never stored (kernel ridge regression operator).  The Gram entries x_i^T x_j
// come from MFMA in one of two modes:
//   * BF16X3: each coordinate is split into bf16 hi + lo parts (round to
//     nearest even) and x^T y ~ hi.hi + hi.lo + lo.hi, three
//     v_mfma_f32_16x16x32_bf16 per 16 x 16 tile, float32 accumulation;
//   * F32:    v_mfma_f32_16x16x4f32 on the float32 coordinates.
// With s = log2(e) / (2 sigma^2) and h_i = s ||x_i||^2, the exponent is
// log2 K_ij = 2 s x_i^T x_j - h_i - h_j.  The row term is folded into the
// MFMA accumulator input (C = -h_i / (2 s)), so each kernel entry costs one
// FMA, one v_exp_f32 and one FMA with the vector.  Coordinates are padded to
// 32 (one bf16 MFMA step, eight f32 steps); rows are padded to a multiple of
// 256 with zeros, so operand loads never leave the prepared arrays.  Products
// with one vector evaluate each pair of point super-blocks once (K is
// symmetric: its rows and its columns both serve), block products every tile.
#include "rbf_lowp.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

namespace nys {

namespace {

// True when every column c0 .. c0 + nc - 1 (below k) is flagged in done
// (uniform across the block: every thread reads the same flags).
__device__ __forceinline__ bool cols_done(const int* __restrict__ done, int64_t c0, int nc, int64_t k) {
  if (!done) return false;
  for (int64_t c = c0; c < c0 + nc && c < k; ++c)
    if (!done[c]) return false;
  return true;
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// float -> bf16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Xhi, Xlo: npad x 32 bf16; X32: npad x 32 float; hs[i] = s ||x_i||^2 (float,
// from the float64 norm of the stored coordinates).  Padding rows are zero.
template <typename TD>
__global__ void rbf_prepare(const TD* __restrict__ X, int64_t n, int64_t d, int64_t ld, int64_t npad, double s,
                            unsigned short* __restrict__ Xhi, unsigned short* __restrict__ Xlo,
                            float* __restrict__ X32, float* __restrict__ hs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  double nrm = 0.0;
  for (int k = 0; k < 32; ++k) {
    const double v = (i < n && k < d) ? double(X[i * ld + k]) : 0.0;
    nrm += v * v;
    const float f = (float)v;
    const unsigned short hi = bf16_rne(f);
    const unsigned short lo = bf16_rne(f - bf16_to_f(hi));
    Xhi[i * 32 + k] = hi;
    Xlo[i * 32 + k] = lo;
    X32[i * 32 + k] = f;
  }
  hs[i] = (float)(s * nrm);
}

template <int MODE>
struct Operand;

// BF16X3: lane l holds row (l % 16), coordinates 8 (l / 16) .. + 7
template <>
struct Operand<0> {
  bf8 hi, lo;
  __device__ __forceinline__ void load(const RbfLowp& L, int64_t row, int lane) {
    const int64_t off = row * 32 + 8 * (lane >> 4);
    hi = *reinterpret_cast<const bf8*>(L.Xhi + off);
    lo = *reinterpret_cast<const bf8*>(L.Xlo + off);
  }
};
// F32: lane l holds row (l % 16), coordinates 4 ks + l / 16 for ks = 0..7
// (the loads of the groups a kernel's Gram does not use are dead code)
template <>
struct Operand<1> {
  float v[8];
  __device__ __forceinline__ void load(const RbfLowp& L, int64_t row, int lane) {
    const float* p = L.X32 + row * 32 + (lane >> 4);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) v[ks] = p[4 * ks];
  }
};

// D = A B^T + C for one 16 x 16 tile (rows of a, points of b).
__device__ __forceinline__ f4 gram_tile(const Operand<0>& a, const Operand<0>& b, f4 c) {
  f4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, d, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, d, 0, 0, 0);
}
// (float32: the first KS coordinate groups, KS a compile-time count that
// covers d, so the MFMA chain is straight-line code; operand registers of the
// groups beyond KS are never loaded)
template <int KS>
__device__ __forceinline__ f4 gram_tile(const Operand<1>& a, const Operand<1>& b, f4 c) {
  f4 d = c;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[ks], b.v[ks], d, 0, 0, 0);
  return d;
}
template <int KS>
__device__ __forceinline__ f4 gram_tile(const Operand<0>& a, const Operand<0>& b, f4 c) {
  return gram_tile(a, b, c);
}
// float32 Gram steps for d coordinates: 2, 4 or 8 groups of four (the padded
// coordinates are zero); the bf16x3 Gram always takes one 32-wide step
__host__ __device__ constexpr int ks_for(int ksteps) { return ksteps <= 2 ? 2 : ksteps <= 4 ? 4 : 8; }

// One vector, every entry evaluated (the form for n past the symmetric
// form's 256 partial slots): part[split][i] = sum_{j in split} K_ij p_j.  Block = 4 waves,
// wave w owns rows rb*256 + w*64 .. + 63 (four 16-row fragments); the lanes
// of a wave walk the points of the split 16 at a time.  Accumulator element
// q of lane l belongs to row 4 (l/16) + q of a fragment and column l % 16.
template <int MODE, int KS>
__global__ __launch_bounds__(256) void rbf_mv_lowp(RbfLowp L, const float* __restrict__ p, float* __restrict__ part,
                                                   int64_t pts_per_split, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = L.n;
  const int64_t row0 = (int64_t)blockIdx.x * 256 + wave * 64;
  const float two_s = L.two_s;
  Operand<MODE> a[4];
  f4 cinit[4], acc[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    a[f].load(L, row0 + f * 16 + (lane & 15), lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cinit[f][q] = -L.hs[row0 + f * 16 + 4 * (lane >> 4) + q] / two_s;
      acc[f][q] = 0.0f;
    }
  }
  const int64_t j0 = (int64_t)blockIdx.y * pts_per_split;
  int64_t j1 = j0 + pts_per_split;
  if (j1 > n) j1 = n;
  for (int64_t jt = j0; jt < j1; jt += 16) {
    const int64_t j = jt + (lane & 15);
    Operand<MODE> b;
    b.load(L, j, lane);  // rows beyond n are zero padding
    const float hj = L.hs[j];
    const float pj = (j < j1) ? p[j] : 0.0f;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const f4 dg = gram_tile<KS>(a[f], b, cinit[f]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e = __builtin_amdgcn_exp2f(fmaf(two_s, dg[q], -hj));
        acc[f][q] = fmaf(e, pj, acc[f][q]);
      }
    }
  }
  // sum over the 16 columns held by lanes with the same l / 16
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v = acc[f][q];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      const int64_t row = row0 + f * 16 + 4 * (lane >> 4) + q;
      if ((lane & 15) == 0 && row < n) part[(int64_t)blockIdx.y * n + row] = v;
    }
}

// One vector using the symmetry of K: the points are cut into super-blocks of
// 256 cb (cb <= kSymCb) and workgroup (I, J), I <= J, evaluates the tile K_IJ
// once.  Its rows give part[J][i] = sum_{j in J} K_ij p_j for i in I, and for
// I < J its columns give part[I][j] = sum_{i in I} K_ij p_i for j in J, so
// every slot part[Y][x] is written by exactly one workgroup and
// (K p)[x] = sum_{Y < nsb} part[Y][x]: half the exponentials of the plain
// form.  Waves take 64 rows of a 256-row sub-block of I as in rbf_mv_lowp;
// each wave adds its column sums into its own LDS row, and the four rows are
// added in a fixed order at the end (deterministic).
constexpr int kSymCb = 8;
#ifndef NYS_SYM_NSB
#define NYS_SYM_NSB 128
#endif
template <int MODE, int KS>
__global__ __launch_bounds__(256) void rbf_mv_lowp_sym(RbfLowp L, const float* __restrict__ p,
                                                       float* __restrict__ part, int nsb, int cb,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ float colsum[4][kSymCb * 256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = L.n, npad = L.npad;
  int I = 0;
  int64_t b = blockIdx.x;
  while (b >= nsb - I) {
    b -= nsb - I;
    ++I;
  }
  const int J = I + (int)b;
  const bool offd = I != J;
  const int64_t bs = (int64_t)cb * 256;
  const int64_t i0 = I * bs, j0 = J * bs;
  const int64_t i1 = i0 + bs < npad ? i0 + bs : npad, j1 = j0 + bs < npad ? j0 + bs : npad;
  const float two_s = L.two_s;
  if (offd)
    for (int x = lane; x < bs; x += 64) colsum[wave][x] = 0.0f;
  for (int64_t rb = i0; rb < i1; rb += 256) {
    const int64_t row0 = rb + wave * 64;
    Operand<MODE> a[4];
    f4 cinit[4], acc[4];
    float prow[4][4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      a[f].load(L, row0 + f * 16 + (lane & 15), lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = row0 + f * 16 + 4 * (lane >> 4) + q;
        cinit[f][q] = -L.hs[row] / two_s;
        acc[f][q] = 0.0f;
        prow[f][q] = row < n ? p[row] : 0.0f;
      }
    }
    for (int64_t jt = j0; jt < j1; jt += 16) {
      const int64_t j = jt + (lane & 15);
      Operand<MODE> bo;
      bo.load(L, j, lane);  // rows beyond n are zero padding
      const float hj = L.hs[j];
      const float pj = (j < n) ? p[j] : 0.0f;
      float cs = 0.0f;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const f4 dg = gram_tile<KS>(a[f], bo, cinit[f]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float e = __builtin_amdgcn_exp2f(fmaf(two_s, dg[q], -hj));
          acc[f][q] = fmaf(e, pj, acc[f][q]);
          cs = fmaf(e, prow[f][q], cs);
        }
      }
      if (offd) {
        // column l % 16 of the wave's 64 rows: add the four lane groups
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        if (lane < 16) colsum[wave][jt - j0 + lane] += cs;
      }
    }
    // rows: sum over the 16 columns held by lanes with the same l / 16
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v = acc[f][q];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        const int64_t row = row0 + f * 16 + 4 * (lane >> 4) + q;
        if ((lane & 15) == 0 && row < n) part[(int64_t)J * n + row] = v;
      }
  }
  if (offd) {
    __syncthreads();
    for (int64_t x = threadIdx.x; x < j1 - j0; x += 256)
      if (j0 + x < n)
        part[(int64_t)I * n + j0 + x] = (colsum[0][x] + colsum[1][x]) + (colsum[2][x] + colsum[3][x]);
  }
}

// Block of columns: V[I, cb*64 .. +63] = scale * K_IJ P_J (+ mu_c P) over all J,
// float32.  Block = 4 waves, 64 rows x 64 output columns; per point tile of
// 32: stage 1 forms K (64 x 32, wave w rows w*16..) with the Gram MFMA and
// exp, splits it into bf16 hi/lo in LDS; stage 2 multiplies K (hi/lo) by the
// P tile (hi/lo, staged transposed in LDS) with three bf16 MFMAs per tile.
template <int MODE, int CF, int FR>
struct KvStage2;

// BF16X3 second stage: K and P split into bf16 hi/lo in LDS, three bf16 MFMAs.
// FR row fragments of 16 per wave: every P fragment read from LDS serves FR
// MFMA chains, which halves the LDS reads per MFMA at FR = 2.
template <int CF, int FR>
struct KvStage2<0, CF, FR> {
  unsigned short Khi[64 * FR][40], Klo[64 * FR][40];  // [row][point]
  unsigned short Phi[16 * CF][40], Plo[16 * CF][40];  // [col][point]
  // 8 points (part) of column cc, already split (piece 0: hi, 1: lo)
  __device__ __forceinline__ void put_p16(int piece, int cc, int part, uint4 v) {
    *reinterpret_cast<uint4*>(piece ? &Plo[cc][8 * part] : &Phi[cc][8 * part]) = v;
  }
  __device__ __forceinline__ void put_k(int r, int pc, float e) {
    const unsigned short hi = bf16_rne(e);
    Khi[r][pc] = hi;
    Klo[r][pc] = bf16_rne(e - bf16_to_f(hi));
  }
  __device__ __forceinline__ void mac(int wave, int lane, f4 (&acc)[FR][CF]) {
    bf8 khi[FR], klo[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f) {
      const int r = wave * 16 * FR + f * 16 + (lane & 15);
      khi[f] = *reinterpret_cast<const bf8*>(&Khi[r][8 * (lane >> 4)]);
      klo[f] = *reinterpret_cast<const bf8*>(&Klo[r][8 * (lane >> 4)]);
    }
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) {
      const int cc = cf * 16 + (lane & 15);
      const bf8 phi = *reinterpret_cast<const bf8*>(&Phi[cc][8 * (lane >> 4)]);
      const bf8 plo = *reinterpret_cast<const bf8*>(&Plo[cc][8 * (lane >> 4)]);
#pragma unroll
      for (int f = 0; f < FR; ++f) {
        acc[f][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(khi[f], phi, acc[f][cf], 0, 0, 0);
        acc[f][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(khi[f], plo, acc[f][cf], 0, 0, 0);
        acc[f][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(klo[f], phi, acc[f][cf], 0, 0, 0);
      }
    }
  }
};
// F32 second stage: K and P each split exactly into three bf16 pieces
// (8 + 8 + 8 significant bits = the float32 significand), and K P formed from
// all nine piece products with v_mfma_f32_16x16x32_bf16 and float32
// accumulation: every piece product is exact, so the result carries the
// rounding of a float32 product (the same class as v_mfma_f32_16x16x4f32)
// at 9 x 16 instead of 8 x 32 MFMA cycles per 16 x 16 x 32 step.
__device__ __forceinline__ void split3(float v, unsigned short& h0, unsigned short& h1, unsigned short& h2) {
  h0 = bf16_rne(v);
  const float r1 = v - bf16_to_f(h0);
  h1 = bf16_rne(r1);
  h2 = bf16_rne(r1 - bf16_to_f(h1));
}

// Float32 second stage: K and P each split into three exact bf16 pieces (nine
// piece products, smallest first).  FR as above.
template <int CF, int FR>
struct KvStage2<1, CF, FR> {
  unsigned short Kp[3][64 * FR][40];  // [piece][row][point]
  unsigned short Pp[3][16 * CF][40];  // [piece][col][point]
  __device__ __forceinline__ void put_p16(int piece, int cc, int part, uint4 v) {
    *reinterpret_cast<uint4*>(&Pp[piece][cc][8 * part]) = v;
  }
  __device__ __forceinline__ void put_k(int r, int pc, float e) {
    unsigned short h0, h1, h2;
    split3(e, h0, h1, h2);
    Kp[0][r][pc] = h0;
    Kp[1][r][pc] = h1;
    Kp[2][r][pc] = h2;
  }
  __device__ __forceinline__ void mac(int wave, int lane, f4 (&acc)[FR][CF]) {
    bf8 kk[FR][3];
#pragma unroll
    for (int f = 0; f < FR; ++f) {
      const int r = wave * 16 * FR + f * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 3; ++q) kk[f][q] = *reinterpret_cast<const bf8*>(&Kp[q][r][8 * (lane >> 4)]);
    }
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) {
      const int cc = cf * 16 + (lane & 15);
      bf8 pp[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) pp[q] = *reinterpret_cast<const bf8*>(&Pp[q][cc][8 * (lane >> 4)]);
#pragma unroll
      for (int f = 0; f < FR; ++f) {
        f4 c = acc[f][cf];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][2], pp[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][1], pp[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][2], pp[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][0], pp[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][1], pp[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][2], pp[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][0], pp[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][1], pp[0], c, 0, 0, 0);
        acc[f][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kk[f][0], pp[0], c, 0, 0, 0);
      }
    }
  }
};

// Storage position of point jj (0..31) of a 32-point step in the register
// kernel's order: position 8 g + t holds point 4 g + t (t < 4) or
// 16 + 4 g + t - 4 (t >= 4), the points lane group g holds after the
// transposed Gram tiles.
__device__ __forceinline__ int kv_perm(int jj) { return 8 * ((jj & 15) >> 2) + 4 * (jj >> 4) + (jj & 3); }

// P (n x k float, row-major) -> NP bf16 pieces (2: hi, lo; 3: the exact
// three-piece split), transposed: Pq[piece][c][j] for c < kq, j < npad (zero
// outside n x k), so a tile's 8-point runs of one column are 16-byte chunks.
// 32 x 32 tiles through LDS.
template <int NP, bool PERM>
__global__ __launch_bounds__(256) void split_p_bf16(const float* __restrict__ P, int64_t ldp, int64_t n,
                                                    int64_t k, int64_t kq, int64_t npad,
                                                    unsigned short* __restrict__ Pq) {
  __shared__ float tl[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t j0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = j0 + ty + 8 * u, c = c0 + tx;
    tl[ty + 8 * u][tx] = (j < n && c < k) ? P[j * ldp + c] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t c = c0 + ty + 8 * u;
    const int64_t j = j0 + (PERM ? kv_perm(tx) : tx);
    if (c < kq && j < npad) {
      const float v = tl[tx][ty + 8 * u];
      if (NP == 2) {
        const unsigned short hi = bf16_rne(v);
        Pq[c * npad + j] = hi;
        Pq[(kq + c) * npad + j] = bf16_rne(v - bf16_to_f(hi));
      } else {
        unsigned short h0, h1, h2;
        split3(v, h0, h1, h2);
        Pq[c * npad + j] = h0;
        Pq[(kq + c) * npad + j] = h1;
        Pq[(2 * kq + c) * npad + j] = h2;
      }
    }
  }
}

// Block of columns: V[I, cb*16CF .. +16CF-1] = oscale * K_IJ P_J over the points
// of split z, float32.  Block = 4 waves, 64 rows x 16 CF output columns; per
// point tile of 32: stage 1 forms K (wave w: rows w*16 .. +15) with the Gram
// MFMA and exp into LDS; stage 2 multiplies K by the P tile staged in LDS.
// The P tile and the point operands of the next tile are loaded into
// registers while the current tile is multiplied.
template <int MODE, int CF, int KS, int FR>
__global__ __launch_bounds__(256) void rbf_kv_lowp(RbfLowp L, const float* __restrict__ P, int64_t ldp, int64_t k,
                                                   const uint4* __restrict__ Pq, int64_t ldq,
                                                   float* __restrict__ out, int64_t ldo, int64_t pts_per_split,
                                                   float oscale, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int NC = 16 * CF;               // output columns of the block
  // P tile per thread: 16-byte chunks (8 points of one column) of the
  // pre-split bf16 pieces, NPC pieces (MODE 0: hi / lo; MODE 1: three)
  constexpr int NPC = MODE == 0 ? 2 : 3;
  constexpr int PE = NPC * NC * 4 / 256;
  __shared__ __attribute__((aligned(16))) KvStage2<MODE, CF, FR> st;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = L.n;
  const int64_t i0 = (int64_t)blockIdx.x * 64 * FR;  // wave w: rows i0 + 16 FR w .. + 16 FR - 1
  const int64_t c0 = (int64_t)blockIdx.y * NC;
  const bool dead = cols_done(L.coldone, c0, NC, k);  // zeros out, no products
  const float two_s = L.two_s;
  Operand<MODE> a[FR];
  f4 cinit[FR];
#pragma unroll
  for (int f = 0; f < FR; ++f) {
    const int64_t rb = i0 + wave * 16 * FR + f * 16;
    a[f].load(L, rb + (lane & 15), lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) cinit[f][q] = -L.hs[rb + 4 * (lane >> 4) + q] / two_s;
  }
  f4 acc[FR][CF];
#pragma unroll
  for (int f = 0; f < FR; ++f)
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) acc[f][cf] = f4{0, 0, 0, 0};
  const int64_t j0 = (int64_t)blockIdx.z * pts_per_split;
  int64_t j1 = j0 + pts_per_split;
  if (j1 > n) j1 = n;
  if (dead) j1 = j0;
  // registers for the next tile: P entries and the two 16-point operands
  uint4 pr[PE];
  Operand<MODE> b0, b1;
  float h0 = 0.0f, h1 = 0.0f;
  auto fetch = [&](int64_t jt) {
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = t + 256 * u;
      // chunk (piece, column, part): Pq holds [piece][column][point / 8], ldq chunks per column
      const int part = e & 3, cc = (e >> 2) % NC, piece = (e >> 2) / NC;
      pr[u] = Pq[((int64_t)piece * L.kq + c0 + cc) * ldq + (jt >> 3) + part];
    }
    // rows jt .. jt + 31 lie inside the padded operand arrays (jt < n, npad a multiple of 256)
    b0.load(L, jt + (lane & 15), lane);
    b1.load(L, jt + 16 + (lane & 15), lane);
    h0 = L.hs[jt + (lane & 15)];
    h1 = L.hs[jt + 16 + (lane & 15)];
  };
  if (j0 < j1) fetch(j0);
  for (int64_t jt = j0; jt < j1; jt += 32) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = t + 256 * u;
      st.put_p16((e >> 2) / NC, (e >> 2) % NC, e & 3, pr[u]);
    }
    // stage 1: K rows of each fragment, points jt .. jt+31 (two 16-point tiles)
    const int64_t ja = jt + (lane & 15), jb = jt + 16 + (lane & 15);
#pragma unroll
    for (int f = 0; f < FR; ++f) {
      const f4 dg0 = gram_tile<KS>(a[f], b0, cinit[f]);
      const f4 dg1 = gram_tile<KS>(a[f], b1, cinit[f]);
      const int rl = wave * 16 * FR + f * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e0 = (ja < j1) ? __builtin_amdgcn_exp2f(fmaf(two_s, dg0[q], -h0)) : 0.0f;
        const float e1 = (jb < j1) ? __builtin_amdgcn_exp2f(fmaf(two_s, dg1[q], -h1)) : 0.0f;
        st.put_k(rl + q, (lane & 15), e0);
        st.put_k(rl + q, 16 + (lane & 15), e1);
      }
    }
    __syncthreads();
    if (jt + 32 < j1) fetch(jt + 32);  // in flight during stage 2
    st.mac(wave, lane, acc);
  }
  float* o = out + (int64_t)blockIdx.z * n * ldo;
#pragma unroll
  for (int f = 0; f < FR; ++f)
#pragma unroll
    for (int cf = 0; cf < CF; ++cf)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = i0 + wave * 16 * FR + f * 16 + 4 * (lane >> 4) + q;
        const int64_t col = c0 + cf * 16 + (lane & 15);
        if (row < n && col < k) o[row * ldo + col] = oscale * acc[f][cf][q];
      }
}

// Float32 mode, few columns (k <= 64): out[I, c0 .. c0 + 16 CF - 1] =
// oscale * K_IJ P_J over the points of split z, in registers only.  Each wave owns F fragments of 16
// rows and walks the points 16 at a time.  The Gram tile is formed transposed
// (points as the MFMA row index, rows as the column index), so lane l holds
// K[point 4 (l/16) + q][row l % 16] for q = 0..3: for each q this is exactly
// the B operand of v_mfma_f32_16x16x4f32 over the four points {4 g + q}, and
// the matching A operand is P[point 4 g + q][column l % 16].  K P is therefore
// four float32 MFMAs per 16 x 16 tile and 16 columns, with no LDS, no barrier
// and no conversion of K.  Pz: P copied to npad x kq floats, zero outside
// n x k (so tail points and columns contribute exact zeros).
template <int CF, int F, int KS>
__global__ __launch_bounds__(256) void rbf_kv_reg32(RbfLowp L, const float* __restrict__ Pz, int64_t kq, int64_t k,
                                                  float* __restrict__ out, int64_t ldo, int64_t pts_per_split,
                                                  float oscale, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t n = L.n;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * F);
  const int64_t c0 = (int64_t)blockIdx.y * (16 * CF);
  const float two_s = L.two_s;
  // rows i0 + 16 f + r: operands and the row term folded into the accumulator
  Operand<1> a[F];
  f4 crow[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    a[f].load(L, i0 + 16 * f + r, lane);
    const float c = -L.hs[i0 + 16 * f + r] / two_s;
    crow[f] = f4{c, c, c, c};
  }
  f4 acc[F][CF];
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) acc[f][cf] = f4{0, 0, 0, 0};
  const int64_t j0 = (int64_t)blockIdx.z * pts_per_split;
  int64_t j1 = j0 + pts_per_split;
  if (j1 > n) j1 = n;
  if (cols_done(L.coldone, c0, 16 * CF, k)) j1 = j0;  // zeros out, no products
  for (int64_t jt = j0; jt < j1; jt += 16) {
    // points jt .. jt + 15 lie inside the padded arrays (jt < n, npad a multiple of 256)
    Operand<1> b;
    b.load(L, jt + r, lane);
    const f4 hj = *reinterpret_cast<const f4*>(L.hs + jt + 4 * g);
    float pv[CF][4];
#pragma unroll
    for (int cf = 0; cf < CF; ++cf)
#pragma unroll
      for (int q = 0; q < 4; ++q) pv[cf][q] = Pz[(jt + 4 * g + q) * kq + c0 + 16 * cf + r];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const f4 dg = gram_tile<KS>(b, a[f], crow[f]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e = __builtin_amdgcn_exp2f(fmaf(two_s, dg[q], -hj[q]));
#pragma unroll
        for (int cf = 0; cf < CF; ++cf)
          acc[f][cf] = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[cf][q], e, acc[f][cf], 0, 0, 0);
      }
    }
  }
  // lane l holds out[row 16 f + l % 16][column 16 cf + 4 (l / 16) + q]
  float* o = out + (int64_t)blockIdx.z * n * ldo;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t row = i0 + 16 * f + r;
    if (row >= n) continue;
#pragma unroll
    for (int cf = 0; cf < CF; ++cf)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = c0 + 16 * cf + 4 * g + q;
        if (col < k) o[row * ldo + col] = oscale * acc[f][cf][q];
      }
  }
}

// Pz[j][c] = P[j][c] for j < n, c < k; zero elsewhere (npad x kq)
__global__ void pad_p(const float* __restrict__ P, int64_t ldp, int64_t n, int64_t k, int64_t npad, int64_t kq,
                      float* __restrict__ Pz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npad * kq) return;
  const int64_t j = idx / kq, c = idx % kq;
  Pz[idx] = (j < n && c < k) ? P[j * ldp + c] : 0.0f;
}

// bf16x3 mode, few columns (k <= 64), in registers only:
// out[I, c0 .. c0 + 16 CF - 1] = oscale * K_IJ P_J over the points of split z.  Each wave owns F fragments of 16 rows and walks the
// points 32 at a time.  The Gram tiles are formed transposed (points as the
// MFMA row index, rows as the column index), so after the exp lane l holds
// K[point 4 g + q][row l % 16] and K[point 16 + 4 g + q][row l % 16],
// g = l / 16, q = 0..3.  These eight values are the lane's k-slice of the B
// operand of v_mfma_f32_16x16x32_bf16 when the 32 points of the step are taken
// in the order of kv_perm below; P is pre-split into bf16 pieces stored in
// that order (split_p_bf16 with PERM), so the A operand (P transposed) is one
// 16-byte load per piece.  K is split into bf16 hi + lo in registers and
// K P ~ hi.hi + hi.lo + lo.hi (three MFMAs per 32 points and 16 columns), as
// in the LDS kernel's bf16x3 mode.  No LDS, no barrier, float32 accumulation.
// (For the float32 mode the three-piece split of K costs more VALU time than
// the float32 MFMAs it saves: rbf_kv_reg32 above multiplies K unsplit.)
__device__ __forceinline__ void split_k(const float (&e)[8], bf8 (&kb)[2]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 h = (__bf16)e[t];
    kb[0][t] = h;
    kb[1][t] = (__bf16)(e[t] - (float)h);
  }
}
// acc += P^T K over one 32-point step (A: P pieces, B: K pieces), smallest first
__device__ __forceinline__ f4 kp_products(const bf8 (&pp)[2], const bf8 (&kb)[2], f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pp[1], kb[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pp[0], kb[1], c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(pp[0], kb[0], c, 0, 0, 0);
}
template <int CF, int F>
__global__ __launch_bounds__(256) void rbf_kv_reg(RbfLowp L, const uint4* __restrict__ Pq, int64_t ldq, int64_t k,
                                                  float* __restrict__ out, int64_t ldo, int64_t pts_per_split,
                                                  float oscale, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int NP = 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t n = L.n;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * F);
  const int64_t c0 = (int64_t)blockIdx.y * (16 * CF);
  const float two_s = L.two_s;
  // rows i0 + 16 f + r: operands and the row term folded into the accumulator
  Operand<0> a[F];
  f4 crow[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    a[f].load(L, i0 + 16 * f + r, lane);
    const float c = -L.hs[i0 + 16 * f + r] / two_s;
    crow[f] = f4{c, c, c, c};
  }
  f4 acc[F][CF];
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) acc[f][cf] = f4{0, 0, 0, 0};
  const int64_t j0 = (int64_t)blockIdx.z * pts_per_split;
  int64_t j1 = j0 + pts_per_split;
  if (j1 > n) j1 = n;
  if (cols_done(L.coldone, c0, 16 * CF, k)) j1 = j0;  // zeros out, no products
  for (int64_t jt = j0; jt < j1; jt += 32) {
    // points jt .. jt + 31 lie inside the padded arrays (jt < n, npad a
    // multiple of 256); P pieces are zero for points >= n
    Operand<0> b0, b1;
    b0.load(L, jt + r, lane);
    b1.load(L, jt + 16 + r, lane);
    const f4 h0 = *reinterpret_cast<const f4*>(L.hs + jt + 4 * g);
    const f4 h1 = *reinterpret_cast<const f4*>(L.hs + jt + 16 + 4 * g);
    bf8 kb[F][NP];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const f4 d0 = gram_tile(b0, a[f], crow[f]);
      const f4 d1 = gram_tile(b1, a[f], crow[f]);
      float e[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        e[q] = __builtin_amdgcn_exp2f(fmaf(two_s, d0[q], -h0[q]));
        e[4 + q] = __builtin_amdgcn_exp2f(fmaf(two_s, d1[q], -h1[q]));
      }
      split_k(e, kb[f]);
    }
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) {
      // column c0 + 16 cf + r, positions 8 g .. 8 g + 7 of the step
      bf8 pp[NP];
#pragma unroll
      for (int pc = 0; pc < NP; ++pc)
        pp[pc] = __builtin_bit_cast(bf8, Pq[((int64_t)pc * L.kq + c0 + 16 * cf + r) * ldq + (jt >> 3) + g]);
#pragma unroll
      for (int f = 0; f < F; ++f) acc[f][cf] = kp_products(pp, kb[f], acc[f][cf]);
    }
  }
  // lane l holds out[row 16 f + l % 16][column 16 cf + 4 (l / 16) + q]
  float* o = out + (int64_t)blockIdx.z * n * ldo;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t row = i0 + 16 * f + r;
    if (row >= n) continue;
#pragma unroll
    for (int cf = 0; cf < CF; ++cf)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = c0 + 16 * cf + 4 * g + q;
        if (col < k) o[row * ldo + col] = oscale * acc[f][cf][q];
      }
  }
}

// V = scale * sum_z part[z] + mu_c P  (n x k float), fixed order over z
__global__ void rbf_lowp_finish(const float* __restrict__ part, int nz, int64_t n, int64_t k, float scale,
                                const float* __restrict__ P, int64_t ldp, const double* __restrict__ mu,
                                int64_t nrhs, float* __restrict__ V, int64_t ldv, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  float s = 0.0f;
  for (int z = 0; z < nz; ++z) s += part[((int64_t)z * n + i) * k + c];
  s *= scale;
  if (mu) s += float(mu[c / nrhs]) * P[i * ldp + c];
  V[i * ldv + c] = s;
}

}  // namespace

size_t rbf_lowp_bytes(int64_t n) {
  const int64_t npad = cdiv(n, 256) * 256;
  return (size_t)npad * 32 * (2 + 2 + 4) + (size_t)npad * 4 + 1024;
}

nys_status rbf_lowp_prepare(const OpDesc& op, void* buf, RbfLowp& L, hipStream_t s) {
  const int64_t n = op.n, d = op.cols;
  if (d > 32) {
    set_error("reduced-precision RBF path supports d <= 32 (got %lld)", (long long)d);
    return NYS_ERR_ARG;
  }
  const int64_t npad = cdiv(n, 256) * 256;
  char* b = static_cast<char*>(buf);
  L.n = n;
  L.npad = npad;
  L.Xhi = reinterpret_cast<unsigned short*>(b);
  L.Xlo = L.Xhi + npad * 32;
  L.X32 = reinterpret_cast<float*>(L.Xlo + npad * 32);
  L.hs = L.X32 + npad * 32;
  const double sc = 1.4426950408889634 / (2.0 * op.sigma * op.sigma);  // log2(e) / (2 sigma^2)
  L.two_s = (float)(2.0 * sc);
  L.scale = (float)op.scale;
  L.ksteps = (int)cdiv(d, (int64_t)4);
  L.d = (int)d;
  L.kq = 0;
  L.coldone = nullptr;
  if (op.dtype == NYS_F64)
    hipLaunchKernelGGL(rbf_prepare<double>, dim3((unsigned)cdiv(npad, 256)), dim3(256), 0, s,
                       static_cast<const double*>(op.data), n, d, op.ld, npad, sc, L.Xhi, L.Xlo, L.X32, L.hs);
  else
    hipLaunchKernelGGL(rbf_prepare<float>, dim3((unsigned)cdiv(npad, 256)), dim3(256), 0, s,
                       static_cast<const float*>(op.data), n, d, op.ld, npad, sc, L.Xhi, L.Xlo, L.X32, L.hs);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

nys_status rbf_lowp_mv_partials(const RbfLowp& L, int mode, const float* p, float* part, size_t part_elems,
                                int* ng_out, const int* skip, hipStream_t s) {
  const int64_t n = L.n;
  // symmetric form: super-blocks of 256 cb points, about NYS_SYM_NSB of them
  // (at most 256 partial slots; larger n keeps the plain form, whose slots
  // stay few)
  {
    const int64_t nb256 = cdiv(L.npad, 256);
    int64_t cb = cdiv(nb256, NYS_SYM_NSB);
    if (cb < 1) cb = 1;
    if (cb > kSymCb) cb = kSymCb;
    const int64_t nsb = cdiv(nb256, cb);
    if (nsb <= 256 && (size_t)(nsb * n) <= part_elems) {
      const unsigned pairs = (unsigned)(nsb * (nsb + 1) / 2);
      if (mode == 0)
        hipLaunchKernelGGL((rbf_mv_lowp_sym<0, 1>), dim3(pairs), dim3(256), 0, s, L, p, part, (int)nsb, (int)cb,
                           skip);
      else
        switch (ks_for(L.ksteps)) {
          case 2:
            hipLaunchKernelGGL((rbf_mv_lowp_sym<1, 2>), dim3(pairs), dim3(256), 0, s, L, p, part, (int)nsb, (int)cb,
                               skip);
            break;
          case 4:
            hipLaunchKernelGGL((rbf_mv_lowp_sym<1, 4>), dim3(pairs), dim3(256), 0, s, L, p, part, (int)nsb, (int)cb,
                               skip);
            break;
          default:
            hipLaunchKernelGGL((rbf_mv_lowp_sym<1, 8>), dim3(pairs), dim3(256), 0, s, L, p, part, (int)nsb, (int)cb,
                               skip);
            break;
        }
      NYS_CHECK_LAUNCH();
      *ng_out = (int)nsb;
      return NYS_OK;
    }
  }
  const int64_t nrb = cdiv(n, 256);
  const int cus = num_cus() < 256 ? num_cus() : 256;
  int64_t ns = cdiv(8 * cus, nrb);  // about eight blocks per compute unit
  if (ns < 1) ns = 1;
  while (ns > 1 && (size_t)(ns * n) > part_elems) --ns;
  const int64_t pps = cdiv(cdiv(n, ns), 16) * 16;
  ns = cdiv(n, pps);
  dim3 grid((unsigned)nrb, (unsigned)ns);
  if (mode == 0)
    hipLaunchKernelGGL((rbf_mv_lowp<0, 1>), grid, dim3(256), 0, s, L, p, part, pps, skip);
  else
    switch (ks_for(L.ksteps)) {
      case 2: hipLaunchKernelGGL((rbf_mv_lowp<1, 2>), grid, dim3(256), 0, s, L, p, part, pps, skip); break;
      case 4: hipLaunchKernelGGL((rbf_mv_lowp<1, 4>), grid, dim3(256), 0, s, L, p, part, pps, skip); break;
      default: hipLaunchKernelGGL((rbf_mv_lowp<1, 8>), grid, dim3(256), 0, s, L, p, part, pps, skip); break;
    }
  NYS_CHECK_LAUNCH();
  *ng_out = (int)ns;
  return NYS_OK;
}

nys_status rbf_lowp_mv(const RbfLowp& L, int mode, const float* p, const double* mu_dev, float* v, float* part,
                       size_t part_elems, hipStream_t s) {
  int ns = 0;
  NYS_TRY(rbf_lowp_mv_partials(L, mode, p, part, part_elems, &ns, nullptr, s));
  hipLaunchKernelGGL(rbf_lowp_finish, dim3((unsigned)cdiv(L.n, 256)), dim3(256), 0, s, part, ns, L.n, (int64_t)1,
                     L.scale, p, (int64_t)1, mu_dev, (int64_t)1, v, (int64_t)1, (const int*)nullptr);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Launch plan of V = K P.  k <= 64: a register kernel with 16 CF columns and
// 4 waves x 16 F rows per block (bf16x3 mode: rbf_kv_reg on P pre-split in
// the point order of a step; float32 mode: rbf_kv_reg32 on P zero-padded to
// npad x kq floats).  k > 64: the LDS kernel, 64 rows x 128 columns per
// block, P pre-split into bf16 pieces.
struct KvPlan {
  bool reg;
  int cf, f, bpc;
  int64_t nc, kq, rows, tiles;
  size_t prep_elems;  // float elements of the prepared P
};

// The built-in choice: register kernel up to 64 columns (one, two or four
// 16-column tiles), the LDS kernel past that (256 columns per block past 128
// columns: half the Gram / exp / split work per column), about eight
// workgroups per compute unit.
KvChoice kv_heuristic(int64_t k) {
  KvChoice c{};
  c.reg = k <= 64 ? 1 : 0;
  // past 64 columns: the LDS kernel with 128 rows and 128 columns per
  // workgroup, the shape the autotuner picks for both Gram modes at
  // n = 5e4 .. 1e5 (k = 128 .. 1000)
  c.cf = c.reg ? (k <= 16 ? 1 : k <= 32 ? 2 : 4) : 8;
  c.bpc = 8;
  c.fr = c.reg ? 1 : 2;
  return c;
}

KvPlan make_plan(int64_t n, int64_t k, int mode, KvChoice c) {
  KvPlan p{};
  const int64_t npad = cdiv(n, 256) * 256;
  p.reg = c.reg != 0;
  p.cf = c.cf;
  p.bpc = c.bpc;
  if (p.reg) {
    p.f = mode == RBF_GRAM_F32 && p.cf < 4 ? 4 : 2;
    p.nc = 16 * p.cf;
    p.rows = 64 * p.f;
  } else {
    p.f = c.fr == 2 ? 2 : 1;  // row fragments per wave
    p.nc = 16 * p.cf;
    p.rows = 64 * p.f;
  }
  p.kq = cdiv(k, p.nc) * p.nc;
  p.tiles = cdiv(n, p.rows) * cdiv(k, p.nc);
  if (p.reg && mode == RBF_GRAM_F32)
    p.prep_elems = (size_t)npad * (size_t)p.kq;
  else
    p.prep_elems = (mode == RBF_GRAM_F32 ? 3 : 2) * (size_t)p.kq * (size_t)npad / 2;
  return p;
}

// Every choice the autotuner times (and that a tuned table may name).
std::vector<KvChoice> kv_candidates() {
  std::vector<KvChoice> v;
  const int regcf[3] = {1, 2, 4}, ldscf[2] = {8, 16}, bpcs[3] = {4, 8, 16};
  for (int b : bpcs) {
    for (int cf : regcf) v.push_back(KvChoice{1, cf, b, 1});
    for (int cf : ldscf)
      for (int fr = 1; fr <= 2; ++fr) v.push_back(KvChoice{0, cf, b, fr});
  }
  return v;
}

bool valid_choice(const KvChoice& c) {
  const bool cf_ok = c.reg ? (c.cf == 1 || c.cf == 2 || c.cf == 4) : (c.cf == 8 || c.cf == 16);
  const bool fr_ok = c.reg ? c.fr == 1 : (c.fr == 1 || c.fr == 2);
  return (c.reg == 0 || c.reg == 1) && cf_ok && fr_ok && (c.bpc == 4 || c.bpc == 8 || c.bpc == 16);
}

// ---- autotuner table

struct TuneEntry {
  int64_t n, k;
  int d, mode;
  KvChoice c;
  double us;
};

static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;
static bool g_tune_env_done = false;

// caller holds g_tune_mu
static void tune_put(const TuneEntry& e) {
  for (TuneEntry& t : g_tune)
    if (t.n == e.n && t.k == e.k && t.d == e.d && t.mode == e.mode) {
      t = e;
      return;
    }
  g_tune.push_back(e);
}

// caller holds g_tune_mu
static nys_status tune_load_locked(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) {
    set_error("autotune cache %s cannot be opened", path);
    return NYS_ERR_ARG;
  }
  std::vector<TuneEntry> got;
  char line[512];
  int lineno = 0;
  nys_status st = NYS_OK;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n' || line[0] == '\0') continue;
    TuneEntry e{};
    long long n = 0, k = 0;
    char tag[32] = "";
    e.c.fr = 1;  // lines without the last field: one row fragment per wave
    const int got_n = std::sscanf(line, "%31s %lld %d %d %lld %d %d %d %lf %d", tag, &n, &e.d, &e.mode, &k,
                                  &e.c.reg, &e.c.cf, &e.c.bpc, &e.us, &e.c.fr);
    e.n = n;
    e.k = k;
    if (got_n < 9 || std::strcmp(tag, "rbf_kv") != 0 || n < 1 || k < 1 || e.d < 1 || e.d > 32 ||
        (e.mode != RBF_GRAM_BF16X3 && e.mode != RBF_GRAM_F32) || !valid_choice(e.c)) {
      set_error("autotune cache %s: line %d is not a valid entry", path, lineno);
      st = NYS_ERR_ARG;
      break;
    }
    got.push_back(e);
  }
  std::fclose(f);
  if (st != NYS_OK) return st;
  for (const TuneEntry& e : got) tune_put(e);
  return NYS_OK;
}

static void tune_env_load_locked() {
  if (g_tune_env_done) return;
  g_tune_env_done = true;
  const char* p = std::getenv("NYS_AUTOTUNE_CACHE");
  if (p && *p) {
    FILE* f = std::fopen(p, "r");
    if (f) {
      std::fclose(f);
      (void)tune_load_locked(p);  // an unreadable cache leaves the heuristic in place
    }
  }
}

KvChoice kv_choice(const RbfLowp& L, int64_t k, int mode, bool* tuned) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_env_load_locked();
  const TuneEntry* best = nullptr;
  for (const TuneEntry& t : g_tune)
    if (t.n == L.n && t.d == L.d && t.mode == mode && t.k >= k && (!best || t.k < best->k)) best = &t;
  if (tuned) *tuned = best != nullptr;
  return best ? best->c : kv_heuristic(k);
}

int64_t kv_tune_entries() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return (int64_t)g_tune.size();
}

void kv_tune_clear() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  g_tune_env_done = true;  // a cleared table stays empty until loaded again
}

nys_status kv_tune_load(const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return tune_load_locked(path);
}

nys_status kv_tune_save(const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) {
    set_error("autotune cache %s cannot be written", path);
    return NYS_ERR_ARG;
  }
  std::fprintf(f, "# nyspcg autotune cache: rbf_kv n d mode k reg cf bpc microseconds fr\n");
  for (const TuneEntry& t : g_tune)
    std::fprintf(f, "rbf_kv %lld %d %d %lld %d %d %d %.3f %d\n", (long long)t.n, t.d, t.mode, (long long)t.k,
                 t.c.reg, t.c.cf, t.c.bpc, t.us, t.c.fr);
  const bool ok = std::fclose(f) == 0;
  if (!ok) {
    set_error("autotune cache %s: write failed", path);
    return NYS_ERR_ARG;
  }
  return NYS_OK;
}

void kv_tune_env_save() {
  const char* p = std::getenv("NYS_AUTOTUNE_CACHE");
  if (p && *p) (void)kv_tune_save(p);
}

size_t rbf_lowp_kv_scratch(int64_t n, int64_t k) {
  // the largest prepared P over every choice, plus the point-split partial
  // sums at eight workgroups per compute unit (choices that ask for more
  // splits are cut to what the scratch holds)
  size_t m = 0;
  for (int mode = 0; mode < 2; ++mode) {
    size_t prep = 0;
    int64_t tiles_min = 0;
    for (const KvChoice& c : kv_candidates()) {
      const KvPlan p = make_plan(n, k, mode, c);
      prep = p.prep_elems > prep ? p.prep_elems : prep;
      tiles_min = tiles_min == 0 || p.tiles < tiles_min ? p.tiles : tiles_min;
    }
    const int64_t nz = cdiv(8 * 256, tiles_min);
    const size_t e = prep + (nz > 1 ? (size_t)nz * (size_t)n * (size_t)k : 0);
    m = e > m ? e : m;
  }
  return m;
}

// V += mu_c P
__global__ void rbf_lowp_add_mu(int64_t n, int64_t k, const float* __restrict__ P, int64_t ldp,
                                const double* __restrict__ mu, int64_t nrhs, float* __restrict__ V, int64_t ldv,
                                const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  V[i * ldv + c] += float(mu[c / nrhs]) * P[i * ldp + c];
}

nys_status rbf_lowp_kv_plan(const RbfLowp& L, int mode, const KvPlan& pl, const float* P, int64_t ldp, int64_t k,
                            const double* mu_dev, int64_t nrhs, float* V, int64_t ldv, float* scratch,
                            size_t scratch_elems, const int* skip, hipStream_t s);

nys_status rbf_lowp_kv(const RbfLowp& L, int mode, const float* P, int64_t ldp, int64_t k, const double* mu_dev,
                       int64_t nrhs, float* V, int64_t ldv, float* scratch, size_t scratch_elems, const int* skip,
                       hipStream_t s, const int* coldone) {
  const int64_t n = L.n;
  RbfLowp Lc = L;
  Lc.coldone = coldone;
  // with column flags, the shape chosen for 16 columns (blocks of 16 columns
  // at most), so that finished columns free whole blocks
  const KvPlan pl = make_plan(n, k, mode, kv_choice(L, coldone && k > 16 ? 16 : k, mode, nullptr));
  return rbf_lowp_kv_plan(Lc, mode, pl, P, ldp, k, mu_dev, nrhs, V, ldv, scratch, scratch_elems, skip, s);
}

nys_status rbf_lowp_kv_plan(const RbfLowp& L, int mode, const KvPlan& pl, const float* P, int64_t ldp, int64_t k,
                            const double* mu_dev, int64_t nrhs, float* V, int64_t ldv, float* scratch,
                            size_t scratch_elems, const int* skip, hipStream_t s) {
  const int64_t n = L.n;
  const int64_t nc = pl.nc;
  // the kernels read P split once into bf16 pieces (front of the scratch)
  const size_t se = pl.prep_elems;
  if (scratch_elems < se) {
    set_error("rbf_lowp_kv: scratch of %zu floats < %zu", scratch_elems, se);
    return NYS_ERR_WORKSPACE;
  }
  RbfLowp Lq = L;
  Lq.kq = pl.kq;
  const uint4* Pq = reinterpret_cast<const uint4*>(scratch);
  const float* Pz = scratch;
  if (pl.reg && mode == RBF_GRAM_F32) {
    hipLaunchKernelGGL(pad_p, dim3((unsigned)cdiv(L.npad * pl.kq, 256)), dim3(256), 0, s, P, ldp, n, k, L.npad,
                       pl.kq, scratch);
    NYS_CHECK_LAUNCH();
  } else {
    const dim3 sg((unsigned)cdiv(L.npad, 32), (unsigned)cdiv(Lq.kq, 32));
    unsigned short* q = reinterpret_cast<unsigned short*>(scratch);
    if (pl.reg) {
      hipLaunchKernelGGL((split_p_bf16<2, true>), sg, dim3(256), 0, s, P, ldp, n, k, Lq.kq, L.npad, q);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((split_p_bf16<2, false>), sg, dim3(256), 0, s, P, ldp, n, k, Lq.kq, L.npad, q);
      else
        hipLaunchKernelGGL((split_p_bf16<3, false>), sg, dim3(256), 0, s, P, ldp, n, k, Lq.kq, L.npad, q);
    }
    NYS_CHECK_LAUNCH();
  }
  scratch += se;
  scratch_elems -= se;
  const int64_t tiles = pl.tiles;
  // about bpc blocks per compute unit (eight by default): the per-tile chain
  // (loads, LDS, barriers, MFMA) is latency-bound with fewer waves per SIMD
  int64_t nz = cdiv(pl.bpc * (num_cus() < 256 ? num_cus() : 256), tiles);
  if (nz < 1) nz = 1;
  while (nz > 1 && (size_t)(nz * n * k) > scratch_elems) --nz;
  const int64_t pps = cdiv(cdiv(n, nz), 32) * 32;
  nz = cdiv(n, pps);
  dim3 grid((unsigned)cdiv(n, pl.rows), (unsigned)cdiv(k, nc), (unsigned)nz);
  float* dst = nz > 1 ? scratch : V;
  const int64_t ldo = nz > 1 ? k : ldv;
  const float oscale = nz > 1 ? 1.0f : L.scale;
  const int kss = ks_for(L.ksteps);
  if (pl.reg) {
#define KR(CF) \
  hipLaunchKernelGGL((rbf_kv_reg<CF, 2>), grid, dim3(256), 0, s, Lq, Pq, Lq.npad / 8, k, dst, ldo, pps, oscale, skip)
#define K32(CF, F, KS) \
  hipLaunchKernelGGL((rbf_kv_reg32<CF, F, KS>), grid, dim3(256), 0, s, Lq, Pz, pl.kq, k, dst, ldo, pps, oscale, skip)
#define K32S(CF, F) \
  do { if (kss == 2) K32(CF, F, 2); else if (kss == 4) K32(CF, F, 4); else K32(CF, F, 8); } while (0)
    if (mode == RBF_GRAM_BF16X3) {
      if (pl.cf == 1) KR(1); else if (pl.cf == 2) KR(2); else KR(4);
    } else {
      if (pl.cf == 1) K32S(1, 4); else if (pl.cf == 2) K32S(2, 4); else K32S(4, 2);
    }
#undef K32S
#undef K32
#undef KR
  } else {
#define KV(M, CF, KS, FR) hipLaunchKernelGGL((rbf_kv_lowp<M, CF, KS, FR>), grid, dim3(256), 0, s, Lq, P, ldp, k, Pq, Lq.npad / 8, dst, ldo, pps, oscale, skip)
#define KVF(M, CF, KS) do { if (pl.f == 2) KV(M, CF, KS, 2); else KV(M, CF, KS, 1); } while (0)
    if (mode == 0) {
      if (pl.cf == 16) KVF(0, 16, 1); else KVF(0, 8, 1);
    } else if (pl.cf == 16) {
      if (kss == 2) KVF(1, 16, 2); else if (kss == 4) KVF(1, 16, 4); else KVF(1, 16, 8);
    } else if (kss == 2) KVF(1, 8, 2); else if (kss == 4) KVF(1, 8, 4); else KVF(1, 8, 8);
#undef KVF
#undef KV
  }
  NYS_CHECK_LAUNCH();
  if (nz > 1) {
    hipLaunchKernelGGL(rbf_lowp_finish, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, scratch, (int)nz, n, k,
                       L.scale, P, ldp, mu_dev, nrhs, V, ldv, skip);
    NYS_CHECK_LAUNCH();
  } else if (mu_dev) {
    hipLaunchKernelGGL(rbf_lowp_add_mu, dim3((unsigned)cdiv(n * k, 256)), dim3(256), 0, s, n, k, P, ldp, mu_dev, nrhs,
                       V, ldv, skip);
    NYS_CHECK_LAUNCH();
  }
  return NYS_OK;
}

__global__ void fill_value(float* __restrict__ p, int64_t count, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

nys_status rbf_lowp_autotune(const RbfLowp& L0, int mode, const int64_t* ks, int nks, float* P, float* V,
                             float* scratch, size_t scratch_elems, hipStream_t s) {
  RbfLowp L = L0;
  L.coldone = nullptr;
  const int64_t n = L.n;
  int64_t kmax = 0;
  for (int i = 0; i < nks; ++i) kmax = ks[i] > kmax ? ks[i] : kmax;
  // any finite block: the timing does not depend on the values
  hipLaunchKernelGGL(fill_value, dim3((unsigned)cdiv(n * kmax, 256)), dim3(256), 0, s, P, n * kmax, 1.0f / 64.0f);
  NYS_CHECK_LAUNCH();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NYS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("autotune: event creation failed");
    return NYS_ERR_DEVICE;
  }
  nys_status st = NYS_OK;
  std::vector<TuneEntry> found;
  for (int i = 0; i < nks && st == NYS_OK; ++i) {
    const int64_t k = ks[i];
    double best_us = 0.0;
    KvChoice best{};
    for (const KvChoice& c : kv_candidates()) {
      const KvPlan pl = make_plan(n, k, mode, c);
      if (pl.prep_elems > scratch_elems) continue;
      // one untimed launch, then the mean of three
      st = rbf_lowp_kv_plan(L, mode, pl, P, k, k, nullptr, 1, V, k, scratch, scratch_elems, nullptr, s);
      if (st != NYS_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) {
        set_error("autotune: event record failed");
        st = NYS_ERR_DEVICE;
        break;
      }
      for (int r = 0; r < 3 && st == NYS_OK; ++r)
        st = rbf_lowp_kv_plan(L, mode, pl, P, k, k, nullptr, 1, V, k, scratch, scratch_elems, nullptr, s);
      if (st != NYS_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        set_error("autotune: event timing failed");
        st = NYS_ERR_DEVICE;
        break;
      }
      const double us = 1e3 * (double)ms / 3.0;
      if (best_us == 0.0 || us < best_us) {
        best_us = us;
        best = c;
      }
    }
    if (st == NYS_OK && best_us > 0.0) found.push_back(TuneEntry{n, k, L.d, mode, best, best_us});
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != NYS_OK) return st;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_env_load_locked();
    for (const TuneEntry& e : found) tune_put(e);
  }
  return NYS_OK;
}

}  // namespace nys
