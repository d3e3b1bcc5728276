#pragma once
#include "common.hpp"

namespace nys {

// C = alpha op(A) op(B) + beta C  (row-major).  `scratch` (scratch_elems
// elements of the compute type) holds split-K partial tiles; with too little
// scratch the K dimension is not split.
template <typename TC, typename TAs, typename TBs>
nys_status gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, TC alpha, const TAs* A,
                int64_t lda, const TBs* B, int64_t ldb, TC beta, TC* C, int64_t ldc, TC* scratch,
                size_t scratch_elems, hipStream_t s, const int* skip = nullptr);

// C = alpha op(A) op(B) + beta C for float32 operands with the products on
// bf16 MFMA (hi/lo three-product split, relative error ~2^-16 per product,
// float32 accumulation).  Same scratch rule as gemm(); shapes whose rows
// cannot take 16-byte loads fall back to gemm<float>.
nys_status gemm_bf16x3(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float beta, float* C, int64_t ldc, float* scratch,
                       size_t scratch_elems, hipStream_t s);

// Scratch (floats) that lets gemm_bf16x3 split B (K x N) into bf16 pieces once
// instead of in every workgroup that reads it; added to the split-K share.
size_t gemm_bf16x3_split_elems(int64_t K, int64_t N);

// Scratch that lets gemm() split K for an M x N output.
// gemm() splits K only when the output has fewer than 512 tiles of 64 x 64.
inline size_t gemm_scratch_elems(int64_t M, int64_t N) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  return tiles >= 512 ? 0 : (size_t)(16 * M * N);
}

}  // namespace nys
