#pragma once
#include "common.hpp"
#include "operators.hpp"

namespace nys {

// Points prepared for the reduced-precision RBF kernels (see rbf_lowp.hip).
struct RbfLowp {
  int64_t n, npad;
  unsigned short* Xhi;  // npad x 32 bf16 (high parts)
  unsigned short* Xlo;  // npad x 32 bf16 (low parts)
  float* X32;           // npad x 32 float
  float* hs;            // npad: log2(e) ||x_i||^2 / (2 sigma^2)
  float two_s;          // log2(e) / sigma^2
  float scale;          // operator scale
  int ksteps;           // float32 Gram: 4-coordinate MFMA steps that cover d (<= 8)
  int64_t kq;           // columns of the pre-split P of a K P call (set per call)
};

enum { RBF_GRAM_BF16X3 = 0, RBF_GRAM_F32 = 1 };

size_t rbf_lowp_bytes(int64_t n);
nys_status rbf_lowp_prepare(const OpDesc& op, void* buf, RbfLowp& L, hipStream_t s);

// One vector in partial form: (A p)[i] = scale * sum_{g < ng} part[g][i].
nys_status rbf_lowp_mv_partials(const RbfLowp& L, int mode, const float* p, float* part, size_t part_elems,
                                int* ng_out, const int* skip, hipStream_t s);

// v = scale K p + mu p for one contiguous vector (part: the partial buffer above).
nys_status rbf_lowp_mv(const RbfLowp& L, int mode, const float* p, const double* mu_dev, float* v, float* part,
                       size_t part_elems, hipStream_t s);

// V = scale K P (+ mu_c P) for k columns, float32 (scratch: rbf_lowp_kv_scratch).
size_t rbf_lowp_kv_scratch(int64_t n, int64_t k);
nys_status rbf_lowp_kv(const RbfLowp& L, int mode, const float* P, int64_t ldp, int64_t k, const double* mu_dev,
                       int64_t nrhs, float* V, int64_t ldv, float* scratch, size_t scratch_elems, const int* skip,
                       hipStream_t s);

}  // namespace nys
