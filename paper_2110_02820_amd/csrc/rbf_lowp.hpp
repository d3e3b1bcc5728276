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
  int d;                // point dimension (autotuner key)
  int64_t kq;           // columns of the pre-split P of a K P call (set per call)
  const int* coldone;   // K P call: device per-column flags; a block whose columns are all
                        // flagged writes zeros instead of its products (nullable)
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
// coldone (nullable): device flags of the k columns; column blocks whose
// columns are all flagged are not computed (their entries of V are mu_c P), and
// the tile shape is the one chosen for min(k, 16) columns, so that blocks stay
// narrow enough for finished columns to free them.
nys_status rbf_lowp_kv(const RbfLowp& L, int mode, const float* P, int64_t ldp, int64_t k, const double* mu_dev,
                       int64_t nrhs, float* V, int64_t ldv, float* scratch, size_t scratch_elems, const int* skip,
                       hipStream_t s, const int* coldone = nullptr);

// Tile-shape choice of the block product V = K P (see make_plan in
// rbf_lowp.hip): the register kernel (reg = 1, 16 cf columns per block,
// cf in {1, 2, 4}) or the LDS kernel (reg = 0, cf in {8, 16}, fr in {1, 2}
// row fragments of 16 per wave), and the target number of workgroups per
// compute unit that sets the split over points (bpc in {4, 8, 16}).
struct KvChoice {
  int reg, cf, bpc, fr;
};

// The choice a call with k columns would use on these prepared points:
// the autotuner's entry for (n, d, mode) with the smallest tuned k' >= k, else
// the built-in heuristic.  *tuned tells which.
KvChoice kv_choice(const RbfLowp& L, int64_t k, int mode, bool* tuned);

// Time every candidate choice for each k of ks (V = K P with P of k columns,
// the caller's scratch as in rbf_lowp_kv) on stream s and record the fastest
// in the process-wide table.  P, V: n x kmax float32 buffers.
nys_status rbf_lowp_autotune(const RbfLowp& L, int mode, const int64_t* ks, int nks, float* P, float* V,
                             float* scratch, size_t scratch_elems, hipStream_t s);

// Process-wide autotuner table: entries, clear, text file load (merged) and save.
int64_t kv_tune_entries();
void kv_tune_clear();
nys_status kv_tune_load(const char* path);
nys_status kv_tune_save(const char* path);
// Environment cache (NYS_AUTOTUNE_CACHE): loaded before the first lookup,
// written after each autotuning call.
void kv_tune_env_save();

}  // namespace nys
