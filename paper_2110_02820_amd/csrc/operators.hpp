#pragma once
#include "common.hpp"

namespace nys {

struct RbfLowp;

// Validated copy of a nys_operator.
struct OpDesc {
  int kind;
  int dtype;
  int64_t n;
  const void* data;
  int64_t rows, cols, ld;
  double sigma, scale;
  const int* skip = nullptr;  // device flag: kernels return at once when *skip != 0
  const int* coldone = nullptr;  // device per-column flags of a block product: finished columns (nullable)
  const double* w = nullptr;     // NYS_OP_XTX: row weights d (A = scale X^T D X), nullable
  const RbfLowp* lowp = nullptr;  // prepared points for reduced-precision RBF products
  int gram = 0;                   // RBF_GRAM_BF16X3 or RBF_GRAM_F32 (with lowp)
  nys_apply_fn apply = nullptr;   // NYS_OP_CALLBACK: the caller's product routine
  void* ctx = nullptr;
};

// T[i][c] *= w[i] for an m x k row-major block (ld k): the row weights of a
// weighted X^T X product between its two GEMMs.
template <typename T>
nys_status scale_rows(T* t, int64_t m, int64_t k, const double* w, hipStream_t s);

// NYS_OP_CALLBACK product: V = scale * (caller's A P) + mu_c P_c for k
// columns of type T (mu_dev: device array indexed by c / nrhs, or nullptr and
// the value mu_host for every column; neither shifts when both are absent).
template <typename T>
nys_status callback_apply(const OpDesc& op, const T* P, int64_t k, int64_t ldp, const double* mu_dev,
                          int64_t nrhs, double mu_host, T* V, int64_t ldv, hipStream_t s);

// Scratch (in elements of the arithmetic type) used by one operator product
// with k columns.
size_t op_scratch_elems(const OpDesc& op, int64_t k);

// V = A P + mu_c P_c for k columns, float64 arithmetic (float32 data promoted
// exactly).  mu_dev: device array indexed by c / nrhs, or nullptr for V = A P.
nys_status op_apply_f64(const OpDesc& op, const double* P, int64_t k, int64_t ldp,
                        const double* mu_dev, int64_t nrhs, double* V, int64_t ldv,
                        double* scratch, size_t scratch_elems, hipStream_t s);

// One contiguous vector: v = A p + mu p in arithmetic TA (XTX and dense).
template <typename TA>
nys_status op_matvec(const OpDesc& op, const TA* p, TA mu, TA* v, TA* scratch, size_t scratch_elems,
                     hipStream_t s);

// Single vector in partial-sum form: (A p)[j] = scale * sum_{g < ng} part[g][j]
// (X^T X: float or double arithmetic; RBF: double).  *ng_out = number of groups.
template <typename TA>
nys_status op_matvec_partials(const OpDesc& op, const TA* p, TA* part, size_t part_elems, int* ng_out,
                              hipStream_t s, double* pvq = nullptr, int* npvq = nullptr, int* npp = nullptr);

// Slots of pvq that op_matvec_partials may fill: *npvq parts of p^T A p / scale
// (XTX: per product workgroup; square RBF: per (row block, split) workgroup)
// then *npp parts of ||p||^2 from pvq[*npvq] on (XTX: one; RBF: per row
// block); *npvq = *npp = 0 when the product form has none.
constexpr int64_t kPvqMax = 2048;

// out (nr) = W p with W = K(Xr, Xc) (mode 0) or dK/dsigma (mode 1), float64
// arithmetic; Xr: nr x d (ldr), Xc: nc x d (ldc), both of storage `dtype`.
// scratch: >= 4 * 256 * nr doubles.
nys_status rbf_rect_mv(const void* Xr, int64_t nr, int64_t ldr, const void* Xc, int64_t nc,
                       int64_t ldc, int d, int dtype, double sigma, int mode, const double* p,
                       double* out, double* scratch, size_t scratch_elems, hipStream_t s);

}  // namespace nys
