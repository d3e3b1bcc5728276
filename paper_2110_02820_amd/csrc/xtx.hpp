#pragma once
#include "operators.hpp"

namespace nys {

// Partial form of A p = scale X^T X p for one contiguous vector: part[g][j],
// g < *ng_out, in arithmetic TA for data TD; A p = scale * sum_g part[g].
// With pvq and pvq_filled given, the one-pass product also writes
// pvq[g] = sum over group g's rows of w_r (x_r^T p)^2 and pvq[ng] = ||p||^2
// (so p^T A p = scale * sum_g pvq[g]) and sets *pvq_filled; the two-pass
// product for wide X leaves *pvq_filled false.
template <typename TD, typename TA>
nys_status xtx_partials(const OpDesc& op, const TA* p, TA* scratch, size_t scratch_elems, int* ng_out,
                        hipStream_t s, double* pvq = nullptr, bool* pvq_filled = nullptr);

// v = scale X^T X p + mu p (partials in scratch, then a fixed-order sum).
template <typename TD, typename TA>
nys_status xtx_apply(const OpDesc& op, const TA* p, TA mu, TA* v, TA* scratch, size_t scratch_elems,
                     hipStream_t s);

}  // namespace nys
