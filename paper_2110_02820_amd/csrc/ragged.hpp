#pragma once
#include "operators.hpp"
#include "pcg.hpp"

namespace nys {

// Batched solve of independent ridge problems (X^T X operators) with their
// own Nystrom preconditioners and regularisations: problem c is column c of a
// padded n_max x nprob block, so every CG vector kernel handles all problems
// in one launch, and the operator product and the preconditioner apply read a
// device table of the problems.  Requirements (checked by ragged_supported):
// every operator is X^T X with the same storage type, every preconditioner
// has the same U type, nprob <= 256, n_c <= 8192, l_c <= 2048.
bool ragged_supported(const OpDesc* ops, const PrecDesc* pds, int nprob);

size_t ragged_workspace(const OpDesc* ops, const PrecDesc* pds, int nprob, int prec);

// Same contract as nys_pcg_solve_ragged (device B[c], X[c] of length n_c;
// X is also the initial guess).  Per-problem results go to info.
nys_status ragged_solve(const OpDesc* ops, const PrecDesc* pds, const double* mu, const double* const* B,
                        double* const* X, int nprob, const nys_solve_opts* o, nys_solve_info* info, void* ws,
                        size_t ws_bytes, hipStream_t s);

}  // namespace nys
