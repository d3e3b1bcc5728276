#pragma once
#include "common.hpp"

namespace nys {
nys_status gaussian(uint64_t seed, int64_t n, int64_t l, double* out, int64_t ld, hipStream_t s);
}
