// C ABI of the Nystrom PCG library: argument checks, workspace layout and the
// host-side ordering of the device kernels.  Every numerical step runs in the
// HIP kernels of this directory; the host only enqueues work and reads flags.
#include <atomic>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "dense_small.hpp"
#include "gemm.hpp"
#include "operators.hpp"
#include "pcg.hpp"
#include "ragged.hpp"
#include "rbf_lowp.hpp"
#include "rng.hpp"
#include "xtx.hpp"

// Eigensolver stopping ratio when U is stored in float32 (see jac_end_sweep):
// a sweep whose subproblems met no |a_pq| above this times sqrt(|a_pp a_qq|)
// is the last.  Its own rotations leave ratios of about its square (1e-6),
// which bounds the departure of U's float32 columns from orthonormality;
// P^{-1} = I + U F U^T stays positive definite while that departure is well
// below (lam_l + mu) / (lam_1 + mu).
#ifndef NYS_JACOBI_RATIO_F32
#define NYS_JACOBI_RATIO_F32 1e-3
#endif

namespace nys {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

// Diagnostics on stderr (Jacobi sweeps, refinement progress) when NYS_VERBOSE is set.
bool verbose() {
  static const bool v = std::getenv("NYS_VERBOSE") != nullptr;
  return v;
}

int next_pinned_seq() {
  static thread_local int seq = 0;
  seq = seq >= 0x3fffffff ? 1 : seq + 1;
  return seq;
}

bool wait_pinned(const volatile int* seq, int expect, hipStream_t s, int alt) {
  const auto seen = [&]() {
    const int v = *seq;
    return v == expect || (alt != 0 && v == alt);
  };
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spin = 0;; ++spin) {
    if (seen()) {
      std::atomic_thread_fence(std::memory_order_acquire);
      return true;
    }
    if ((spin & 1023u) == 1023u &&
        std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2))
      break;
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("stream failed while waiting for a device flag: %s", hipGetErrorString(e));
    return false;
  }
  if (seen()) {
    std::atomic_thread_fence(std::memory_order_acquire);
    return true;
  }
  set_error("device flag not written (expected sequence %d, found %d)", expect, *seq);
  return false;
}

// Launch timing of the X^T X product kernel (nys_timing_begin / _end):
// while enabled, each launch is bracketed by two HIP events recorded on the
// stream it is launched on.  Host thread of the caller only.
namespace {
struct LaunchTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;  // start, end, start, end, ...
};
thread_local LaunchTimer g_timer;

void record(hipStream_t s) {
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    g_timer.on = false;  // no event: give up timing, never the launch
    return;
  }
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    g_timer.on = false;
    return;
  }
  g_timer.ev.push_back(e);
}
}  // namespace

void timing_mark_begin(hipStream_t s) {
  if (g_timer.on) record(s);
}
void timing_mark_end(hipStream_t s) {
  if (g_timer.on) record(s);
}

int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

namespace {

constexpr int kMaxGroups = 512;  // upper bound on partial-sum groups
constexpr int kMaxSweeps = 40;   // Jacobi sweep cap
constexpr int64_t kMaxCols = 256;

int groups() {
  const int g = 2 * num_cus();
  return g < kMaxGroups ? g : kMaxGroups;
}

// ---------------------------------------------------------------- checks

nys_status check_op(const nys_operator* A, OpDesc& o) {
  NYS_ARG(A != nullptr, "operator is NULL");
  NYS_ARG(A->kind >= NYS_OP_DENSE && A->kind <= NYS_OP_CALLBACK, "unknown operator kind %d", A->kind);
  NYS_ARG(A->n >= 1, "operator dimension n = %lld < 1", (long long)A->n);
  NYS_ARG(std::isfinite(A->scale) && A->scale > 0.0, "operator scale must be finite and > 0");
  NYS_ARG(A->weights == nullptr || A->kind == NYS_OP_XTX, "row weights belong to the X^T X operator only");
  o.apply = nullptr;
  o.ctx = nullptr;
  o.w = nullptr;
  if (A->kind == NYS_OP_CALLBACK) {
    NYS_ARG(A->apply != nullptr, "callback operator: apply is NULL");
    o.kind = A->kind;
    o.dtype = NYS_F64;
    o.n = A->n;
    o.data = nullptr;
    o.rows = A->n;
    o.cols = A->n;
    o.ld = A->n;
    o.sigma = 0.0;
    o.scale = A->scale;
    o.skip = nullptr;
    o.apply = A->apply;
    o.ctx = A->ctx;
    return NYS_OK;
  }
  NYS_ARG(A->dtype == NYS_F64 || A->dtype == NYS_F32, "operator dtype must be NYS_F64 or NYS_F32");
  NYS_ARG(A->data != nullptr, "operator data is NULL");
  NYS_ARG(A->ld >= A->cols && A->cols >= 1 && A->rows >= 1, "operator shape/ld invalid");
  if (A->kind == NYS_OP_DENSE) NYS_ARG(A->rows == A->n && A->cols == A->n, "dense operator must be n x n");
  if (A->kind == NYS_OP_XTX) NYS_ARG(A->cols == A->n, "X^T X operator: cols must equal n");
  if (A->kind == NYS_OP_RBF) {
    NYS_ARG(A->rows == A->n, "RBF operator: rows must equal n");
    NYS_ARG(std::isfinite(A->sigma) && A->sigma > 0.0, "RBF operator: sigma must be > 0");
    NYS_ARG(A->cols <= 64, "RBF operator: d must be <= 64");
  }
  o.kind = A->kind;
  o.dtype = A->dtype;
  o.n = A->n;
  o.data = A->data;
  o.rows = A->rows;
  o.cols = A->cols;
  o.ld = A->ld;
  o.sigma = A->sigma;
  o.scale = A->scale;
  o.skip = nullptr;
  o.w = A->kind == NYS_OP_XTX ? A->weights : nullptr;
  return NYS_OK;
}

nys_status check_prec(const nys_precond* P, PrecDesc& d) {
  NYS_ARG(P != nullptr, "preconditioner is NULL");
  NYS_ARG(P->n >= 1 && P->ell >= 1 && P->ell <= P->n, "preconditioner needs 1 <= ell <= n");
  NYS_ARG(P->U != nullptr && P->lam != nullptr, "preconditioner U / lam is NULL");
  NYS_ARG(P->ldu >= P->ell, "preconditioner ldu < ell");
  NYS_ARG(P->dtype == NYS_F64 || P->dtype == NYS_F32, "preconditioner dtype invalid");
  NYS_ARG(P->ell <= 2048, "preconditioner rank > 2048 not supported");
  d.n = P->n;
  d.ell = P->ell;
  d.U = P->U;
  d.ldu = P->ldu;
  d.dtype = P->dtype;
  d.lam = P->lam;
  return NYS_OK;
}

hipStream_t S(void* stream) { return static_cast<hipStream_t>(stream); }

// ---------------------------------------------------------------- layouts

struct Core {  // l x l float64 work shared by sketch and factor
  double *G, *L, *Linv, *Dinv, *T, *eig, *gscr, *nu, *part, *sig2;
  int *info, *flags, *sweeps, *conv;
  size_t gscr_elems;
};

void carve_core(Arena& a, int64_t l, Core& c) {
  c.G = a.take<double>(l * l);
  c.L = a.take<double>(l * l);
  c.Linv = a.take<double>(l * l);
  c.T = a.take<double>(l * l);
  c.Dinv = a.take<double>(chol_ws_doubles(l));
  c.eig = a.take<double>(eig_ws_doubles(l));
  c.gscr_elems = gemm_scratch_elems(l, l);
  c.gscr = a.take<double>(c.gscr_elems);
  c.nu = a.take<double>(1);
  c.part = a.take<double>(frob_partials());
  c.sig2 = a.take<double>(l);
  c.info = a.take<int>(2);  // pivot flags: [0] the core Cholesky / first CholeskyQR pass, [1] second pass
  c.flags = a.take<int>(kMaxSweeps);
  c.sweeps = a.take<int>(1);
  c.conv = a.take<int>(1);
}

struct SketchWs {
  Core c;
  double* opscr;
  size_t opscr_elems;
  float *Om32, *T32, *Y32, *f32scr;
  size_t f32scr_elems;
  void* lowp_buf;
};

bool sketch_f32(const OpDesc& op, int prec) {
  return prec != NYS_PREC_FP64 && op.kind == NYS_OP_XTX && op.dtype == NYS_F32;
}

bool rbf_lowp_mode(const OpDesc& op, int prec) { return prec != NYS_PREC_FP64 && op.kind == NYS_OP_RBF; }

int rbf_gram(int prec) { return prec == NYS_PREC_BF16X3_REFINE64 ? RBF_GRAM_BF16X3 : RBF_GRAM_F32; }

void carve_sketch(Arena& a, const OpDesc& op, int64_t l, int prec, SketchWs& w) {
  carve_core(a, l, w.c);
  w.opscr_elems = op_scratch_elems(op, l);
  w.opscr = a.take<double>(w.opscr_elems);
  w.Om32 = w.T32 = w.Y32 = w.f32scr = nullptr;
  w.f32scr_elems = 0;
  w.lowp_buf = nullptr;
  if (rbf_lowp_mode(op, prec)) {
    w.Om32 = a.take<float>(op.n * l);
    w.Y32 = a.take<float>(op.n * l);
    w.f32scr_elems = rbf_lowp_kv_scratch(op.n, l);
    w.f32scr = a.take<float>(w.f32scr_elems);
    w.lowp_buf = a.take<char>(rbf_lowp_bytes(op.n));
  }
  if (sketch_f32(op, prec)) {
    w.Om32 = a.take<float>(op.n * l);
    w.T32 = a.take<float>(op.rows * l);
    w.Y32 = a.take<float>(op.n * l);
    w.f32scr_elems = gemm_scratch_elems(op.n, l);
    // bf16x3 products: room for B split into bf16 pieces once per product
    if (prec == NYS_PREC_BF16X3_REFINE64)
      w.f32scr_elems += gemm_bf16x3_split_elems(op.rows > op.n ? op.rows : op.n, l) + 4;
    w.f32scr = a.take<float>(w.f32scr_elems);
  }
}

struct FactorWs {
  Core c;
  double* B;
};

void carve_factor(Arena& a, int64_t n, int64_t l, FactorWs& w) {
  carve_core(a, l, w.c);
  w.B = a.take<double>(n * l);
}

template <typename T>
struct PcgBufs {
  T *V, *R, *Z, *P, *X, *B;
  T* Xw;       // working copy of the active columns of X once columns are compacted
  double* mu;  // per-column mu of the active columns
  int *cidx, *cmap;  // compaction: kept columns (old positions), original column of each active column
  PcgWork w;
  CgScalars sc;
  T* opscr;
  size_t opscr_elems;
};

template <typename T>
void carve_pcg(Arena& a, const OpDesc& op, int64_t l, int64_t k, PcgBufs<T>& b) {
  const int64_t n = op.n;
  b.V = a.take<T>(n * k);
  b.R = a.take<T>(n * k);
  b.Z = a.take<T>(n * k);
  b.P = a.take<T>(n * k);
  b.X = a.take<T>(n * k);
  b.B = a.take<T>(n * k);
  b.Xw = k > 1 ? a.take<T>(n * k) : nullptr;
  b.mu = a.take<double>(k);
  b.cidx = a.take<int>(k);
  b.cmap = a.take<int>(k);
  b.w.pb = a.take<double>(kMaxGroups * k);
  b.w.prr = a.take<double>(kMaxGroups * k);
  b.w.ppv = a.take<double>(std::max<int64_t>(kMaxGroups * k, kPvqMax + 1));
  b.w.prz = a.take<double>(kMaxGroups * k);
  b.w.apart_elems = precond_part_elems(n, l, k);
  b.w.apart = a.take<double>(b.w.apart_elems);
  b.w.Cs = a.take<double>(l * k);
  b.w.Ct = a.take<double>(l * k);
  b.sc.rz = a.take<double>(2 * k);
  b.sc.bnorm2 = a.take<double>(k);
  b.sc.rnorm2 = a.take<double>(k);
  b.sc.alpha = a.take<double>(k);
  b.sc.beta = a.take<double>(k);
  b.sc.done = a.take<int>(k);
  b.sc.conv = a.take<int>(k);
  b.sc.iters = a.take<int>(k);
  b.sc.status = a.take<int>(k);
  b.sc.alldone = a.take<int>(1);
  b.sc.ctr = a.take<unsigned>(64);
  b.opscr_elems = op_scratch_elems(op, k);
  b.opscr = a.take<T>(b.opscr_elems);
}

struct SolveWs {
  PcgBufs<double> d;
  PcgBufs<float> f;
  double *mu, *R64, *V64, *X64, *B64, *dots;
  double* mu_act;  // mu of the columns still refined
  int* omap;       // original column of each refined column
  // device-info form: per-column state kept on the device
  double *relres_d, *prev_d;
  int *iters_d, *brk_d, *active_d;
  int* xzero;  // 1 while the start vectors are all zero (their product is skipped)
  bool has_f;
  void* lowp_buf;
  RbfLowp L;
};

void carve_solve(Arena& a, const OpDesc& op, int64_t l, int64_t k, int prec, SolveWs& w) {
  const int64_t n = op.n;
  w.mu = a.take<double>(k);
  w.mu_act = a.take<double>(k);
  w.omap = a.take<int>(k);
  w.dots = a.take<double>(kMaxGroups * k + 2 * k);
  w.relres_d = a.take<double>(k);
  w.prev_d = a.take<double>(k);
  w.iters_d = a.take<int>(k);
  w.brk_d = a.take<int>(k);
  w.active_d = a.take<int>(k);
  w.xzero = a.take<int>(1);
  w.R64 = a.take<double>(n * k);
  w.V64 = a.take<double>(n * k);
  w.X64 = a.take<double>(n * k);
  w.B64 = a.take<double>(n * k);
  carve_pcg<double>(a, op, l, k, w.d);
  w.has_f = prec != NYS_PREC_FP64;
  if (w.has_f) carve_pcg<float>(a, op, l, k, w.f);
  w.lowp_buf = rbf_lowp_mode(op, prec) ? a.take<char>(rbf_lowp_bytes(op.n)) : nullptr;
}

// ---------------------------------------------------------------- small kernels

template <typename TS, typename TD>
__global__ void gather_cols(int64_t n, int64_t k, const TS* __restrict__ src, int64_t lds,
                            int64_t nsrc_cols, TD* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k, c = idx % k;
  dst[i * ldd + c] = TD(src[i * lds + (c % nsrc_cols)]);
}

// R = B - V and per-column partial ||R||^2, ||B||^2 (one group per block of rows)
__global__ void residual_norms(int64_t n, int64_t k, const double* __restrict__ B,
                               const double* __restrict__ V, double* __restrict__ R,
                               double* __restrict__ part) {
  // part[g][c] = ||R_c||^2 partial, part[G + g][c] = ||B_c||^2 partial; k <= 256
  __shared__ double sh[256];
  const int64_t rows = cdiv(n, gridDim.x);
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  for (int64_t c0 = 0; c0 < k; c0 += 1) {
    double sr = 0.0, sb = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
      const double b = B[i * k + c0];
      const double r = b - V[i * k + c0];
      R[i * k + c0] = r;
      sr += r * r;
      sb += b * b;
    }
    sr = block_sum(sr, sh);
    sb = block_sum(sb, sh);
    if (threadIdx.x == 0) {
      part[(int64_t)blockIdx.x * k + c0] = sr;
      part[((int64_t)gridDim.x + blockIdx.x) * k + c0] = sb;
    }
  }
}

// The relative residual of a single column (from residual_norms' partials,
// summed in the host's order) and a completion tag, published to pinned host
// memory (bytes 160..175 of pinned_flags()) with the tag written last.
struct ResSnap {
  int seq;
  int pad;
  double relres;
};

ResSnap* res_snap() {
  int* p = pinned_flags();
  return p ? reinterpret_cast<ResSnap*>(reinterpret_cast<char*>(p) + 160) : nullptr;
}

// part: residual_norms' output for k = 1 over g workgroups; null: the tag only
__global__ void residual_snapshot(const double* __restrict__ part, int g, ResSnap* out, int seq) {
  volatile ResSnap* o = out;
  if (part) {
    double rr = 0.0, bb = 0.0;
    for (int q = 0; q < g; ++q) {
      rr += part[q];
      bb += part[g + q];
    }
    o->relres = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  }
  __threadfence_system();
  o->seq = seq;
}

template <typename T>
__global__ void copy_dev(const T* __restrict__ src, T* __restrict__ dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

template <typename T>
__global__ void zero_fill(T* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = T(0);
}

// PCG set-up in one launch: mu (k values) into the run's buffer, the 64
// counters cleared, and, for a zero initial guess, X and V (n k each) cleared.
// With xflag (a given start X that may be zero): V cleared and *xflag = 1,
// which zero_test then clears if X has a nonzero entry.
template <typename T>
__global__ void pcg_start(const double* __restrict__ mu_src, double* __restrict__ mu_dst, int64_t k,
                          unsigned* __restrict__ ctr, T* __restrict__ X, T* __restrict__ V, int64_t nk,
                          int* __restrict__ xflag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) mu_dst[i] = mu_src[i];
  if (i < 64) ctr[i] = 0u;
  if ((X || xflag) && i < nk) {
    if (X) X[i] = T(0);
    V[i] = T(0);
  }
  if (xflag && i == 0) *xflag = 1;
}

// *flag = 0 if any of x[0 .. count) is nonzero (all writers store the same
// value).  A product launched with skip = flag then runs only for a nonzero
// start: every product kernel returns at once while *flag != 0.
template <typename T>
__global__ void zero_test(const T* __restrict__ x, int64_t count, int* __restrict__ flag) {
  bool nz = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    nz = nz || x[i] != T(0);
  if (nz) *flag = 0;
}

// V (count values) cleared and *flag = 1 (see zero_test)
__global__ void zero_flag_init(double* __restrict__ V, int64_t count, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) V[i] = 0.0;
  if (i == 0) *flag = 1;
}

template <typename TS>
__global__ void add_to(double* __restrict__ dst, const TS* __restrict__ src, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] += double(src[i]);
}

__global__ void dot_partial(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                            double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// gX[r][j] = -scale (t1[r] lam[j] + t2[r] x[j])
__global__ void outer2(int64_t m, int64_t n, double scale, const double* __restrict__ t1,
                       const double* __restrict__ lam, const double* __restrict__ t2,
                       const double* __restrict__ x, double* __restrict__ gX) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t r = idx / n, j = idx % n;
  gX[idx] = -scale * (t1[r] * lam[j] + t2[r] * x[j]);
}

template <typename TS>
__global__ void gemv_rows(const TS* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                          const double* __restrict__ v, double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s += double(X[row * ld + j]) * v[j];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

// Up to 256 column indices passed by value (no host-to-device copy).
struct ColList {
  int v[256];
};

__global__ void set_indices(int* __restrict__ dst, int64_t count, ColList l) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = l.v[i];
}

// dst (n x knew) = columns idx[0..knew) of src (n x kold)
template <typename TS, typename TD>
__global__ void gather_idx(int64_t n, int64_t kold, const TS* __restrict__ src, const int* __restrict__ idx,
                           int64_t knew, TD* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * knew) return;
  const int64_t i = t / knew, j = t % knew;
  dst[t] = TD(src[i * kold + idx[j]]);
}

// dst (n x kfull) columns map[j] (+)= src (n x ksub) column j
template <typename TS, bool ADD>
__global__ void scatter_idx(int64_t n, int64_t ksub, const TS* __restrict__ src, const int* __restrict__ map,
                            int64_t kfull, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ksub) return;
  const int64_t i = t / ksub, j = t % ksub;
  double* d = dst + i * kfull + map[j];
  if (ADD) *d += double(src[t]);
  else *d = double(src[t]);
}

template <typename T>
__global__ void scatter_idx_same(int64_t n, int64_t ksub, const T* __restrict__ src, const int* __restrict__ map,
                                 int64_t kfull, T* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ksub) return;
  const int64_t i = t / ksub, j = t % ksub;
  dst[i * kfull + map[j]] = src[t];
}

// Keep the per-column CG scalars (and mu) of columns idx[0..knew), one
// workgroup: every kept value is read into registers before any is written.
__global__ void compact_scalars(CgScalars sc, double* __restrict__ mu, int64_t kold, const int* __restrict__ idx,
                                int64_t knew) {
  const int t = threadIdx.x;
  double r0 = 0, r1 = 0, bn = 0, rn = 0, al = 0, be = 0, m = 0;
  int dn = 0, cv = 0, it = 0, st = 0;
  if (t < knew) {
    const int j = idx[t];
    r0 = sc.rz[j];
    r1 = sc.rz[kold + j];
    bn = sc.bnorm2[j];
    rn = sc.rnorm2[j];
    al = sc.alpha[j];
    be = sc.beta[j];
    m = mu[j];
    dn = sc.done[j];
    cv = sc.conv[j];
    it = sc.iters[j];
    st = sc.status[j];
  }
  __syncthreads();
  if (t < knew) {
    sc.rz[t] = r0;
    sc.rz[knew + t] = r1;
    sc.bnorm2[t] = bn;
    sc.rnorm2[t] = rn;
    sc.alpha[t] = al;
    sc.beta[t] = be;
    mu[t] = m;
    sc.done[t] = dn;
    sc.conv[t] = cv;
    sc.iters[t] = it;
    sc.status[t] = st;
  }
}

// ---- device-info form of the solve: every decision made on the device

// relres[c] = sqrt(sum_g part[g][c] / sum_g part[G + g][c]) (sqrt of the
// residual norm alone when ||b|| = 0), groups summed in order
__global__ void relres_from_parts(int64_t k, int ng, const double* __restrict__ part, double* __restrict__ relres) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double rr = 0.0, bb = 0.0;
  for (int q = 0; q < ng; ++q) {
    rr += part[(int64_t)q * k + c];
    bb += part[(int64_t)(ng + q) * k + c];
  }
  relres[c] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

// Refinement step selection: a column is refined while its true residual
// exceeds tol, it has not broken down, and the last step at least halved its
// residual (first step: prev = +inf).  prev <- relres.
__global__ void refine_select(int64_t k, const double* __restrict__ relres, double* __restrict__ prev,
                              const int* __restrict__ brk, int* __restrict__ active, double tol) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const double r = relres[c];
  active[c] = (!brk[c] && !(r <= tol) && r <= 0.5 * prev[c]) ? 1 : 0;
  prev[c] = r;
}

// inner right-hand sides: column c of R64 (float32) where active, else 0
__global__ void gather_active(int64_t n, int64_t k, const double* __restrict__ R, const int* __restrict__ active,
                              float* __restrict__ fB) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  fB[t] = active[t % k] ? float(R[t]) : 0.0f;
}

// iterations and breakdowns of an inner solve added to the column totals
__global__ void refine_count(int64_t k, CgScalars sc, int* __restrict__ iters, int* __restrict__ brk) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  iters[c] += sc.iters[c];
  if (sc.status[c] == NYS_ERR_BREAKDOWN) brk[c] = 1;
}

__global__ void init_refine_state(int64_t k, double* __restrict__ prev, int* __restrict__ iters,
                                  int* __restrict__ brk) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  prev[c] = __builtin_huge_val();
  iters[c] = 0;
  brk[c] = 0;
}

// caller's device info: iterations, true residual, status of every column
// (iters_src / status_src: a PCG run's scalars, or the refinement totals when
// brk is given)
__global__ void write_device_info(int64_t k, const int* __restrict__ iters_src, const int* __restrict__ status_src,
                                  const int* __restrict__ brk, const double* __restrict__ relres, double tol,
                                  int32_t* __restrict__ o_iters, double* __restrict__ o_relres,
                                  int32_t* __restrict__ o_status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const bool broke = brk ? brk[c] != 0 : status_src[c] == NYS_ERR_BREAKDOWN;
  const double r = relres[c];
  if (o_iters) o_iters[c] = iters_src[c];
  if (o_relres) o_relres[c] = r;
  if (o_status) o_status[c] = broke ? NYS_ERR_BREAKDOWN : (r <= tol ? NYS_OK : NYS_NOT_CONVERGED);
}

unsigned nblk(int64_t count) { return (unsigned)(count > 0 ? cdiv(count, 256) : 1); }

nys_status upload_indices(int* dst, const std::vector<int>& v, hipStream_t s) {
  ColList l{};
  for (size_t i = 0; i < v.size() && i < 256; ++i) l.v[i] = v[i];
  hipLaunchKernelGGL(set_indices, dim3(1), dim3(256), 0, s, dst, (int64_t)v.size(), l);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

template <typename T>
nys_status zero(T* p, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(zero_fill<T>, dim3(nblk(count)), dim3(256), 0, s, p, count);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Up to 256 values passed by value (no host-to-device copy, so the call is
// safe inside stream capture and needs no pinned memory).
struct ValList {
  double v[256];
};

__global__ void set_values(double* __restrict__ dst, int64_t count, ValList l) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = l.v[i];
}

nys_status set_mu(double* mu_dev, const double* mu, int64_t nmu, hipStream_t s) {
  for (int64_t i = 0; i < nmu; i += 256) {
    ValList l{};
    const int64_t cnt = (nmu - i) < 256 ? (nmu - i) : 256;
    for (int64_t j = 0; j < cnt; ++j) l.v[j] = mu[i + j];
    hipLaunchKernelGGL(set_values, dim3(1), dim3(256), 0, s, mu_dev + i, cnt, l);
    NYS_CHECK_LAUNCH();
  }
  return NYS_OK;
}

// Pivot flags (and the shift) of a Cholesky, published to pinned host memory
// (bytes 128..151 of pinned_flags()) with the sequence tag written last, so
// that the host can read them while the device goes on with later kernels.
// The sketch (two CholeskyQR passes) and the factorisation (the core
// Cholesky and its shift) share the slot: each call waits for its tag.
struct PivotSnap {
  int seq;
  int info[2];
  int pad;
  double nu;
};

PivotSnap* pivot_snap() {
  int* p = pinned_flags();
  return p ? reinterpret_cast<PivotSnap*>(reinterpret_cast<char*>(p) + 128) : nullptr;
}

// info: ninfo (1 or 2) device flags; nu: device shift or null
__global__ void pivot_snapshot(const int* __restrict__ info, int ninfo, const double* __restrict__ nu, PivotSnap* out,
                               int seq) {
  volatile PivotSnap* o = out;
  o->info[0] = info[0];
  o->info[1] = ninfo > 1 ? info[1] : 0;
  o->nu = nu ? nu[0] : 0.0;
  __threadfence_system();
  o->seq = seq;
}

// Publish the flags and return the tag to wait for.
int publish_pivots(const int* info, int ninfo, const double* nu, PivotSnap* snap, hipStream_t s) {
  const int seq = next_pinned_seq();
  hipLaunchKernelGGL(pivot_snapshot, dim3(1), dim3(1), 0, s, info, ninfo, nu, snap, seq);
  return seq;
}

// ---------------------------------------------------------------- CholQR

// Omega <- Omega C^{-1} with C^T C = Omega^T Omega (CholeskyQR), using tmp
// (n x l).  One pass leaves ||Q^T Q - I|| of order kappa(Omega)^2 u; a Gaussian
// n x l matrix with n >= 3 l has kappa <= (sqrt(3) + 1)/(sqrt(3) - 1) ~ 3.7
// with overwhelming probability, so one pass is orthonormal to ~1e-15 there;
// squarer test matrices, and any caller-supplied matrix, get a second pass.
nys_status cholqr(double* Om, double* tmp, int64_t n, int64_t l, bool gaussian, Core& c, int* passes_out,
                  hipStream_t s) {
  const int passes = gaussian && n >= 3 * l ? 1 : 2;
  *passes_out = passes;
  double* src = Om;
  double* dst = tmp;
  for (int pass = 0; pass < passes; ++pass) {
    NYS_TRY((gemm<double, double, double>(true, false, l, l, n, 1.0, src, l, src, l, 0.0, c.G, l,
                                          c.gscr, c.gscr_elems, s)));
    // pass p's pivot flag stays in c.info[p] for the caller to read with the
    // products that follow (no host round trip here)
    NYS_TRY(cholesky(c.G, l, c.L, c.Dinv, c.info + pass, s));
    NYS_TRY(tri_inverse(c.L, l, c.Dinv, c.Linv, s));
    NYS_TRY((gemm<double, double, double>(false, true, n, l, l, 1.0, src, l, c.Linv, l, 0.0, dst, l,
                                          c.gscr, c.gscr_elems, s)));
    double* t = src;
    src = dst;
    dst = t;
  }
  if (src != Om) NYS_HIP(hipMemcpyAsync(Om, src, sizeof(double) * n * l, hipMemcpyDeviceToDevice, s));
  return NYS_OK;
}

// ---------------------------------------------------------------- PCG core

template <typename T>
nys_status matvec(const OpDesc& op, const T* P, int64_t k, const double* mu_dev, int64_t nrhs,
                  double mu_host, T* V, PcgBufs<T>& b, hipStream_t s);

template <>
nys_status matvec<double>(const OpDesc& op, const double* P, int64_t k, const double* mu_dev,
                          int64_t nrhs, double mu_host, double* V, PcgBufs<double>& b,
                          hipStream_t s) {
  if (k == 1 && (op.kind == NYS_OP_XTX || op.kind == NYS_OP_DENSE))
    return op_matvec<double>(op, P, mu_host, V, b.opscr, b.opscr_elems, s);
  return op_apply_f64(op, P, k, k, mu_dev, nrhs, V, k, b.opscr, b.opscr_elems, s);
}

template <>
nys_status matvec<float>(const OpDesc& op, const float* P, int64_t k, const double* mu_dev,
                         int64_t nrhs, double mu_host, float* V, PcgBufs<float>& b, hipStream_t s) {
  if (op.kind == NYS_OP_CALLBACK) return callback_apply<float>(op, P, k, k, mu_dev, nrhs, 0.0, V, k, s);
  if (k == 1 && (op.kind == NYS_OP_XTX || op.kind == NYS_OP_DENSE))
    return op_matvec<float>(op, P, (float)mu_host, V, b.opscr, b.opscr_elems, s);
  if (op.kind == NYS_OP_RBF && op.lowp)
    return rbf_lowp_kv(*op.lowp, op.gram, P, k, k, mu_dev, nrhs, V, k, b.opscr, b.opscr_elems, op.skip, s,
                       op.coldone);
  set_error("float32 arithmetic is available for X^T X, dense, callback and prepared RBF operators (k = 1 for "
            "X^T X)");
  return NYS_ERR_ARG;
}

struct PcgResult {
  std::vector<int> iters, status;
  std::vector<double> rnorm2, bnorm2;
  int sweeps = 0;
};

// Left-preconditioned CG (algorithm "Nystrom PCG") on k independent columns,
// column c with its own mu (mu_dev / mu_host, k entries).  B (n x k, ld = k)
// and X (n x k, ld = k, in: x0 unless x0_zero) are arrays of type T.
//
// Columns that have met the stopping test are compacted away at the
// convergence polls (every check_every iterations): the active columns of X,
// R, the direction and the per-column scalars are gathered to the front, so
// the block products and the preconditioner apply only pay for the columns
// still iterating.  Each column follows exactly the recurrence it would follow
// alone; results are scattered back to the original column order.
//
// dev_mode (the device-info form of nys_pcg_solve): nothing is read back and
// nothing is decided on the host.  Exactly maxit iterations are enqueued on
// all k columns (a column that has stopped is frozen by its device flags) and
// res is left empty: the results stay in b.sc.
template <typename T>
nys_status pcg_run(const OpDesc& op0, const PrecDesc& P, int64_t k, const double* mu_dev,
                   const std::vector<double>& mu_host, const T* B, T* X, bool x0_zero, double tol, int maxit,
                   int check_every, PcgBufs<T>& b, PcgResult& res, hipStream_t s, bool dev_mode = false,
                   int* xflag = nullptr) {
  const int64_t n = op0.n;
  OpDesc op = op0;
  op.skip = nullptr;
  // a given start X that is all zero (xflag; not for host callbacks) needs no product
  if (x0_zero || op.kind == NYS_OP_CALLBACK) xflag = nullptr;
  const int64_t cover = std::max<int64_t>(std::max<int64_t>(k, 64), (x0_zero || xflag) ? n * k : 0);
  hipLaunchKernelGGL(pcg_start<T>, dim3(nblk(cover)), dim3(256), 0, s, mu_dev, b.mu, k, b.sc.ctr,
                     x0_zero ? X : (T*)nullptr, b.V, n * k, xflag);
  NYS_CHECK_LAUNCH();
  if (!x0_zero) {
    if (xflag) {
      hipLaunchKernelGGL(zero_test<T>, dim3((unsigned)std::min<int64_t>(nblk(n * k), 1024)), dim3(256), 0, s, X,
                         n * k, xflag);
      NYS_CHECK_LAUNCH();
      op.skip = xflag;
    }
    NYS_TRY(matvec<T>(op, X, k, b.mu, 1, mu_host[0], b.V, b, s));
    op.skip = nullptr;
  }
  NYS_TRY(pcg_setup<T>(n, k, P, b.mu, 1, B, b.V, b.R, b.Z, b.P, b.w, b.sc, tol, s));
  op.skip = b.sc.alldone;
  // device-info form (no compaction): block products skip column blocks whose
  // columns have all stopped (their products are not read: a stopped
  // column's alpha is 0); the host-polled form compacts such columns away
  op.coldone = dev_mode && k > 1 ? b.sc.done : nullptr;
  res.iters.assign(k, 0);
  res.status.assign(k, 0);
  res.rnorm2.assign(k, 0.0);
  res.bnorm2.assign(k, 0.0);
  // current column c is original column map[c]; Xc holds the active columns
  std::vector<int> map(k);
  for (int64_t c = 0; c < k; ++c) map[c] = (int)c;
  int64_t kc = k;
  T* Xc = X;
  bool compacted = false;
  std::vector<int> hi(k), hs(k), hd(k);
  std::vector<double> hr(k), hb(k);
  auto harvest = [&](int64_t kk, bool only_done) -> nys_status {
    NYS_HIP(hipMemcpyAsync(hi.data(), b.sc.iters, sizeof(int) * kk, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipMemcpyAsync(hs.data(), b.sc.status, sizeof(int) * kk, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipMemcpyAsync(hr.data(), b.sc.rnorm2, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipMemcpyAsync(hb.data(), b.sc.bnorm2, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
    for (int64_t c = 0; c < kk; ++c) {
      if (only_done && !hd[c]) continue;
      res.iters[map[c]] = hi[c];
      res.status[map[c]] = hs[c];
      res.rnorm2[map[c]] = hr[c];
      res.bnorm2[map[c]] = hb[c];
    }
    return NYS_OK;
  };
  int it = 0;
  int alldone_h = 0;
  // a single column learns whether the set-up already met tol from its first
  // snapshot; blocks read the flag now (their polls synchronise anyway)
  const bool snap_path = !dev_mode && kc == 1 && pinned_flags() != nullptr;
  if (!snap_path && !dev_mode) {
    NYS_HIP(hipMemcpyAsync(&alldone_h, b.sc.alldone, sizeof(int), hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
  }
  // Convergence polls cost a host round trip (~25 us).  check_every > 0 fixes
  // the interval; otherwise it is tuned from the measured iteration time so
  // that polling stays near 2.5% of the run (1 for costly products, up to 32
  // for cheap ones), which also bounds the iterations run past convergence.
  int interval = check_every > 0 ? check_every : 1;
  bool tune = check_every <= 0;
  const auto t_start = std::chrono::steady_clock::now();
  int last_poll = 0;
  // p^T A p from the product itself: X^T X, and square RBF products in float64
  const bool pvq_path = (op.kind == NYS_OP_XTX || (op.kind == NYS_OP_RBF && sizeof(T) == 8)) && pcg_pvq_ok(P, n);
  // one iteration on the current kc columns
  auto step = [&]() -> nys_status {
    const int par = it & 1;
    // single column with a partial-sum operator product: fused iteration
    const bool fused = kc == 1 && (op.kind == NYS_OP_XTX ||
                                   (op.kind == NYS_OP_RBF && (sizeof(T) == 8 || op.lowp != nullptr)));
    if (fused && pvq_path) {
      // the product also gives its p^T A p parts, so alpha needs no summed product
      int ng = 0, npvq = 0, npp = 0;
      NYS_TRY(op_matvec_partials<T>(op, b.P, b.opscr, b.opscr_elems, &ng, s, b.w.ppv, &npvq, &npp));
      if (npvq > 0)
        NYS_TRY(pcg_iteration_pvq<T>(n, P, b.mu, mu_host[map[0]], b.opscr, ng, b.w.ppv, npvq, npp, op.scale, b.V,
                                     Xc, b.R, b.Z, b.P, b.w, b.sc, par, tol, s));
      else
        NYS_TRY(pcg_iteration_fused<T>(n, P, b.mu, mu_host[map[0]], b.opscr, ng, op.scale, b.V, Xc, b.R, b.Z,
                                       b.P, b.w, b.sc, par, tol, s));
    } else if (fused) {
      int ng = 0;
      NYS_TRY(op_matvec_partials<T>(op, b.P, b.opscr, b.opscr_elems, &ng, s));
      NYS_TRY(pcg_iteration_fused<T>(n, P, b.mu, mu_host[map[0]], b.opscr, ng, op.scale, b.V, Xc, b.R, b.Z,
                                     b.P, b.w, b.sc, par, tol, s));
    } else {
      NYS_TRY(matvec<T>(op, b.P, kc, b.mu, 1, mu_host[map[0]], b.V, b, s));
      NYS_TRY(pcg_iteration<T>(n, kc, P, b.mu, 1, b.V, Xc, kc, b.R, b.Z, b.P, b.w, b.sc, par, tol, s));
    }
    ++it;
    return NYS_OK;
  };
  if (dev_mode) {
    while (it < maxit) NYS_TRY(step());
    res.sweeps = it;
    return NYS_OK;
  }
  // A single column needs no compaction, so its polls need not stop the
  // device: a batch is enqueued before the host waits for the snapshot
  // (iterations, residual) of the batch before it, which the device writes to
  // pinned memory.  Batch sizes come from the residual's measured rate of
  // decrease: the next batch holds the iterations predicted to remain beyond
  // the batch in flight (at most the poll interval), so few iterations are
  // enqueued past convergence (those return at once in every kernel).
  PcgSnap* hsnap = snap_path ? reinterpret_cast<PcgSnap*>(reinterpret_cast<char*>(pinned_flags()) + 64) : nullptr;
  bool have_final = false;  // final state of the column known from a snapshot
  PcgSnap fin{};
  if (hsnap) {
    int batch = 0, inflight = -1, inflight_n = 0, next_n = 1;
    int seqs[2] = {0, 0};
    bool have_prev = false;
    int prev_it = 0;
    double prev_rn2 = 0.0;
    while (true) {
      int slot = -1, n_now = 0;
      if (next_n > 0 && it < maxit) {
        n_now = next_n < maxit - it ? next_n : maxit - it;
        for (int j = 0; j < n_now; ++j) NYS_TRY(step());
        slot = batch & 1;
        ++batch;
        seqs[slot] = next_pinned_seq();
        NYS_TRY(pcg_snapshot(b.sc, hsnap + slot, seqs[slot], s));
      }
      const int wait_slot = inflight >= 0 ? inflight : slot;
      if (wait_slot < 0) break;  // iteration cap reached, nothing in flight
      if (!wait_pinned(&hsnap[wait_slot].seq, seqs[wait_slot], s)) return NYS_ERR_DEVICE;
      PcgSnap sp;
      {
        const volatile PcgSnap* v = hsnap + wait_slot;
        sp.alldone = v->alldone;
        sp.iters = v->iters;
        sp.status = v->status;
        sp.seq = v->seq;
        sp.rnorm2 = v->rnorm2;
        sp.bnorm2 = v->bnorm2;
      }
      int ahead = 0;  // iterations enqueued beyond the snapshot
      if (wait_slot == inflight && slot >= 0) {
        inflight = slot;
        inflight_n = n_now;
        ahead = n_now;
      } else {
        inflight = -1;
        inflight_n = 0;
      }
      if (sp.alldone || (it >= maxit && inflight < 0)) {
        have_final = true;
        fin = sp;
        break;
      }
      if (tune) {  // the first batch (one iteration) has finished
        const double per = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        const double want = 1e-3 / (per > 1e-9 ? per : 1e-9);
        interval = want < 1.0 ? 1 : want > 32.0 ? 32 : (int)std::ceil(want);
        tune = false;
      }
      next_n = interval;
      if (have_prev && sp.iters > prev_it && sp.rnorm2 > 0.0 && prev_rn2 > 0.0) {
        const double rate = (std::log(sp.rnorm2) - std::log(prev_rn2)) / (double)(sp.iters - prev_it);
        const double goal = std::log(tol * tol * sp.bnorm2);
        if (rate < 0.0 && std::isfinite(rate) && std::isfinite(goal)) {
          const double rem = (goal - std::log(sp.rnorm2)) / rate;
          if (std::isfinite(rem)) {
            const double left = std::ceil(rem) - ahead;
            next_n = left < 0.0 ? 0 : left > interval ? interval : (int)left;
          }
        }
      }
      if (inflight < 0 && next_n == 0) next_n = 1;  // nothing in flight: keep going
      have_prev = true;
      prev_it = sp.iters;
      prev_rn2 = sp.rnorm2;
      (void)inflight_n;
    }
  }
  while (!hsnap && !alldone_h && it < maxit) {
    NYS_TRY(step());
    if (it - last_poll >= interval || it == maxit) {
      last_poll = it;
      NYS_HIP(hipMemcpyAsync(&alldone_h, b.sc.alldone, sizeof(int), hipMemcpyDeviceToHost, s));
      if (kc > 1) NYS_HIP(hipMemcpyAsync(hd.data(), b.sc.done, sizeof(int) * kc, hipMemcpyDeviceToHost, s));
      NYS_HIP(hipStreamSynchronize(s));
      if (tune && it >= 3) {
        const double per =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count() / it;
        const double want = 1e-3 / (per > 1e-9 ? per : 1e-9);
        interval = want < 1.0 ? 1 : want > 32.0 ? 32 : (int)std::ceil(want);
        tune = false;
      }
      if (kc > 1 && !alldone_h && it < maxit) {
        std::vector<int> keep;
        for (int64_t c = 0; c < kc; ++c)
          if (!hd[c]) keep.push_back((int)c);
        const int64_t kn = (int64_t)keep.size();
        if (kn > 0 && kn < kc) {
          NYS_TRY(harvest(kc, true));
          NYS_TRY(upload_indices(b.cidx, keep, s));
          if (!compacted) {
            // X keeps every column (the finished ones are final); work on a copy
            hipLaunchKernelGGL((gather_idx<T, T>), dim3(nblk(n * kn)), dim3(256), 0, s, n, kc, X, b.cidx, kn,
                               b.Xw);
            NYS_CHECK_LAUNCH();
            Xc = b.Xw;
            compacted = true;
          } else {
            NYS_TRY(upload_indices(b.cmap, map, s));
            hipLaunchKernelGGL(scatter_idx_same<T>, dim3(nblk(n * kc)), dim3(256), 0, s, n, kc, Xc, b.cmap, k, X);
            hipLaunchKernelGGL((gather_idx<T, T>), dim3(nblk(n * kn)), dim3(256), 0, s, n, kc, Xc, b.cidx, kn,
                               b.V);
            NYS_CHECK_LAUNCH();
            NYS_HIP(hipMemcpyAsync(Xc, b.V, sizeof(T) * n * kn, hipMemcpyDeviceToDevice, s));
          }
          hipLaunchKernelGGL((gather_idx<T, T>), dim3(nblk(n * kn)), dim3(256), 0, s, n, kc, b.R, b.cidx, kn, b.V);
          NYS_CHECK_LAUNCH();
          NYS_HIP(hipMemcpyAsync(b.R, b.V, sizeof(T) * n * kn, hipMemcpyDeviceToDevice, s));
          hipLaunchKernelGGL((gather_idx<T, T>), dim3(nblk(n * kn)), dim3(256), 0, s, n, kc, b.P, b.cidx, kn, b.V);
          NYS_CHECK_LAUNCH();
          NYS_HIP(hipMemcpyAsync(b.P, b.V, sizeof(T) * n * kn, hipMemcpyDeviceToDevice, s));
          hipLaunchKernelGGL(compact_scalars, dim3(1), dim3(256), 0, s, b.sc, b.mu, kc, b.cidx, kn);
          NYS_CHECK_LAUNCH();
          std::vector<int> nm(kn);
          for (int64_t j = 0; j < kn; ++j) nm[j] = map[keep[j]];
          map.swap(nm);
          kc = kn;
        }
      }
    }
  }
  if (have_final && !compacted) {  // single column: the last snapshot holds its results
    res.iters[map[0]] = fin.iters;
    res.status[map[0]] = fin.status;
    res.rnorm2[map[0]] = fin.rnorm2;
    res.bnorm2[map[0]] = fin.bnorm2;
  } else {
    for (int64_t c = 0; c < kc; ++c) hd[c] = 1;
    NYS_TRY(harvest(kc, false));
  }
  if (compacted) {
    NYS_TRY(upload_indices(b.cmap, map, s));
    hipLaunchKernelGGL(scatter_idx_same<T>, dim3(nblk(n * kc)), dim3(256), 0, s, n, kc, Xc, b.cmap, k, X);
    NYS_CHECK_LAUNCH();
  }
  res.sweeps = it;
  if (hsnap) {  // iterations enqueued past convergence did not run
    res.sweeps = 0;
    for (int64_t c = 0; c < k; ++c) res.sweeps = res.iters[c] > res.sweeps ? res.iters[c] : res.sweeps;
  }
  return NYS_OK;
}

// R64 = B64 - (A + mu_c I) X64 in float64 (mu_dev: one mu per column);
// returns per-column relative residuals.
nys_status true_residual(const OpDesc& op, int64_t k, const double* mu_dev, double mu0, SolveWs& w,
                         std::vector<double>& relres, hipStream_t s, bool maybe_zero = false) {
  const int64_t n = op.n;
  OpDesc o = op;
  o.skip = nullptr;
  if (maybe_zero && op.kind != NYS_OP_CALLBACK) {
    // an all-zero X (the usual start) needs no product: V stays zero
    hipLaunchKernelGGL(zero_flag_init, dim3(nblk(n * k)), dim3(256), 0, s, w.V64, n * k, w.xzero);
    hipLaunchKernelGGL(zero_test<double>, dim3((unsigned)std::min<int64_t>(nblk(n * k), 1024)), dim3(256), 0, s,
                       w.X64, n * k, w.xzero);
    NYS_CHECK_LAUNCH();
    o.skip = w.xzero;
  }
  if (k == 1 && (op.kind == NYS_OP_XTX || op.kind == NYS_OP_DENSE))
    NYS_TRY(op_matvec<double>(o, w.X64, mu0, w.V64, w.d.opscr, w.d.opscr_elems, s));
  else
    NYS_TRY(op_apply_f64(o, w.X64, k, k, mu_dev, 1, w.V64, k, w.d.opscr, w.d.opscr_elems, s));
  const int g = 64;
  hipLaunchKernelGGL(residual_norms, dim3(g), dim3(256), 0, s, n, k, w.B64, w.V64, w.R64, w.dots);
  NYS_CHECK_LAUNCH();
  if (ResSnap* rs = k == 1 ? res_snap() : nullptr) {
    // one column: the device sums the partials and the host spins on pinned
    // memory instead of synchronising the stream
    const int seq = next_pinned_seq();
    hipLaunchKernelGGL(residual_snapshot, dim3(1), dim3(1), 0, s, w.dots, g, rs, seq);
    NYS_CHECK_LAUNCH();
    if (!wait_pinned(&rs->seq, seq, s)) return NYS_ERR_DEVICE;
    const volatile ResSnap* v = rs;
    const double rv = v->relres;
    relres.assign(1, rv);
    return NYS_OK;
  }
  std::vector<double> h(2 * g * k);
  NYS_HIP(hipMemcpyAsync(h.data(), w.dots, sizeof(double) * 2 * g * k, hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  relres.assign(k, 0.0);
  for (int64_t c = 0; c < k; ++c) {
    double rr = 0.0, bb = 0.0;
    for (int q = 0; q < g; ++q) {
      rr += h[q * k + c];
      bb += h[(g + q) * k + c];
    }
    relres[c] = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  }
  return NYS_OK;
}

// R64 = B64 - (A + mu_c I) X64 and relres_d[c] on the device (no read-back)
nys_status true_residual_dev(const OpDesc& op, int64_t k, const double* mu_dev, double mu0, SolveWs& w,
                             hipStream_t s) {
  const int64_t n = op.n;
  OpDesc o = op;
  o.skip = nullptr;
  if (k == 1 && (op.kind == NYS_OP_XTX || op.kind == NYS_OP_DENSE))
    NYS_TRY(op_matvec<double>(o, w.X64, mu0, w.V64, w.d.opscr, w.d.opscr_elems, s));
  else
    NYS_TRY(op_apply_f64(o, w.X64, k, k, mu_dev, 1, w.V64, k, w.d.opscr, w.d.opscr_elems, s));
  const int g = 64;
  hipLaunchKernelGGL(residual_norms, dim3(g), dim3(256), 0, s, n, k, w.B64, w.V64, w.R64, w.dots);
  hipLaunchKernelGGL(relres_from_parts, dim3(nblk(k)), dim3(256), 0, s, k, g, w.dots, w.relres_d);
  NYS_CHECK_LAUNCH();
  return NYS_OK;
}

// Device-info form of the solve (opts.device_info = 1): fixed iteration
// counts, device flags for every per-column decision, results written to the
// caller's device arrays.  Enqueues kernels only.
nys_status solve_device_info(const OpDesc& op, const OpDesc& opf, const PrecDesc& P,
                             const std::vector<double>& mu_col, int64_t k, const nys_solve_opts* o,
                             nys_solve_info* info, SolveWs& w, hipStream_t s) {
  const int64_t n = op.n;
  const double tol = o->tol;
  const int maxit = o->maxit > 0 ? o->maxit : 500;
  const int prec = o->prec;
  int32_t* oi = info ? info->iters : nullptr;
  double* orr = info ? info->relres : nullptr;
  int32_t* ost = info ? info->status : nullptr;
  int refine_steps = 0, total = 0;
  if (prec == NYS_PREC_FP64) {
    PcgResult r;
    NYS_TRY(pcg_run<double>(op, P, k, w.mu, mu_col, w.B64, w.X64, false, tol, maxit, 0, w.d, r, s, true));
    total = r.sweeps;
    NYS_TRY(true_residual_dev(op, k, w.mu, mu_col[0], w, s));
    hipLaunchKernelGGL(write_device_info, dim3(nblk(k)), dim3(256), 0, s, k, w.d.sc.iters, w.d.sc.status,
                       (const int*)nullptr, w.relres_d, tol, oi, orr, ost);
    NYS_CHECK_LAUNCH();
  } else if (prec == NYS_PREC_FP32) {
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.B64, k, k, w.f.B, k);
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.X64, k, k, w.f.X, k);
    NYS_CHECK_LAUNCH();
    PcgResult r;
    NYS_TRY(pcg_run<float>(opf, P, k, w.mu, mu_col, w.f.B, w.f.X, false, tol, maxit, 0, w.f, r, s, true));
    total = r.sweeps;
    hipLaunchKernelGGL((gather_cols<float, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.f.X, k, k, w.X64, k);
    NYS_CHECK_LAUNCH();
    NYS_TRY(true_residual_dev(op, k, w.mu, mu_col[0], w, s));
    hipLaunchKernelGGL(write_device_info, dim3(nblk(k)), dim3(256), 0, s, k, w.f.sc.iters, w.f.sc.status,
                       (const int*)nullptr, w.relres_d, tol, oi, orr, ost);
    NYS_CHECK_LAUNCH();
  } else {
    const int max_ref = o->max_refine > 0 ? o->max_refine : 10;
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
    hipLaunchKernelGGL(init_refine_state, dim3(nblk(k)), dim3(256), 0, s, k, w.prev_d, w.iters_d, w.brk_d);
    NYS_CHECK_LAUNCH();
    NYS_TRY(true_residual_dev(op, k, w.mu, mu_col[0], w, s));
    for (int step = 0; step < max_ref; ++step) {
      hipLaunchKernelGGL(refine_select, dim3(nblk(k)), dim3(256), 0, s, k, w.relres_d, w.prev_d, w.brk_d,
                         w.active_d, tol);
      hipLaunchKernelGGL(gather_active, dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.R64, w.active_d, w.f.B);
      NYS_CHECK_LAUNCH();
      PcgResult r;
      NYS_TRY(pcg_run<float>(opf, P, k, w.mu, mu_col, w.f.B, w.f.X, true, itol, maxit, 0, w.f, r, s, true));
      hipLaunchKernelGGL(add_to<float>, dim3(nblk(n * k)), dim3(256), 0, s, w.X64, w.f.X, n * k);
      hipLaunchKernelGGL(refine_count, dim3(nblk(k)), dim3(256), 0, s, k, w.f.sc, w.iters_d, w.brk_d);
      NYS_CHECK_LAUNCH();
      total += r.sweeps;
      ++refine_steps;
      NYS_TRY(true_residual_dev(op, k, w.mu, mu_col[0], w, s));
    }
    hipLaunchKernelGGL(write_device_info, dim3(nblk(k)), dim3(256), 0, s, k, w.iters_d, (const int*)nullptr,
                       w.brk_d, w.relres_d, tol, oi, orr, ost);
    NYS_CHECK_LAUNCH();
  }
  if (info) {
    info->refine_steps = refine_steps;
    info->total_iters = total;
  }
  return NYS_OK;
}

nys_status solve_impl(const OpDesc& op, const PrecDesc& P, const double* mu, int64_t nmu,
                      const double* B, int64_t nrhs, int64_t ldb, double* X, int64_t ldx,
                      const nys_solve_opts* o, nys_solve_info* info, SolveWs& w, hipStream_t s) {
  const int64_t n = op.n, k = nmu * nrhs;
  const double tol = o->tol;
  const int maxit = o->maxit > 0 ? o->maxit : 500;
  const int check = o->check_every;  // <= 0: tuned from the measured iteration time
  const int prec = o->prec;
  // one mu per column: column c = m * nrhs + r solves with mu[m]
  std::vector<double> mu_col(k);
  for (int64_t c = 0; c < k; ++c) mu_col[c] = mu[c / nrhs];
  NYS_TRY(set_mu(w.mu, mu_col.data(), k, s));
  // contiguous float64 copies of B (expanded over the mu grid) and X
  hipLaunchKernelGGL((gather_cols<double, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, B, ldb,
                     nrhs, w.B64, k);
  NYS_CHECK_LAUNCH();
  hipLaunchKernelGGL((gather_cols<double, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, X, ldx,
                     k, w.X64, k);
  NYS_CHECK_LAUNCH();
  std::vector<int> iters(k, 0), status(k, NYS_NOT_CONVERGED);
  std::vector<double> relres(k, 0.0);
  int refine_steps = 0, total = 0;
  // operator for the float32 inner solves (prepared points for the RBF kernels)
  OpDesc opf = op;
  if (rbf_lowp_mode(op, prec)) {
    NYS_TRY(rbf_lowp_prepare(op, w.lowp_buf, w.L, s));
    opf.lowp = &w.L;
    opf.gram = rbf_gram(prec);
  }
  if (o->device_info) {
    NYS_TRY(solve_device_info(op, opf, P, mu_col, k, o, info, w, s));
    hipLaunchKernelGGL((gather_cols<double, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.X64, k, k, X, ldx);
    NYS_CHECK_LAUNCH();
    return NYS_OK;
  }
  if (prec == NYS_PREC_FP64) {
    PcgResult r;
    NYS_TRY(pcg_run<double>(op, P, k, w.mu, mu_col, w.B64, w.X64, false, tol, maxit, check, w.d, r, s, false,
                            w.xzero));
    iters = r.iters;
    status = r.status;
    total = r.sweeps;
    NYS_TRY(true_residual(op, k, w.mu, mu_col[0], w, relres, s));
    // The stopping test reads the recursive residual; where the true residual
    // has drifted above tol, solve (A + mu I) d = r for the correction (a few
    // iterations: r is already within a small factor of tol ||b||).
    for (int pass = 0; pass < 3; ++pass) {
      std::vector<int> act;
      std::vector<double> mu_act;
      double worst = 0.0;
      for (int64_t c = 0; c < k; ++c)
        if (!(relres[c] <= tol) && status[c] == NYS_OK) {
          act.push_back((int)c);
          mu_act.push_back(mu_col[c]);
          worst = relres[c] > worst ? relres[c] : worst;
        }
      const int64_t ka = (int64_t)act.size();
      if (ka == 0 || !std::isfinite(worst)) break;
      NYS_TRY(upload_indices(w.omap, act, s));
      hipLaunchKernelGGL((gather_idx<double, double>), dim3(nblk(n * ka)), dim3(256), 0, s, n, k, w.R64, w.omap,
                         ka, w.d.B);
      hipLaunchKernelGGL((gather_idx<double, double>), dim3(1), dim3(256), 0, s, (int64_t)1, k, w.mu, w.omap, ka,
                         w.mu_act);
      NYS_CHECK_LAUNCH();
      PcgResult rc;
      NYS_TRY(pcg_run<double>(op, P, ka, w.mu_act, mu_act, w.d.B, w.d.X, true, 0.5 * tol / worst, maxit, check,
                              w.d, rc, s));
      hipLaunchKernelGGL((scatter_idx<double, true>), dim3(nblk(n * ka)), dim3(256), 0, s, n, ka, w.d.X, w.omap,
                         k, w.X64);
      NYS_CHECK_LAUNCH();
      for (int64_t j = 0; j < ka; ++j) {
        iters[act[j]] += rc.iters[j];
        if (rc.status[j] == NYS_ERR_BREAKDOWN) status[act[j]] = NYS_ERR_BREAKDOWN;
      }
      total += rc.sweeps;
      NYS_TRY(true_residual(op, k, w.mu, mu_col[0], w, relres, s));
    }
    for (int64_t c = 0; c < k; ++c)
      if (status[c] == NYS_OK && !(relres[c] <= tol)) status[c] = NYS_NOT_CONVERGED;
  } else if (prec == NYS_PREC_FP32) {
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.B64, k,
                       k, w.f.B, k);
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.X64, k,
                       k, w.f.X, k);
    NYS_CHECK_LAUNCH();
    PcgResult r;
    NYS_TRY(pcg_run<float>(opf, P, k, w.mu, mu_col, w.f.B, w.f.X, false, tol, maxit, check, w.f, r, s));
    hipLaunchKernelGGL((gather_cols<float, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.f.X, k,
                       k, w.X64, k);
    NYS_CHECK_LAUNCH();
    iters = r.iters;
    status = r.status;
    total = r.sweeps;
    NYS_TRY(true_residual(op, k, w.mu, mu_col[0], w, relres, s));
  } else {
    // iterative refinement: float64 residual and update, float32 inner PCG on
    // the columns that have not yet met the tolerance
    const int max_ref = o->max_refine > 0 ? o->max_refine : 10;
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
    NYS_TRY(true_residual(op, k, w.mu, mu_col[0], w, relres, s, true));
    std::vector<double> prev(relres);
    for (int step = 0; step < max_ref; ++step) {
      std::vector<int> act;
      std::vector<double> mu_act;
      for (int64_t c = 0; c < k; ++c) {
        // a column whose inner solve broke down, whose residual grew (the
        // reduced-precision operator is not positive definite at this mu) or
        // stagnated (less than a 2x reduction: the float64 residual is at its
        // rounding floor) is not refined further; it is reported as not
        // converged unless it already meets tol
        if (step > 0 && (status[c] == NYS_ERR_BREAKDOWN || !(relres[c] <= 0.5 * prev[c]))) continue;
        if (!(relres[c] <= tol)) {
          act.push_back((int)c);
          mu_act.push_back(mu_col[c]);
        }
      }
      prev = relres;
      const int64_t ka = (int64_t)act.size();
      if (ka == 0) break;
      PcgResult r;
      if (ka == k) {  // every column: no index map
        hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.R64, k, k,
                           w.f.B, k);
        NYS_CHECK_LAUNCH();
        NYS_TRY(pcg_run<float>(opf, P, k, w.mu, mu_act, w.f.B, w.f.X, true, itol, maxit, check, w.f, r, s));
        hipLaunchKernelGGL(add_to<float>, dim3(nblk(n * k)), dim3(256), 0, s, w.X64, w.f.X, n * k);
        NYS_CHECK_LAUNCH();
      } else {
        NYS_TRY(upload_indices(w.omap, act, s));
        hipLaunchKernelGGL((gather_idx<double, float>), dim3(nblk(n * ka)), dim3(256), 0, s, n, k, w.R64, w.omap,
                           ka, w.f.B);
        hipLaunchKernelGGL((gather_idx<double, double>), dim3(1), dim3(256), 0, s, (int64_t)1, k, w.mu, w.omap,
                           ka, w.mu_act);
        NYS_CHECK_LAUNCH();
        NYS_TRY(pcg_run<float>(opf, P, ka, w.mu_act, mu_act, w.f.B, w.f.X, true, itol, maxit, check, w.f, r, s));
        hipLaunchKernelGGL((scatter_idx<float, true>), dim3(nblk(n * ka)), dim3(256), 0, s, n, ka, w.f.X, w.omap,
                           k, w.X64);
        NYS_CHECK_LAUNCH();
      }
      for (int64_t j = 0; j < ka; ++j) {
        iters[act[j]] += r.iters[j];
        if (r.status[j] == NYS_ERR_BREAKDOWN) status[act[j]] = NYS_ERR_BREAKDOWN;
      }
      total += r.sweeps;
      ++refine_steps;
      NYS_TRY(true_residual(op, k, w.mu, mu_col[0], w, relres, s));
      if (verbose()) {
        double worst = 0.0;
        for (int64_t c = 0; c < k; ++c) worst = relres[c] > worst ? relres[c] : worst;
        std::fprintf(stderr, "[nyspcg] refinement %d: %lld columns, inner iterations %d, max relres %.3e\n",
                     refine_steps, (long long)ka, r.sweeps, worst);
        std::fflush(stderr);
      }
    }
    for (int64_t c = 0; c < k; ++c)
      if (status[c] != NYS_ERR_BREAKDOWN) status[c] = relres[c] <= tol ? NYS_OK : NYS_NOT_CONVERGED;
  }
  // write back X, and wait for it (a tag in pinned memory when there is
  // some: the host spins instead of synchronising the stream)
  hipLaunchKernelGGL((gather_cols<double, double>), dim3(nblk(n * k)), dim3(256), 0, s, n, k, w.X64, k,
                     k, X, ldx);
  NYS_CHECK_LAUNCH();
  if (ResSnap* rs = res_snap()) {
    const int seq = next_pinned_seq();
    hipLaunchKernelGGL(residual_snapshot, dim3(1), dim3(1), 0, s, nullptr, 0, rs, seq);
    NYS_CHECK_LAUNCH();
    if (!wait_pinned(&rs->seq, seq, s)) return NYS_ERR_DEVICE;
  } else {
    NYS_HIP(hipStreamSynchronize(s));
  }
  nys_status worst = NYS_OK;
  for (int64_t c = 0; c < k; ++c) {
    if (status[c] == NYS_ERR_BREAKDOWN) worst = NYS_ERR_BREAKDOWN;
    else if (status[c] != NYS_OK && worst == NYS_OK) worst = NYS_NOT_CONVERGED;
  }
  if (info) {
    for (int64_t c = 0; c < k; ++c) {
      if (info->iters) info->iters[c] = iters[c];
      if (info->status) info->status[c] = status[c];
      if (info->relres) info->relres[c] = relres[c];
    }
    info->refine_steps = refine_steps;
    info->total_iters = total;
  }
  if (worst == NYS_ERR_BREAKDOWN) set_error("PCG breakdown: p^T (A + mu I) p <= 0");
  else if (worst == NYS_NOT_CONVERGED) set_error("PCG did not reach the tolerance within maxit");
  return worst;
}

nys_status check_solve_common(const OpDesc& op, const PrecDesc& P, const double* mu, int64_t nmu,
                              const nys_solve_opts* o, hipStream_t s) {
  NYS_ARG(o != nullptr, "solve options are NULL");
  NYS_ARG(o->tol > 0.0 && std::isfinite(o->tol), "tol must be > 0");
  NYS_ARG(o->prec >= NYS_PREC_FP64 && o->prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  NYS_ARG(P.n == op.n, "preconditioner n (%lld) != operator n (%lld)", (long long)P.n, (long long)op.n);
  NYS_ARG(mu != nullptr && nmu >= 1, "mu array is empty");
  NYS_ARG(o->device_info == 0 || o->device_info == 1, "device_info must be 0 or 1");
  if (o->device_info) {
    // nothing is read from the device: mu > 0 keeps lam_l + mu > 0 for the
    // lam >= 0 that the factorisation returns
    for (int64_t i = 0; i < nmu; ++i)
      NYS_ARG(std::isfinite(mu[i]) && mu[i] > 0.0, "device-info solves need every mu finite and > 0 (mu[%lld])",
              (long long)i);
    if (o->prec != NYS_PREC_FP64 && op.kind == NYS_OP_RBF)
      NYS_ARG(op.cols <= 32, "reduced-precision RBF modes need d <= 32");
    return NYS_OK;
  }
  bool any_zero = false;
  for (int64_t i = 0; i < nmu; ++i) {
    NYS_ARG(std::isfinite(mu[i]) && mu[i] >= 0.0, "mu[%lld] must be finite and >= 0", (long long)i);
    any_zero = any_zero || mu[i] == 0.0;
  }
  // lam >= 0 (the preconditioner's contract), so only mu = 0 needs lam_l
  // itself, which costs a device round trip
  if (any_zero) {
    double lam_l = 0.0;
    NYS_HIP(hipMemcpyAsync(&lam_l, P.lam + (P.ell - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
    NYS_ARG(lam_l > 0.0, "lam_l + mu must be > 0 (mu = 0 needs a positive lam_l)");
  }
  if (o->prec != NYS_PREC_FP64 && op.kind == NYS_OP_RBF)
    NYS_ARG(op.cols <= 32, "reduced-precision RBF modes need d <= 32");
  return NYS_OK;
}

}  // namespace
}  // namespace nys

// ---------------------------------------------------------------- static scratch
// Device memory of the allocation-free solve (nys_pcg_solve_noalloc): one
// array per GPU, held by the code object until the process ends.  In host
// code `scratch` only names the symbol; its device address on the current GPU
// comes from hipGetSymbolAddress (kept per device below) and is what kernels
// receive.
static constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace nys {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device with
// that device current.
nys_status static_scratch(void** out) {
  int dev = -1;
  NYS_HIP(hipGetDevice(&dev));
  NYS_ARG(dev >= 0 && dev < kMaxDevices, "device index %d out of range for the static scratch", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return NYS_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NYS_OK;
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

const char* nys_last_error(void) { return g_err; }

const char* nys_version(void) { return "nyspcg 0.1 (gfx950)"; }

nys_status nys_timing_begin(void) {
  for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
  g_timer.ev.clear();
  g_timer.on = true;
  return NYS_OK;
}

nys_status nys_timing_end(double* avg_ms, int64_t* launches) {
  NYS_ARG(avg_ms != nullptr && launches != nullptr, "nys_timing_end: NULL argument");
  const bool was_on = g_timer.on;
  g_timer.on = false;
  double total = 0.0;
  int64_t count = 0;
  nys_status st = NYS_OK;
  const size_t pairs = g_timer.ev.size() / 2;
  for (size_t i = 0; i < pairs && st == NYS_OK; ++i) {
    hipEvent_t a = g_timer.ev[2 * i], b = g_timer.ev[2 * i + 1];
    float ms = 0.0f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      set_error("nys_timing_end: event timing failed");
      st = NYS_ERR_DEVICE;
      break;
    }
    total += ms;
    ++count;
  }
  for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
  g_timer.ev.clear();
  if (st != NYS_OK) return st;
  NYS_ARG(was_on, "nys_timing_end without nys_timing_begin (or event creation failed)");
  *launches = count;
  *avg_ms = count ? total / (double)count : 0.0;
  return NYS_OK;
}

size_t nys_workspace_size(const nys_operator* A, int64_t ell, int64_t ncols, int32_t prec) {
  OpDesc op;
  if (check_op(A, op) != NYS_OK || ell < 1 || ncols < 1) return 0;
  size_t best = 0;
  {
    Arena a(nullptr, 0);
    SketchWs w;
    carve_sketch(a, op, ell, prec, w);
    best = a.off > best ? a.off : best;
  }
  {
    Arena a(nullptr, 0);
    FactorWs w;
    carve_factor(a, op.n, ell, w);
    best = a.off > best ? a.off : best;
  }
  {
    Arena a(nullptr, 0);
    SolveWs w;
    carve_solve(a, op, ell, ncols, prec, w);
    // the adjoint's extra buffers: two row vectors, dot partials and the dK/dsigma partials
    const int64_t rmax = op.rows > op.n ? op.rows : op.n;
    size_t extra = (size_t)(4 * 256) * (size_t)op.n * sizeof(double) + 2 * (size_t)rmax * sizeof(double) +
                   rbf_lowp_bytes(op.n) + 8192 + 4 * 256;
    best = a.off + extra > best ? a.off + extra : best;
  }
  return best + 256;
}

nys_status nys_gaussian(uint64_t seed, int64_t n, int64_t ell, double* out, int64_t ld,
                        void* stream) {
  NYS_ARG(n >= 1 && ell >= 1 && ld >= ell && out != nullptr, "nys_gaussian: invalid shape");
  return gaussian(seed, n, ell, out, ld, S(stream));
}

nys_status nys_sketch(const nys_operator* A, int64_t ell, uint64_t seed, const double* omega0,
                      double* Omega, double* Y, int32_t prec, void* ws, size_t ws_bytes,
                      void* stream) {
  OpDesc op;
  NYS_TRY(check_op(A, op));
  const int64_t n = op.n, l = ell;
  NYS_ARG(l >= 1 && l <= n, "sketch size ell = %lld must satisfy 1 <= ell <= n = %lld", (long long)l,
          (long long)n);
  NYS_ARG(l <= 2048, "sketch size > 2048 not supported");
  NYS_ARG(Omega != nullptr && Y != nullptr, "Omega / Y is NULL");
  NYS_ARG(prec >= NYS_PREC_FP64 && prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  Arena a(ws, ws_bytes);
  SketchWs w;
  carve_sketch(a, op, l, prec, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = S(stream);
  if (omega0) NYS_HIP(hipMemcpyAsync(Omega, omega0, sizeof(double) * n * l, hipMemcpyDeviceToDevice, s));
  else NYS_TRY(gaussian(seed, n, l, Omega, l, s));
  int passes = 1;
  NYS_TRY(cholqr(Omega, Y, n, l, omega0 == nullptr, w.c, &passes, s));
  // with pinned host memory the pivot flags are read while Y = A Omega runs,
  // and the call returns with the product still enqueued
  PivotSnap* hsnap = pivot_snap();
  int seq = 0;
  if (hsnap) {
    seq = publish_pivots(w.c.info, passes, nullptr, hsnap, s);
    NYS_CHECK_LAUNCH();
  }
  if (rbf_lowp_mode(op, prec)) {
    NYS_ARG(op.cols <= 32, "reduced-precision RBF modes need d <= 32");
    // Y = K Omega with the reduced-precision Gram tiles, float32 accumulation
    RbfLowp L;
    NYS_TRY(rbf_lowp_prepare(op, w.lowp_buf, L, s));
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * l)), dim3(256), 0, s, n, l, Omega, l,
                       l, w.Om32, l);
    NYS_CHECK_LAUNCH();
    NYS_TRY(rbf_lowp_kv(L, rbf_gram(prec), w.Om32, l, l, nullptr, 1, w.Y32, l, w.f32scr, w.f32scr_elems, nullptr,
                        s));
    hipLaunchKernelGGL((gather_cols<float, double>), dim3(nblk(n * l)), dim3(256), 0, s, n, l, w.Y32, l,
                       l, Y, l);
    NYS_CHECK_LAUNCH();
  } else if (sketch_f32(op, prec)) {
    // Y = X^T (X Omega): float32 MFMA, or bf16 MFMA on the hi/lo split (bf16x3 mode)
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * l)), dim3(256), 0, s, n, l, Omega, l,
                       l, w.Om32, l);
    NYS_CHECK_LAUNCH();
    const float* X = static_cast<const float*>(op.data);
    if (prec == NYS_PREC_BF16X3_REFINE64) {  // products on bf16 MFMA (hi/lo split)
      NYS_TRY(gemm_bf16x3(false, false, op.rows, l, n, 1.0f, X, op.ld, w.Om32, l, 0.0f, w.T32, l, w.f32scr,
                          w.f32scr_elems, s));
      if (op.w) NYS_TRY(scale_rows<float>(w.T32, op.rows, l, op.w, s));  // X^T D X: D between the products
      NYS_TRY(gemm_bf16x3(true, false, n, l, op.rows, (float)op.scale, X, op.ld, w.T32, l, 0.0f, w.Y32, l,
                          w.f32scr, w.f32scr_elems, s));
    } else {
      NYS_TRY((gemm<float, float, float>(false, false, op.rows, l, n, 1.0f, X, op.ld, w.Om32, l, 0.0f,
                                         w.T32, l, w.f32scr, w.f32scr_elems, s)));
      if (op.w) NYS_TRY(scale_rows<float>(w.T32, op.rows, l, op.w, s));
      NYS_TRY((gemm<float, float, float>(true, false, n, l, op.rows, (float)op.scale, X, op.ld, w.T32, l,
                                         0.0f, w.Y32, l, w.f32scr, w.f32scr_elems, s)));
    }
    hipLaunchKernelGGL((gather_cols<float, double>), dim3(nblk(n * l)), dim3(256), 0, s, n, l, w.Y32, l,
                       l, Y, l);
    NYS_CHECK_LAUNCH();
  } else {
    NYS_TRY(op_apply_f64(op, Omega, l, l, nullptr, 1, Y, l, w.opscr, w.opscr_elems, s));
  }
  int info[2] = {0, 0};
  if (hsnap) {
    if (!wait_pinned(&hsnap->seq, seq, s)) return NYS_ERR_DEVICE;
    const volatile PivotSnap* v = hsnap;
    info[0] = v->info[0];
    info[1] = v->info[1];
  } else {
    NYS_HIP(hipMemcpyAsync(info, w.c.info, sizeof(int) * passes, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
  }
  if (info[0] != 0 || info[1] != 0) {
    set_error("test matrix is numerically rank deficient (CholeskyQR pivot %d/%d)", info[0], info[1]);
    return NYS_ERR_NOT_PSD;
  }
  return NYS_OK;
}

nys_status nys_factor(const double* Omega, double* Y, nys_precond* P, int32_t prec, void* ws, size_t ws_bytes,
                      void* stream) {
  NYS_ARG(P != nullptr && Omega != nullptr && Y != nullptr, "nys_factor: NULL argument");
  PrecDesc pd;
  NYS_TRY(check_prec(P, pd));
  const int64_t n = P->n, l = P->ell;
  Arena a(ws, ws_bytes);
  FactorWs w;
  carve_factor(a, n, l, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = S(stream);
  Core& c = w.c;
  // nu = eps(||Y||_F) (float64 sketch); a sketch computed in reduced
  // precision carries relative errors up to u_rel, so the shift is raised to
  // u_rel ||Y||_F, which keeps Omega^T Y_nu positive definite
  NYS_ARG(prec >= NYS_PREC_FP64 && prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  const double u_rel = prec == NYS_PREC_FP64 ? 0.0 : prec == NYS_PREC_BF16X3_REFINE64 ? 3.0517578125e-05
                                                                                      : 9.5367431640625e-07;
  NYS_TRY(frob_shift(Y, n * l, c.part, c.nu, u_rel, s));
  NYS_TRY(add_shift(Y, Omega, n * l, c.nu, 1.0, s));
  // B = Y_nu C^{-1} = Y_nu L^{-T}, then the Gram B^T B of the thin SVD of B
  // (B^T B = W S W^T:  U = B W S^{-1/2}, lam = max(0, S - nu))
  const auto b_and_gram = [&]() -> nys_status {
    NYS_TRY(tri_inverse(c.L, l, c.Dinv, c.Linv, s));
    NYS_TRY((gemm<double, double, double>(false, true, n, l, l, 1.0, Y, l, c.Linv, l, 0.0, w.B, l, c.gscr,
                                          c.gscr_elems, s)));
    return gemm<double, double, double>(true, false, l, l, n, 1.0, w.B, l, w.B, l, 0.0, c.G, l, c.gscr,
                                        c.gscr_elems, s);
  };
  // With pinned host memory the pivot flag and the shift are published there
  // and B and its Gram are enqueued before the host reads them, so the device
  // does not idle on the round trip; after a failed pivot they are discarded
  // (they read Y_nu and write only B, L^{-1} and the Gram, which the retry
  // recomputes).
  PivotSnap* hsnap = pivot_snap();
  int info = 0;
  double nu = 0.0;
  for (int attempt = 0; attempt <= 3; ++attempt) {
    if (attempt > 0) {  // nu <- 10 nu: Y_10nu = Y_nu + 9 nu Omega
      NYS_TRY(add_shift(Y, Omega, n * l, c.nu, 9.0, s));
      NYS_TRY(scale_device_scalar(c.nu, 10.0, s));
    }
    // C^T C = Omega^T Y_nu  (lower factor L = C^T)
    NYS_TRY((gemm<double, double, double>(true, false, l, l, n, 1.0, Omega, l, Y, l, 0.0, c.G, l, c.gscr,
                                          c.gscr_elems, s)));
    NYS_TRY(cholesky(c.G, l, c.L, c.Dinv, c.info, s));
    if (hsnap) {
      const int seq = publish_pivots(c.info, 1, c.nu, hsnap, s);
      NYS_CHECK_LAUNCH();
      NYS_TRY(b_and_gram());
      if (!wait_pinned(&hsnap->seq, seq, s)) return NYS_ERR_DEVICE;
      const volatile PivotSnap* v = hsnap;
      info = v->info[0];
      nu = v->nu;
    } else {
      NYS_HIP(hipMemcpyAsync(&info, c.info, sizeof(int), hipMemcpyDeviceToHost, s));
      NYS_HIP(hipStreamSynchronize(s));
    }
    if (info == 0) break;
  }
  if (info != 0) {
    set_error("Cholesky of Omega^T Y_nu failed at column %d after shift retries", info - 1);
    return NYS_ERR_NOT_PSD;
  }
  if (!hsnap) NYS_TRY(b_and_gram());
  // eigenvectors kept in float32 need off-diagonal ratios ~1e-8, not ~1e-16
  NYS_TRY(sym_eig(c.G, l, c.eig, c.flags, kMaxSweeps, c.sweeps, c.conv, c.T, P->lam, c.sig2,
                  c.nu, s, P->dtype == NYS_F32 ? NYS_JACOBI_RATIO_F32 : 1e-9));
  if (P->dtype == NYS_F64) {
    NYS_TRY((gemm<double, double, double>(false, false, n, l, l, 1.0, w.B, l, c.T, l, 0.0,
                                          static_cast<double*>(P->U), P->ldu, c.gscr, c.gscr_elems, s)));
  } else {
    NYS_TRY((gemm<double, double, double>(false, false, n, l, l, 1.0, w.B, l, c.T, l, 0.0, Y, l, c.gscr,
                                          c.gscr_elems, s)));
    hipLaunchKernelGGL((gather_cols<double, float>), dim3(nblk(n * l)), dim3(256), 0, s, n, l, Y, l, l,
                       static_cast<float*>(P->U), P->ldu);
    NYS_CHECK_LAUNCH();
  }
  if (hsnap && !verbose()) {
    // nu came with the pivot flag; U and lam are complete when the stream
    // reaches this point (the call returns once their kernels are enqueued)
    P->nu = nu;
    return NYS_OK;
  }
  int sweeps = 0;
  NYS_HIP(hipMemcpyAsync(&nu, c.nu, sizeof(double), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipMemcpyAsync(&sweeps, c.sweeps, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_HIP(hipStreamSynchronize(s));
  if (verbose())
    std::fprintf(stderr, "[nyspcg] factor n=%lld l=%lld nu=%.3e jacobi_sweeps=%d\n", (long long)n,
                 (long long)l, nu, sweeps);
  P->nu = nu;
  return NYS_OK;
}

nys_status nys_op_apply(const nys_operator* A, double mu, const void* V, int64_t k, int64_t ldv,
                        void* Z, int64_t ldz, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  OpDesc op;
  NYS_TRY(check_op(A, op));
  NYS_ARG(V && Z && k >= 1 && ldv >= k && ldz >= k, "nys_op_apply: invalid vectors");
  NYS_ARG(std::isfinite(mu), "mu must be finite");
  NYS_ARG(prec >= NYS_PREC_FP64 && prec <= NYS_PREC_BF16X3_REFINE64, "unknown precision mode");
  const bool f32 = prec != NYS_PREC_FP64;
  hipStream_t s = S(stream);
  if (op.kind == NYS_OP_CALLBACK) {
    if (f32)
      return callback_apply<float>(op, static_cast<const float*>(V), k, ldv, nullptr, 1, mu, static_cast<float*>(Z),
                                   ldz, s);
    return callback_apply<double>(op, static_cast<const double*>(V), k, ldv, nullptr, 1, mu, static_cast<double*>(Z),
                                  ldz, s);
  }
  NYS_ARG(!f32 || op.kind == NYS_OP_RBF || (k == 1 && ldv == 1 && ldz == 1),
          "nys_op_apply: float32 products of X^T X / dense operators take one contiguous vector");
  NYS_ARG(!f32 || op.kind != NYS_OP_RBF || op.cols <= 32, "reduced-precision RBF products need d <= 32");
  Arena a(ws, ws_bytes);
  double* mu_dev = a.take<double>(1);
  const size_t se = op_scratch_elems(op, k);
  double* scr = a.take<double>(se);
  void* lowp_buf = (f32 && op.kind == NYS_OP_RBF) ? a.take<char>(rbf_lowp_bytes(op.n)) : nullptr;
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  const bool one = k == 1 && ldv == 1 && ldz == 1;
  // single-vector X^T X / dense products take mu by value; the others read it from the device
  if (!(one && op.kind != NYS_OP_RBF)) NYS_TRY(set_mu(mu_dev, &mu, 1, s));
  if (f32 && op.kind == NYS_OP_RBF) {
    RbfLowp L;
    NYS_TRY(rbf_lowp_prepare(op, lowp_buf, L, s));
    if (one)
      return rbf_lowp_mv(L, rbf_gram(prec), static_cast<const float*>(V), mu_dev, static_cast<float*>(Z),
                         reinterpret_cast<float*>(scr), 2 * se, s);
    return rbf_lowp_kv(L, rbf_gram(prec), static_cast<const float*>(V), ldv, k, mu_dev, k, static_cast<float*>(Z),
                       ldz, reinterpret_cast<float*>(scr), se, nullptr, s);
  }
  if (f32)
    return op_matvec<float>(op, static_cast<const float*>(V), (float)mu, static_cast<float*>(Z),
                            reinterpret_cast<float*>(scr), se, s);
  if (one && (op.kind == NYS_OP_XTX || op.kind == NYS_OP_DENSE))
    return op_matvec<double>(op, static_cast<const double*>(V), mu, static_cast<double*>(Z), scr, se, s);
  return op_apply_f64(op, static_cast<const double*>(V), k, ldv, mu_dev, k, static_cast<double*>(Z), ldz,
                      scr, se, s);
}

nys_status nys_precond_apply(const nys_precond* P, double mu, const double* R, int64_t k, int64_t ldr,
                             double* Z, int64_t ldz, void* ws, size_t ws_bytes, void* stream) {
  PrecDesc pd;
  NYS_TRY(check_prec(P, pd));
  NYS_ARG(R && Z && k >= 1 && k <= kMaxCols && ldr == k && ldz == k,
          "nys_precond_apply: R and Z must be contiguous n x k blocks, k <= 256");
  NYS_ARG(std::isfinite(mu) && mu >= 0.0, "mu must be finite and >= 0");
  Arena a(ws, ws_bytes);
  double* mu_dev = a.take<double>(1);
  const size_t pe = precond_part_elems(pd.n, pd.ell, k);
  double* part = a.take<double>(pe);
  double* Cs = a.take<double>(pd.ell * k);
  double* Ct = a.take<double>(pd.ell * k);
  unsigned* ctr = a.take<unsigned>(64);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = S(stream);
  NYS_TRY(set_mu(mu_dev, &mu, 1, s));
  NYS_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned) * 64, s));
  return precond_apply_standalone(pd, mu_dev, R, Z, k, part, pe, Cs, Ct, ctr, s);
}

nys_status nys_pcg_solve(const nys_operator* A, const nys_precond* P, const double* mu, int64_t nmu,
                         const double* B, int64_t nrhs, int64_t ldb, double* X, int64_t ldx,
                         const nys_solve_opts* o, nys_solve_info* info, void* ws, size_t ws_bytes,
                         void* stream) {
  OpDesc op;
  NYS_TRY(check_op(A, op));
  PrecDesc pd;
  NYS_TRY(check_prec(P, pd));
  NYS_ARG(B && X && nrhs >= 1 && ldb >= nrhs, "nys_pcg_solve: invalid B");
  const int64_t k = nmu * nrhs;
  NYS_ARG(k >= 1 && k <= kMaxCols, "nys_pcg_solve: nmu * nrhs must be in [1, 256]");
  NYS_ARG(ldx >= k, "nys_pcg_solve: ldx < nmu * nrhs");
  hipStream_t s = S(stream);
  NYS_TRY(check_solve_common(op, pd, mu, nmu, o, s));
  Arena a(ws, ws_bytes);
  SolveWs w;
  carve_solve(a, op, pd.ell, k, o->prec, w);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  return solve_impl(op, pd, mu, nmu, B, nrhs, ldb, X, ldx, o, info, w, s);
}

size_t nys_workspace_size_ragged(const nys_operator* ops, const nys_precond* Ps, int32_t nprob,
                                 int32_t prec) {
  if (!ops || !Ps || nprob < 1) return 0;
  std::vector<OpDesc> od(nprob);
  std::vector<PrecDesc> pd(nprob);
  size_t best = 0;
  bool valid = true;
  for (int32_t i = 0; i < nprob; ++i) {
    valid = valid && check_op(&ops[i], od[i]) == NYS_OK && check_prec(&Ps[i], pd[i]) == NYS_OK;
    const size_t b = nys_workspace_size(&ops[i], Ps[i].ell, 1, prec);
    best = b > best ? b : best;
  }
  if (valid && ragged_supported(od.data(), pd.data(), nprob)) {
    const size_t r = ragged_workspace(od.data(), pd.data(), nprob, prec);
    best = r > best ? r : best;
  }
  return best;
}

nys_status nys_pcg_solve_ragged(const nys_operator* ops, const nys_precond* Ps, const double* mu,
                                const double* const* B, double* const* X, int32_t nprob,
                                const nys_solve_opts* o, nys_solve_info* info, void* ws,
                                size_t ws_bytes, void* stream) {
  NYS_ARG(ops && Ps && mu && B && X && nprob >= 1, "nys_pcg_solve_ragged: NULL argument");
  NYS_ARG(o != nullptr, "nys_pcg_solve_ragged: options are NULL");
  hipStream_t s = S(stream);
  std::vector<OpDesc> od(nprob);
  std::vector<PrecDesc> pd(nprob);
  for (int32_t i = 0; i < nprob; ++i) {
    NYS_TRY(check_op(&ops[i], od[i]));
    NYS_TRY(check_prec(&Ps[i], pd[i]));
    NYS_ARG(B[i] != nullptr && X[i] != nullptr, "nys_pcg_solve_ragged: NULL vector of problem %d", i);
    NYS_TRY(check_solve_common(od[i], pd[i], &mu[i], 1, o, s));
  }
  // X^T X problems: one batched solve (every CG step of every problem in the same launches)
  if (ragged_supported(od.data(), pd.data(), nprob))
    return ragged_solve(od.data(), pd.data(), mu, B, X, nprob, o, info, ws, ws_bytes, s);
  // other operator mixes: one problem after the other
  nys_status worst = NYS_OK;
  int total = 0, refine = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    int it = 0, st = 0;
    double rr = 0.0;
    nys_solve_info inf{&it, &rr, &st, 0, 0};
    if (o->device_info) {  // the caller's device arrays, entry i
      inf.iters = info && info->iters ? info->iters + i : nullptr;
      inf.relres = info && info->relres ? info->relres + i : nullptr;
      inf.status = info && info->status ? info->status + i : nullptr;
    }
    const nys_status r = nys_pcg_solve(&ops[i], &Ps[i], &mu[i], 1, B[i], 1, 1, X[i], 1, o, &inf, ws,
                                       ws_bytes, stream);
    if (r < 0) return r;
    if (r != NYS_OK) worst = r;
    if (info && !o->device_info) {
      if (info->iters) info->iters[i] = it;
      if (info->relres) info->relres[i] = rr;
      if (info->status) info->status[i] = st;
    }
    total += inf.total_iters;
    refine += inf.refine_steps;
  }
  if (info) {
    info->total_iters = total;
    info->refine_steps = refine;
  }
  return worst;
}

nys_status nys_pcg_backward(const nys_operator* A, const nys_precond* P, double mu, const double* x,
                            const double* gx, double* gb, double* gmu, double* gsigma, double* gX,
                            const nys_solve_opts* o, nys_solve_info* info, void* ws, size_t ws_bytes,
                            void* stream) {
  OpDesc op;
  NYS_TRY(check_op(A, op));
  PrecDesc pd;
  NYS_TRY(check_prec(P, pd));
  NYS_ARG(x && gx && gb, "nys_pcg_backward: NULL vector");
  NYS_ARG(o != nullptr && o->device_info == 0, "nys_pcg_backward: the device-info form is not available here");
  hipStream_t s = S(stream);
  NYS_TRY(check_solve_common(op, pd, &mu, 1, o, s));
  const int64_t n = op.n;
  Arena a(ws, ws_bytes);
  SolveWs w;
  carve_solve(a, op, pd.ell, 1, o->prec, w);
  double* tmp = a.take<double>(n > op.rows ? n : op.rows);
  double* tmp2 = a.take<double>(op.rows);
  double* part = a.take<double>(1024);
  const size_t rscr_elems = (size_t)(4 * 256) * (size_t)n;
  double* rscr = a.take<double>(rscr_elems);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  // adjoint solve (A + mu I) lambda = gx with the same preconditioner, lambda in gb
  NYS_TRY(zero<double>(gb, n, s));
  const nys_status st = solve_impl(op, pd, &mu, 1, gx, 1, 1, gb, 1, o, info, w, s);
  if (st < 0) return st;
  std::vector<double> h(256);
  // dL/dmu = -lambda^T x
  if (gmu) {
    hipLaunchKernelGGL(dot_partial, dim3(256), dim3(256), 0, s, gb, x, n, part);
    NYS_CHECK_LAUNCH();
    NYS_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * 256, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
    double d = 0.0;
    for (int i = 0; i < 256; ++i) d += h[i];
    *gmu = -d;
  }
  if (gsigma) {
    if (op.kind == NYS_OP_RBF) {
      // -lambda^T (dK/dsigma) x
      NYS_TRY(rbf_rect_mv(op.data, n, op.ld, op.data, n, op.ld, (int)op.cols, op.dtype, op.sigma, 1, x,
                          tmp, rscr, rscr_elems, s));
      hipLaunchKernelGGL(dot_partial, dim3(256), dim3(256), 0, s, gb, tmp, n, part);
      NYS_CHECK_LAUNCH();
      NYS_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * 256, hipMemcpyDeviceToHost, s));
      NYS_HIP(hipStreamSynchronize(s));
      double d = 0.0;
      for (int i = 0; i < 256; ++i) d += h[i];
      *gsigma = -op.scale * d;
    } else {
      *gsigma = 0.0;
    }
  }
  if (gX) {
    NYS_ARG(op.kind == NYS_OP_XTX, "gX is defined for the X^T X operator only");
    NYS_ARG(op.w == nullptr, "gX is not formed for a weighted X^T X operator");
    const int64_t m = op.rows;
    // t1 = X x, t2 = X lambda;  gX = -scale (t1 lambda^T + t2 x^T)
    if (op.dtype == NYS_F64) {
      hipLaunchKernelGGL(gemv_rows<double>, dim3((unsigned)cdiv(m, 4)), dim3(256), 0, s,
                         static_cast<const double*>(op.data), m, n, op.ld, x, tmp);
      hipLaunchKernelGGL(gemv_rows<double>, dim3((unsigned)cdiv(m, 4)), dim3(256), 0, s,
                         static_cast<const double*>(op.data), m, n, op.ld, gb, tmp2);
    } else {
      hipLaunchKernelGGL(gemv_rows<float>, dim3((unsigned)cdiv(m, 4)), dim3(256), 0, s,
                         static_cast<const float*>(op.data), m, n, op.ld, x, tmp);
      hipLaunchKernelGGL(gemv_rows<float>, dim3((unsigned)cdiv(m, 4)), dim3(256), 0, s,
                         static_cast<const float*>(op.data), m, n, op.ld, gb, tmp2);
    }
    NYS_CHECK_LAUNCH();
    hipLaunchKernelGGL(outer2, dim3(nblk(m * n)), dim3(256), 0, s, m, n, op.scale, tmp, gb, tmp2, x, gX);
    NYS_CHECK_LAUNCH();
    NYS_HIP(hipStreamSynchronize(s));
  }
  return st;
}

nys_status nys_rbf_cross(const nys_operator* A, const void* Xv, int64_t nv, int64_t ldxv,
                         int32_t transpose, const double* v, double* out, const double* wvec,
                         double* dsig_out, void* ws, size_t ws_bytes, void* stream) {
  OpDesc op;
  NYS_TRY(check_op(A, op));
  NYS_ARG(op.kind == NYS_OP_RBF, "nys_rbf_cross needs an RBF operator");
  NYS_ARG(Xv && nv >= 1 && ldxv >= op.cols && v && out, "nys_rbf_cross: invalid arguments");
  const int64_t n = op.n;
  Arena a(ws, ws_bytes);
  const size_t se = (size_t)(4 * 256) * (size_t)(n > nv ? n : nv);
  double* scr = a.take<double>(se);
  double* part = a.take<double>(256);
  if (!ws || !a.ok()) {
    set_error("workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = S(stream);
  if (wvec || dsig_out) {
    NYS_ARG(wvec != nullptr && dsig_out != nullptr && !transpose,
            "nys_rbf_cross: the dK/dsigma form needs wvec, dsig_out and transpose = 0");
    // out = (dK(Xv, X)/dsigma) wvec (nv), then v^T out
    NYS_TRY(rbf_rect_mv(Xv, nv, ldxv, op.data, n, op.ld, (int)op.cols, op.dtype, op.sigma, 1, wvec, out, scr,
                        se, s));
    hipLaunchKernelGGL(dot_partial, dim3(256), dim3(256), 0, s, v, out, nv, part);
    NYS_CHECK_LAUNCH();
    std::vector<double> h(256);
    NYS_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * 256, hipMemcpyDeviceToHost, s));
    NYS_HIP(hipStreamSynchronize(s));
    double d = 0.0;
    for (int i = 0; i < 256; ++i) d += h[i];
    *dsig_out = d;
    return NYS_OK;
  }
  if (!transpose)
    return rbf_rect_mv(Xv, nv, ldxv, op.data, n, op.ld, (int)op.cols, op.dtype, op.sigma, 0, v, out, scr, se, s);
  return rbf_rect_mv(op.data, n, op.ld, Xv, nv, ldxv, (int)op.cols, op.dtype, op.sigma, 0, v, out, scr, se, s);
}

nys_status nys_pcg_solve_noalloc(const nys_operator* A, const nys_precond* P, const double* mu, int64_t nmu,
                                 const double* B, int64_t nrhs, int64_t ldb, double* X, int64_t ldx,
                                 const nys_solve_opts* o, nys_solve_info* info, void* stream) {
  NYS_ARG(o != nullptr && o->device_info == 1,
          "nys_pcg_solve_noalloc: only the device-info form (opts.device_info = 1) is available");
  OpDesc op;
  NYS_TRY(check_op(A, op));
  PrecDesc pd;
  NYS_TRY(check_prec(P, pd));
  NYS_ARG(B && X && nrhs >= 1 && ldb >= nrhs, "nys_pcg_solve_noalloc: invalid B");
  const int64_t k = nmu * nrhs;
  NYS_ARG(k >= 1 && k <= kMaxCols, "nys_pcg_solve_noalloc: nmu * nrhs must be in [1, 256]");
  NYS_ARG(ldx >= k, "nys_pcg_solve_noalloc: ldx < nmu * nrhs");
  hipStream_t s = S(stream);
  NYS_TRY(check_solve_common(op, pd, mu, nmu, o, s));
  {
    Arena probe(nullptr, 0);
    SolveWs w;
    carve_solve(probe, op, pd.ell, k, o->prec, w);
    if (probe.off > kStaticScratchBytes) {
      set_error("nys_pcg_solve_noalloc: this solve needs %zu bytes of scratch; the static scratch holds %zu",
                probe.off, kStaticScratchBytes);
      return NYS_ERR_WORKSPACE;
    }
  }
  void* base = nullptr;
  NYS_TRY(static_scratch(&base));
  Arena a(base, kStaticScratchBytes);
  SolveWs w;
  carve_solve(a, op, pd.ell, k, o->prec, w);
  return solve_impl(op, pd, mu, nmu, B, nrhs, ldb, X, ldx, o, info, w, s);
}

size_t nys_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

// ---- autotuner of the RBF block-product tile shapes

namespace {
nys_status autotune_op(const nys_operator* A, int32_t prec, OpDesc& op, int& mode) {
  NYS_TRY(check_op(A, op));
  NYS_ARG(op.kind == NYS_OP_RBF, "autotune: the tuned products are the reduced-precision RBF block products");
  NYS_ARG(op.cols <= 32, "autotune: reduced-precision RBF products need d <= 32");
  NYS_ARG(prec == NYS_PREC_FP32 || prec == NYS_PREC_FP32_REFINE64 || prec == NYS_PREC_BF16X3_REFINE64,
          "autotune: prec must be a reduced-precision mode");
  mode = rbf_gram(prec);
  return NYS_OK;
}
}  // namespace

size_t nys_workspace_size_autotune(const nys_operator* A, int64_t kmax) {
  OpDesc op;
  int mode = 0;
  if (kmax < 1 || autotune_op(A, NYS_PREC_FP32, op, mode) != NYS_OK) return 0;
  Arena a(nullptr, 0);
  (void)a.take<char>(rbf_lowp_bytes(op.n));
  (void)a.take<float>(op.n * kmax);
  (void)a.take<float>(op.n * kmax);
  (void)a.take<float>(rbf_lowp_kv_scratch(op.n, kmax));
  return a.off + 256;
}

nys_status nys_autotune(const nys_operator* A, int32_t prec, const int64_t* ks, int32_t nks, void* ws,
                        size_t ws_bytes, void* stream) {
  OpDesc op;
  int mode = 0;
  NYS_TRY(autotune_op(A, prec, op, mode));
  NYS_ARG(ks != nullptr && nks >= 1 && nks <= 64, "autotune: 1 <= nks <= 64 column counts");
  int64_t kmax = 0;
  for (int i = 0; i < nks; ++i) {
    NYS_ARG(ks[i] >= 2 && ks[i] <= 4096, "autotune: column counts must lie in [2, 4096] (ks[%d] = %lld)", i,
            (long long)ks[i]);
    kmax = ks[i] > kmax ? ks[i] : kmax;
  }
  Arena a(ws, ws_bytes);
  char* lp = a.take<char>(rbf_lowp_bytes(op.n));
  float* P = a.take<float>(op.n * kmax);
  float* V = a.take<float>(op.n * kmax);
  const size_t se = rbf_lowp_kv_scratch(op.n, kmax);
  float* scr = a.take<float>(se);
  if (!ws || !a.ok()) {
    set_error("autotune: workspace too small: need %zu bytes", a.off);
    return NYS_ERR_WORKSPACE;
  }
  hipStream_t s = S(stream);
  RbfLowp L{};
  NYS_TRY(rbf_lowp_prepare(op, lp, L, s));
  NYS_TRY(rbf_lowp_autotune(L, mode, ks, nks, P, V, scr, se, s));
  kv_tune_env_save();
  return NYS_OK;
}

nys_status nys_autotune_query(const nys_operator* A, int32_t prec, int64_t k, int32_t* choice, int32_t* tuned) {
  OpDesc op;
  int mode = 0;
  NYS_TRY(autotune_op(A, prec, op, mode));
  NYS_ARG(k >= 1 && choice != nullptr, "autotune query: k >= 1 and a 4-entry choice array");
  RbfLowp L{};
  L.n = op.n;
  L.d = (int)op.cols;
  bool t = false;
  const KvChoice c = kv_choice(L, k, mode, &t);
  choice[0] = c.reg;
  choice[1] = c.cf;
  choice[2] = c.bpc;
  choice[3] = c.fr;
  if (tuned) *tuned = t ? 1 : 0;
  return NYS_OK;
}

int64_t nys_autotune_entries(void) { return kv_tune_entries(); }

nys_status nys_autotune_clear(void) {
  kv_tune_clear();
  return NYS_OK;
}

nys_status nys_autotune_load(const char* path) {
  NYS_ARG(path != nullptr, "autotune load: NULL path");
  return kv_tune_load(path);
}

nys_status nys_autotune_save(const char* path) {
  NYS_ARG(path != nullptr, "autotune save: NULL path");
  return kv_tune_save(path);
}

}  // extern "C"
