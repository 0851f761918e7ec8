// Internal declarations of the QTT library: context, device buffers,
// kernel launchers.  Host code throws qtt::Error; the C entry points in
// qtt_api.hip turn it into return codes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>
#include <map>
#include <memory>

#include "../../include/qtt.h"

namespace qtt {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPC(x) ::qtt::hip_check((x), #x)

// ---------------------------------------------------------------- buffers
// A growing device buffer owned by the context.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct Ctx;

// ---------------------------------------------------------------- MPS view
struct Mps {
  int n = 0;
  int bond[QTT_MAX_SITES + 1] = {0};
  double *data = nullptr;
  int64_t capacity = 0;
  int64_t off(int k) const {
    int64_t o = 0;
    for (int j = 0; j < k; ++j) o += (int64_t)bond[j] * 4 * bond[j + 1];
    return o;
  }
  int64_t size() const { return off(n); }
  double *core(int k) const { return data + off(k); }
  int64_t core_size(int k) const { return (int64_t)bond[k] * 4 * bond[k + 1]; }
};

Mps from_c(const qtt_mps &m);
void to_c(const Mps &m, qtt_mps *out);

// MPO held by the context: forward cores [a][w][w'][b] and, for the
// contraction kernels, the permuted cores [a][w'][w][b] and reversed
// permuted cores [b][w'][w][a] (site order unchanged).
struct Mpo {
  int n = 0;
  int bond[QTT_MAX_SITES + 1] = {0};
  double *fwd = nullptr;   // [a][w][w'][b]
  double *perm = nullptr;  // [a][w'][w][b]
  double *rperm = nullptr; // [b][w'][w][a]
  int64_t off(int k) const {
    int64_t o = 0;
    for (int j = 0; j < k; ++j) o += (int64_t)bond[j] * 16 * bond[j + 1];
    return o;
  }
};

// ---------------------------------------------------------------- kernel timing
struct KernelTimer {
  bool on = false;
  int every = 1;
  int64_t launches[2] = {0, 0};
  int64_t timed[2] = {0, 0};
  double timed_ms[2] = {0.0, 0.0};
  double *flop_ctr = nullptr;  // device, 2 doubles
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
  std::vector<hipEvent_t> pool;
};

// ---------------------------------------------------------------- context
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, DevBuf> bufs;
  std::vector<void *> owned;          // allocations freed at destroy
  std::vector<size_t> owned_sizes;
  double *pinned = nullptr;           // host pinned scratch (4096 doubles)
  bool timing = false;                // host-timed phase statistics (QTT_TIMING=1)
  // MPO cache keyed by (n, kind, dx bits)
  std::map<std::string, std::shared_ptr<Mpo>> mpos;

  KernelTimer kt;
  hipEvent_t take_event();
  void resolve_events();
  // caller buffers registered by the entry point (device address ranges)
  std::vector<std::pair<uintptr_t, size_t>> user_ranges;

  double *buf(const std::string &name, int64_t ndouble);  // grows, contents not kept
  void *raw(const std::string &name, size_t bytes);
  void sync();
  double *alloc_owned(int64_t ndouble);
  void register_user(const void *p, size_t bytes);
  // every kernel launch checks that the element range [lo, hi] of each
  // operand lies inside one known allocation; a violation is an error, not
  // a launch
  void check_range(const void *p, int64_t lo_elem, int64_t hi_elem, size_t esize,
                   const char *what) const;
  ~Ctx();
};

// element offsets touched by a strided access with the given extents
inline void span(int64_t &lo, int64_t &hi, int64_t ext, int64_t stride) {
  if (ext <= 0) return;
  const int64_t d = (ext - 1) * stride;
  if (d > 0) hi += d;
  else lo += d;
}

// ---------------------------------------------------------------- GEMM
// C[b1,b2](m,n) = alpha * sum_k A[b1,b2](m,k) B[b1,b2](k,n) + beta * C
// with arbitrary element strides.  skip: optional device flag; when it is
// non-zero the kernel returns immediately (used to stop converged CG).
// alpha_dev: optional device scalar multiplying alpha.
struct Gemm {
  int M = 0, N = 0, K = 0, B1 = 1, B2 = 1;
  const double *A = nullptr;
  int64_t sAm = 0, sAk = 0, sAb1 = 0, sAb2 = 0;
  const double *B = nullptr;
  int64_t sBk = 0, sBn = 0, sBb1 = 0, sBb2 = 0;
  double *C = nullptr;
  int64_t sCm = 0, sCn = 0, sCb1 = 0, sCb2 = 0;
  double alpha = 1.0, beta = 0.0;
  const int *skip = nullptr;
};
void gemm(Ctx &c, const Gemm &g);
// float32-MFMA variant with float64 inputs/outputs (mixed precision mode)
void gemm_f32(Ctx &c, const Gemm &g);

// ---------------------------------------------------------------- small kernels
void fill(Ctx &c, double *p, int64_t n, double v);
void scale_copy(Ctx &c, double *dst, const double *src, int64_t n, double s);
void axpy_into(Ctx &c, double *y, const double *x, int64_t n, double s);
// dst[i0][i1][i2] = s * src[i0*s0 + i1*s1 + i2*s2], dst packed (d0 x d1 x d2)
void permute3(Ctx &c, double *dst, const double *src, int d0, int d1, int d2, int64_t s0,
              int64_t s1, int64_t s2, double s = 1.0);
// block copy of a core into a larger core: dst[(ol+a)][w][(or+b)] = s * src[a][w][b]
void place_block(Ctx &c, double *dst, int dl, int dr, const double *src, int l, int r, int ol,
                 int orr, double s);
void hadamard_core(Ctx &c, double *y, const double *a, int la, int ra, const double *b, int lb,
                   int rb);
void mpo_core(Ctx &c, double *y, const double *W, int wl, int wr, const double *x, int l, int r);
// one MPO layer of a network chain (sparse, HBM-streaming):
// Tout[p][w_out][m'][q] = sum W[m][w_in][w_out][m'] T[p][m][w_in][q]
void mpo_layer(Ctx &c, const double *T, double *Tout, const double *W, int64_t pre, int mi, int mo,
               int64_t post, const int *skip);
void morton_gather(Ctx &c, double *grid, const double *vec, int n);   // vec (Morton) -> grid
void morton_scatter(Ctx &c, double *vec, const double *grid, int n);  // grid -> vec (Morton)
void dot(Ctx &c, const double *x, const double *y, int64_t n, double *out_dev);
int any_nonfinite(Ctx &c, const double *x, int64_t n);

// ---------------------------------------------------------------- dense linear algebra
// Matrix view: element (i, j) at p[i*rs + j*cs].
struct MatView {
  double *p;
  int rows, cols;
  int64_t rs, cs;
};
struct ConstMatView {
  const double *p;
  int rows, cols;
  int64_t rs, cs;
};
// Batched Householder QR of m x n matrices (reduced): Q (m x k), R (k x n),
// k = min(m, n), diag(R) >= 0.  Outputs may alias nothing.
void qr_batch(Ctx &c, int count, const ConstMatView *A, const MatView *Q, const MatView *R);
// Batched one-sided Jacobi SVD of m x n (m >= n) matrices: A = U diag(S) V^T,
// singular values descending.  U is m x n (zero columns for zero sigma),
// V is n x n, S has n entries (device).
void svd_batch(Ctx &c, int count, const ConstMatView *A, const MatView *U, double *const *S,
               const MatView *V);

// ---------------------------------------------------------------- MPS ops (host orchestration)
void mps_add(Ctx &c, int k, const double *coef, const Mps *x, Mps &y);
// TT-rounding of several MPS in place; returns discarded weight per MPS.
void mps_truncate(Ctx &c, std::vector<Mps *> ys, int chi, double rtol, double *disc);
void mps_apply_mpo(Ctx &c, const Mpo &W, const Mps &x, Mps &y);
void mps_hadamard(Ctx &c, const Mps &a, const Mps &b, Mps &y);
double mps_inner(Ctx &c, const Mps &x, const Mps &y);
void mps_to_dense(Ctx &c, const Mps &x, double *grid);
void mps_from_dense(Ctx &c, const double *grid, int n, int chi, double rtol, Mps &out);
void mps_copy(Ctx &c, const Mps &src, Mps &dst);
void mps_right_canonicalize(Ctx &c, std::vector<Mps *> xs);

// MPO construction (host) and upload
std::shared_ptr<Mpo> get_mpo(Ctx &c, int n, const std::string &kind, double dx, int lap_mode);
void build_derivative_host(int n, int axis, int order, double dx, std::vector<double> &cores,
                           int *bond);

// ---------------------------------------------------------------- sweep / RK4
void project(Ctx &c, const Mps a[2], const Mps b[2], double h, const qtt_params &p, Mps v[2],
             qtt_stats *st, int stage);
void rk4_step(Ctx &c, Mps u[2], const qtt_params &p, qtt_stats *st);

}  // namespace qtt
