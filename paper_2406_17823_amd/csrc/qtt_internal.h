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
// Compressed-column form of a site core viewed as B[k = (m_in, w_in)][o = (w_out, m_out)]:
// column o holds its non-zeros (k, value); offsets per site on the host.
struct MpoCsc {
  int *colptr = nullptr;   // per site: 4*m_out + 1 entries
  int *rowidx = nullptr;
  double *val = nullptr;
  std::vector<int64_t> cp_off, nz_off;  // per-site offsets into colptr / rowidx,val
};

struct Mpo {
  int n = 0;
  int bond[QTT_MAX_SITES + 1] = {0};
  double *fwd = nullptr;   // [a][w][w'][b]
  double *perm = nullptr;  // [a][w'][w][b]
  double *rperm = nullptr; // [b][w'][w][a]
  MpoCsc csc[2];           // 0: perm, 1: rperm
  int64_t off(int k) const {
    int64_t o = 0;
    for (int j = 0; j < k; ++j) o += (int64_t)bond[j] * 16 * bond[j + 1];
    return o;
  }
};

// ---------------------------------------------------------------- kernel timing
// GEMM kernel instantiations told apart by the timer (QTT_KERNEL_GEMM_*):
// 0 float64 64x64 tiles, 1 float32 64x64, 2 float64 128x128, 3 float32 128x128
constexpr int KT_KINDS = 4;
struct KernelTimer {
  bool on = false;
  int every = 1;
  int64_t launches[KT_KINDS] = {0, 0, 0, 0};
  int64_t timed[KT_KINDS] = {0, 0, 0, 0};
  double timed_ms[KT_KINDS] = {0.0, 0.0, 0.0, 0.0};
  double *flop_ctr = nullptr;  // device, KT_KINDS doubles
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[KT_KINDS];
  std::vector<hipEvent_t> pool;
};

// captured graph of a chunk of CG iterations
struct CgGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> key;
  int hits = 0;  // lookups in a row that found the same key
  int64_t launches[KT_KINDS] = {0, 0, 0, 0};  // GEMM launches per replay, by timer kind
};

// ---------------------------------------------------------------- learned preconditioner
// Shared-weight perceptron applied to every (alpha, beta) position of a centre
// tensor: PC_IN features -> PC_W -> PC_W -> PC_OUT factor entries of a 4 x 4
// lower-triangular L; the block of the preconditioner is L L^T.
constexpr int PC_IN = 16, PC_W = 256, PC_OUT = 10;
struct PrecondNet {
  bool ready = false;
  double *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // device, nparam each
  int64_t off[6] = {0, 0, 0, 0, 0, 0};  // W1 b1 W2 b2 W3 b3 (row-major W: out x in)
  int64_t nparam = 0;
  int64_t steps = 0;          // Adam steps taken
  int train_per_solve = 0;    // Adam steps per local system while training
  double lr = 1e-3;
  uint64_t seed = 0x5eed;
  uint64_t probe_ctr = 0;
  double last_loss = -1.0;    // probe loss of the latest training step
  double first_loss = -1.0;   // probe loss of the first training step
  double *loss_dev = nullptr; // device accumulator (1 double)
  // activations of the latest forward pass with keep = true (act_rows rows)
  double *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr;
  double *Lf = nullptr, *dY = nullptr;
  int64_t act_rows = 0;
  int64_t param_count() const { return (int64_t)PC_W * PC_IN + PC_W + (int64_t)PC_W * PC_W + PC_W +
                                       (int64_t)PC_OUT * PC_W + PC_OUT; }
};

// ---------------------------------------------------------------- context
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;            // stream created by the context
  std::string err;
  std::map<std::string, DevBuf> bufs;
  std::vector<void *> owned;          // allocations freed at destroy
  std::vector<size_t> owned_sizes;
  double *pinned = nullptr;           // host pinned scratch (4096 doubles)
  bool timing = false;                // host-timed phase statistics (QTT_TIMING=1)
  // MPO cache keyed by (n, kind, dx bits)
  std::map<std::string, std::shared_ptr<Mpo>> mpos;

  KernelTimer kt;
  PrecondNet pc;
  bool use_graphs = true;             // QTT_GRAPHS=0 disables CG graph capture
  bool autotune = false;              // QTT_AUTOTUNE=1 tunes GEMM tile sizes per shape
  std::map<std::string, int> gemm_tune;  // tuned tile size per GEMM shape
  bool capturing = false;             // a stream capture is open
  int64_t cap_launches[KT_KINDS] = {0, 0, 0, 0};
  std::map<std::string, CgGraph> cg_graphs;
  // iterations of the latest CG solve per (site, direction, preconditioning)
  std::map<int, int> cg_hist;
  // per-shape GEMM timing (QTT_GEMM_STATS=1), printed when the context ends
  bool shape_stats = false;
  // outer sweeps of a Jacobi SVD before it stops with rotations still pending
  // (QTT_SVD_MAX_SWEEPS, default 40); hitting the cap sets the warning below
  int svd_max_sweeps = 40;
  // warning raised below the entry point (QTT_W_SVD_MAXIT); cleared at the
  // start of every call and returned when the call otherwise succeeds
  int warn = 0;
  struct ShapeRec {
    int64_t calls = 0;
    double ms = 0.0, flops = 0.0;
  };
  std::map<std::string, ShapeRec> shapes;
  std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> shape_pending;
  std::vector<double> shape_flops_pending;
  void resolve_shapes();
  hipEvent_t take_event();
  void resolve_events();
  // caller buffers registered by the entry point (device address ranges)
  std::vector<std::pair<uintptr_t, size_t>> user_ranges;
  void clear_user() {
    user_ranges.clear();
    ranges_dirty = true;
  }
  // every known allocation as [begin, end), sorted by begin (rebuilt after an
  // allocation or registration), for the range checks of each launch
  mutable std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
  mutable bool ranges_dirty = true;

  double *buf(const std::string &name, int64_t ndouble);  // grows, contents not kept
  void *raw(const std::string &name, size_t bytes);
  void sync();
  double *alloc_owned(int64_t ndouble);
  void register_user(const void *p, size_t bytes);
  // worker contexts (own stream and workspace) for concurrent independent flows
  std::vector<std::unique_ptr<Ctx>> workers;
  // every kernel launch checks that the element range [lo, hi] of each
  // operand lies inside one known allocation; a violation is an error, not
  // a launch
  void check_range(const void *p, int64_t lo_elem, int64_t hi_elem, size_t esize,
                   const char *what) const;
  ~Ctx();
};

// a worker context on the parent's device: own non-blocking stream (default
// priority), own pinned scratch and workspace, no graph capture
std::unique_ptr<Ctx> make_worker(const Ctx &parent);

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
struct CGState;
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
  // A, B or C held as float32 (the pointer is reinterpreted, strides count
  // float32 elements): the convection networks of the mixed mode keep their
  // environments and chain intermediates in float32 storage
  bool a32 = false, b32 = false, c32 = false;
  // CG operand (float64 B only): B is read as B - alpha (Bw + beta Bs) with
  // alpha, beta of the CG state cgst (see GemmCg)
  const double *Bw = nullptr, *Bs = nullptr;
  const CGState *cgst = nullptr;
};
constexpr int GEMM_GROUP = 4;
void gemm(Ctx &c, const Gemm &g);
// up to GEMM_GROUP problems in one launch; problem i contributes to output
// group group[i] (the problems of a group share C and beta and are summed,
// each scaled by its own alpha); X[group] (nullptr = C) is the beta input.
// With dot, the reduction kernel also forms sum_groups C . Y[group] (Y laid
// out like C, float64) into the device scalar out, deterministically (block
// partials in part, summed in block order by the last block to arrive at the
// counter ctr, which must be 0 and is left 0); every output must go through
// the reduction (summed or split-K).
struct GemmDot {
  const double *Y[GEMM_GROUP];
  double *out;
  unsigned *ctr;
  double *part;
  int nparts;
};
// CG step fused into the matvec (single-reduction CG, the local solves of
// the sweep), one iteration per matvec: with alpha and beta from the state
// (gamma = r.r, delta = w.r with w = A r, gamma_prev, alpha_prev; first
// step: beta = 0, alpha = gamma / delta) the first GEMM of the matvec reads
// its B operand as the next residual r - alpha (w + beta s) (Gemm::Bw and
// Bs point at w and s laid out like B), and the reduction of the last GEMM
// (q its output before the beta term, laid out like the CG vectors from
// position off[group]; C is not written) takes every element through
//   s = w + beta s, p = r + beta p, x += alpha p, r -= alpha s,
//   w = q + beta_C r   (the new A r: the beta term uses the new r),
// while the last block to arrive forms the new gamma and delta (block
// partials in part, 2 per block, summed in block order), counts the
// iteration and sets done on convergence, NaN or the iteration limit.
// Every output must go through the reduction; the state counter must be 0
// and is left 0.
struct GemmCg {
  CGState *st;
  double *x, *r, *w, *p, *s;
  int64_t n;
  int64_t off[GEMM_GROUP];
  double *part;
  int nparts;
};
// prec: QTT_PREC_F64, QTT_PREC_F32 (float32 MFMAs) or QTT_PREC_BF16X3 (split
// bfloat16 MFMAs) for every problem of the launch
void gemm_grouped(Ctx &c, int np, const Gemm *q, int ngroups, const int *group,
                  const double *const *X, const int *skip, int prec,
                  const GemmDot *dot = nullptr, const GemmCg *cg = nullptr);
// float32-MFMA variant with float64 inputs/outputs (mixed precision mode)
void gemm_f32(Ctx &c, const Gemm &g);
// bfloat16-MFMA variant (float32 accumulation) with float64 inputs/outputs
void gemm_bf16(Ctx &c, const Gemm &g);
// compensated split-bfloat16 variant: hi*hi + hi*lo + lo*hi on bfloat16 MFMA
// (about 16 significant bits per operand), float64 inputs/outputs
void gemm_bf16x3(Ctx &c, const Gemm &g);

// ---------------------------------------------------------------- small kernels
void fill(Ctx &c, double *p, int64_t n, double v);
// dst[k][0:n[k]) = src[k][0:n[k]) for up to four non-overlapping pairs, one launch
void copy_pairs(Ctx &c, int np, double *const *dst, const double *const *src, const int64_t *n);
void fill_f32(Ctx &c, float *p, int64_t n, float v);
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
// f32: T and Tout are float32 arrays (sums in float64)
void mpo_layer(Ctx &c, const double *T, double *Tout, const Mpo &W, int site, bool rev,
               int64_t pre, int mi, int mo, int64_t post, const int *skip, bool f32 = false);
struct MpoJob {
  const double *T;
  double *Tout;
  const Mpo *W;
  int site;
  bool rev;
  int64_t pre, post;
  int mi, mo;
};
// several MPO layers in one launch (at most 4)
// f32: every job's tensors are float32 (the pointers are reinterpreted)
void mpo_layer_grouped(Ctx &c, int nj, const MpoJob *jobs, const int *skip, bool f32 = false);
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
// k = min(m, n), diag(R) >= 0.  Outputs may alias nothing.  A view with a
// null pointer in Q asks for R only (the explicit Q is then not formed).
void qr_batch(Ctx &c, int count, const ConstMatView *A, const MatView *Q, const MatView *R);
// Batched one-sided Jacobi SVD of m x n (m >= n) matrices: A = U diag(S) V^T,
// singular values descending.  U is m x n, V is n x n, S has n entries
// (device).  A view with a null pointer in U asks for S and V only, one with
// a null pointer in V for U and S only.
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
// spectra (optional): the squared singular values of every cut k = 1..n-1
// as the sequential decomposition meets them (before that cut's truncation)
void mps_from_dense(Ctx &c, const double *grid, int n, int chi, double rtol, Mps &out,
                    std::vector<std::vector<double>> *spectra = nullptr);
// chi_l(eps) of every bipartition l = 1..n-1 of a dense grid (counts, host)
void schmidt_counts(Ctx &c, const double *grid, int n, double eps, int cap, int32_t *counts);
// dense DNS reference, fidelity and TKE spectrum (k_dns.hip)
void dns_rhs(Ctx &c, const double *u1, const double *u2, double *f1, double *f2, int n, double re);
void dns_project(Ctx &c, double *u1, double *u2, int n);
void dns_step(Ctx &c, double *u1, double *u2, int n, double re, double dt, int order, int steps);
int tke_shells(int n);
void dns_tke(Ctx &c, const double *u1, const double *u2, const double *m1, const double *m2, int n,
             double *E_dev);
void fidelity(Ctx &c, const double *a, const double *b, int64_t len, double *out_dev3);
void mps_copy(Ctx &c, const Mps &src, Mps &dst);
void mps_right_canonicalize(Ctx &c, std::vector<Mps *> xs);

// MPO construction (host) and upload
std::shared_ptr<Mpo> get_mpo(Ctx &c, int n, const std::string &kind, double dx, int lap_mode);
void build_derivative_host(int n, int axis, int order, double dx, std::vector<double> &cores,
                           int *bond);

// ---------------------------------------------------------------- sweep / RK4
// What the four stages of one RK4 step share: the stages start from the same
// guess a = u/4, so its right-canonical form and the initial right
// environments of the networks that do not involve b (overlap and penalty
// pairs) are computed by the first stage and copied by the others.
struct StageCache {
  bool valid = false;
  int bond[2][QTT_MAX_SITES + 1];
};
void project(Ctx &c, const Mps a[2], const Mps b[2], double h, const qtt_params &p, Mps v[2],
             qtt_stats *st, int stage, StageCache *cache = nullptr);
void rk4_step(Ctx &c, Mps u[2], const qtt_params &p, qtt_stats *st);
// order 1 (explicit Euler), 2 (midpoint) or 4 (rk4_step)
void rk_step(Ctx &c, Mps u[2], const qtt_params &p, int order, qtt_stats *st);

// ---------------------------------------------------------------- learned preconditioner
void pc_init(Ctx &c);                   // allocate and draw the weights once
void pc_reset(Ctx &c, uint64_t seed);   // (re)draw the weights from seed, clear Adam
// features X (npos x PC_IN) and exact diagonal blocks Bblk (npos x 16) of the
// local matrix for one component, from its own penalty pair's environments
void pc_features(Ctx &c, const double *Lenv, const double *Renv, const Mpo &Wii, int d, int la,
                 int ra, double mu_h2, double pen_scale, int n, int comp, double *X,
                 double *Bblk);
// network forward: M blocks (npos x 16); keep = store activations for training
void pc_forward(Ctx &c, const double *X, int64_t npos, double *M, bool keep);
void pc_block_inverse(Ctx &c, const double *Bblk, double *M, int64_t npos);
void pc_apply(Ctx &c, const double *M, const double *r, double *z, int la, int ra,
              const int *skip);
void pc_probe(Ctx &c, double *z, int64_t n, uint64_t seed);
// loss and output gradient for one component's positions (after pc_forward
// with keep = true); rows [row0, row0 + la*ra) of the stored activations
void pc_loss_grad(Ctx &c, const double *M, int64_t row0, const double *z, const double *Az,
                  int la, int ra, const double *zz);
// backward through the network from the stored output gradient, then Adam
void pc_backward_adam(Ctx &c, const double *X, int64_t npos);
// gradient of sum(dY * Y) for given inputs (device pointers): Y and grad out
void pc_net_grad(Ctx &c, const double *X, int64_t npos, const double *dY, double *Y,
                 double *grad);

}  // namespace qtt
