/*
 * qtt.h -- C ABI of the MI355X (gfx950) quantics-tensor-train Navier-Stokes
 * library.
 *
 * What it computes (arXiv 2406.17823, "Quantum-Inspired Fluid Simulation of
 * 2D Turbulence with GPU Acceleration"): the velocity components u_1, u_2 of
 * 2D incompressible flow on a periodic 2^n x 2^n grid are each held as a
 * matrix product state over the quantics index omega_k = 2*bit_k(x1) +
 * bit_k(x2) (Sec. II.B, bit 0 = most significant, site 0 = coarsest scale).
 * One time step is RK4 written as four Euler minimisations of the penalty
 * cost Theta (App. B, Eq. Theta, Table RK4, Eqs. U1-U4), each minimised by
 * a one-site variational sweep with conjugate-gradient local solves
 * (Sec. II.C, App. B).
 *
 * Memory and ownership
 *   All tensors are caller-owned device memory on the context's device,
 *   float64.  The library allocates only its own workspace, inside the
 *   context, and frees it in qtt_ctx_destroy.  Output bond dimensions are
 *   computed by the library; a caller buffer that is too small yields
 *   QTT_E_CAPACITY and the required number of doubles in qtt_last_error().
 *
 * Streams
 *   Every call is enqueued on the stream given to qtt_ctx_create (NULL: a
 *   stream owned by the context, which waits for the null stream at the
 *   start of every call) and returns after that stream has finished the
 *   call's work, so host-side results (discarded weights, statistics, bonds)
 *   and device outputs are valid on return.  Inner CG iterations are
 *   replayed from captured HIP graphs (QTT_GRAPHS=0 disables this).
 *
 * Environment (read when a context is created)
 *   QTT_GRAPHS=0    no graph capture of CG iterations
 *   QTT_AUTOTUNE=1  time both GEMM tile sizes on the first use of each
 *                   shape and keep the faster (results are unchanged)
 *   QTT_TIMING=1    host-timed phase statistics in qtt_stats.phase_ms
 *   QTT_VERBOSE=1   per-call diagnostics on stderr
 *   QTT_SVD_MAX_SWEEPS=k  outer-sweep cap of the Jacobi SVDs (default 40)
 *
 * Errors
 *   0 = success, > 0 = warning (result valid), < 0 = error (outputs
 *   undefined).  No C++ exception crosses this interface.  One context per
 *   host thread; a context is not thread-safe.
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QTT_MAX_SITES 16

enum {
  QTT_OK = 0,
  QTT_W_CG_MAXIT = 1,          /* a local CG solve stopped at cg_maxit          */
  QTT_W_SWEEP_MAXIT = 2,       /* the sweep stopped at max_sweeps (sweep_rtol>0) */
  QTT_W_PRECOND_FALLBACK = 3,  /* the learned preconditioner was rejected        */
  QTT_W_SVD_MAXIT = 4,         /* a Jacobi SVD of a truncation stopped at its
                                  sweep cap (QTT_SVD_MAX_SWEEPS, default 40) with
                                  rotations pending; its factors were used      */
  QTT_E_ARG = -1,
  QTT_E_SHAPE = -2,
  QTT_E_CAPACITY = -3,
  QTT_E_HIP = -4,
  QTT_E_NAN = -5,
  QTT_E_UNSUPPORTED = -6
};

/* contraction precision of the 8 convection networks, the only ones whose
 * contributions are scaled by the stage step h (the overlap, diffusion and
 * penalty networks, the CG, the QR and the SVD always stay float64):
 * float64 MFMA, float32 MFMA, or compensated split bfloat16 MFMA (each
 * operand as a sum of two bfloat16, three products) */
enum { QTT_PREC_F64 = 0, QTT_PREC_F32 = 1, QTT_PREC_BF16X3 = 2 };

/* preconditioner of the local CG solves */
enum { QTT_PC_NONE = 0, QTT_PC_BLOCK_JACOBI = 1, QTT_PC_LEARNED = 2 };

typedef struct qtt_ctx qtt_ctx;

/* One MPS (one velocity component).  Core k occupies
 * bond[k] * 4 * bond[k+1] doubles, row-major [bond[k]][4][bond[k+1]], and
 * the cores are packed in site order from data[0].  bond[0] = bond[n] = 1. */
typedef struct {
  int32_t n;                        /* sites, 1 <= n <= QTT_MAX_SITES     */
  int32_t bond[QTT_MAX_SITES + 1];  /* bond dimensions                    */
  int64_t capacity;                 /* doubles available at data          */
  double *data;                     /* device pointer                     */
} qtt_mps;

/* One MPO.  Core k is row-major [bond[k]][4][4][bond[k+1]] (output physical
 * index first, then the index contracted with the MPS), packed like qtt_mps. */
typedef struct {
  int32_t n;
  int32_t bond[QTT_MAX_SITES + 1];
  int64_t capacity;
  double *data;                     /* device pointer */
} qtt_mpo;

typedef struct {
  double re;          /* Reynolds number                                      */
  double dt;          /* time step                                            */
  double mu;          /* penalty factor (App. B: 2.5e5)                       */
  double dx;          /* grid spacing, 1 / 2^n on the periodic unit square    */
  int32_t chi;        /* maximal bond dimension                               */
  double svd_rtol;    /* singular values <= svd_rtol * sigma_max are dropped  */
  double cg_rtol;     /* CG stops at ||r|| <= cg_rtol ||rhs||                 */
  int32_t cg_maxit;   /* CG iteration cap (paper: 100)                        */
  double sweep_rtol;  /* sweep stops when |dN| <= sweep_rtol N; 0 = never     */
  int32_t max_sweeps; /* sweep cap                                            */
  int32_t lap_mode;   /* 0 = three-point D_j^2, 1 = D_j o D_j                 */
  int32_t prec;       /* QTT_PREC_*                                           */
  int32_t precond;    /* QTT_PC_*                                             */
  int32_t rhs_mode;   /* 0: B(b) inside the local networks (App. B, Sec. II.C);
                       * 1: explicit right-hand side: B(b) first fitted as one
                       * chi-bounded MPS on the bonds of b (one-site sweep,
                       * least squares, max_sweeps sweeps; cf. Sec. II.B on
                       * compressing the Hadamard product), then every
                       * minimisation sees a - h w through layer-free networks */
  int32_t fit_sweeps; /* rhs_mode 1: sweeps of the fit of B(b); 0 = max_sweeps  */
} qtt_params;

typedef struct {
  int32_t sweeps[4];        /* sweeps per RK4 stage (qtt_project: [0])          */
  int32_t cg_iters_total;   /* CG iterations over all local solves             */
  int32_t cg_iters_max;     /* largest iteration count of one local solve      */
  int32_t cg_solves;        /* local solves                                    */
  int32_t cg_maxit_hits;    /* local solves that stopped at cg_maxit           */
  int32_t fallbacks;        /* learned preconditioner rejections               */
  int32_t graph_replays;    /* replays of captured CG chunk graphs             */
  double discarded_sq;      /* summed discarded singular weight of truncations */
  double phase_ms[8];       /* host-timed phases: 0 add/truncate, 1 env build,
                               2 local rhs, 3 CG, 4 shift, 5 env update        */
} qtt_stats;

/* Context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t,
 * NULL = the null stream).  Returns QTT_E_HIP if the device is unusable. */
int qtt_ctx_create(qtt_ctx **ctx, int device, void *hip_stream);
void qtt_ctx_destroy(qtt_ctx *ctx);
/* Message of the last failing call on this context ("" if none). */
const char *qtt_last_error(const qtt_ctx *ctx);

/* Doubles needed for an MPS with the given n + 1 bonds. */
int64_t qtt_mps_size(int32_t n, const int32_t *bond);

/* Finite-difference MPO (Sec. II.B, Eq. fdm; App. A, Table diff_mpo):
 * axis 1 acts on x1, axis 2 on x2; order 1 is the central difference
 * (u(x+1) - u(x-1)) / (2 dx), order 2 the three-point second difference.
 * Periodic.  Fills out->bond and out->data (capacity >= n * 144 doubles). */
int qtt_mpo_derivative(qtt_ctx *ctx, int32_t n, int32_t axis, int32_t order, double dx,
                       qtt_mpo *out);

/* y = sum_j coef[j] * x[j]  (exact; Sec. II.C, the RK4 step is a sum of
 * Euler steps).  Bonds add (ends stay 1); cores are block-diagonal with the
 * coefficients folded into site 0.  coef and x are host arrays of length k;
 * the x[j].data and y->data are device pointers. */
int qtt_add(qtt_ctx *ctx, int32_t k, const double *coef, const qtt_mps *x, qtt_mps *y);

/* In-place TT-rounding (Sec. II.B/II.C, compression to chi by repeated
 * SVDs): left-to-right QR sweep, then right-to-left SVD keeping
 * min(chi, 4^k, 4^(n-k), #sigma > svd_rtol * sigma_max) values at each bond.
 * The orthogonality centre ends at site 0.  *discarded_sq (host, may be
 * NULL) receives the summed squares of the dropped singular values, which
 * equals ||y_in - y_out||^2. */
int qtt_truncate(qtt_ctx *ctx, qtt_mps *y, int32_t chi, double svd_rtol, double *discarded_sq);

/* y = W x (App. A; the MPO's second physical index contracts with x).
 * chi = 0: exact, bonds multiply; chi > 0: followed by qtt_truncate. */
int qtt_apply_mpo(qtt_ctx *ctx, const qtt_mpo *W, const qtt_mps *x, int32_t chi,
                  double svd_rtol, qtt_mps *y, double *discarded_sq);

/* y = a (.) b pointwise (Sec. II.B, copy tensors): cores
 * y[(al,al'),w,(be,be')] = a[al,w,be] b[al',w,be'], bonds multiply;
 * chi > 0 truncates afterwards. */
int qtt_hadamard(qtt_ctx *ctx, const qtt_mps *a, const qtt_mps *b, int32_t chi,
                 double svd_rtol, qtt_mps *y, double *discarded_sq);

/* <x|y> (host result). */
int qtt_inner(qtt_ctx *ctx, const qtt_mps *x, const qtt_mps *y, double *out);

/* <x|y> for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no context, no
 * allocation.  The same contraction as qtt_inner, with its workspace in a
 * fixed 3 MiB device array of the library (one copy per device, held until
 * the process ends).  hip_stream: the stream to enqueue on (NULL: the null
 * stream), on the current device; x, y: caller-owned device MPS as for
 * qtt_inner; out: device pointer to one double, written asynchronously
 * (valid once the stream has reached the call's end).  Every bond product
 * x.bond[s] * y.bond[s] and x.bond[s] * y.bond[s+1] must be <= 65536
 * (both bonds <= 256 suffices), else QTT_E_CAPACITY; malformed descriptors,
 * a null out or differing site counts give QTT_E_ARG, a launch failure
 * QTT_E_HIP.  All calls on one device share the workspace: calls that
 * overlap on one device (other streams or host threads) race and must be
 * serialised by the caller. */
int qtt_inner_noalloc(void *hip_stream, const qtt_mps *x, const qtt_mps *y, double *out);

/* Dense grid (device, N x N, x1-major, float64) of an MPS, n <= 13. */
int qtt_to_dense(qtt_ctx *ctx, const qtt_mps *x, double *grid);

/* Input compression of a dense grid (device, N x N, x1-major) into an MPS
 * with bonds <= min(chi, 4^k, 4^(n-k)) by sequential truncated
 * eigen-decompositions of the unfoldings' Gram matrices (input preparation,
 * not part of the time step).  The Gram route resolves singular values only
 * down to about 1e-8 sigma_max, so singular values below
 * max(svd_rtol, 1e-7) * sigma_max are dropped; results agree with an exact
 * TT-SVD to about 1e-7 relative L2. */
int qtt_from_dense(qtt_ctx *ctx, const double *grid, int32_t n, int32_t chi, double svd_rtol,
                   qtt_mps *out);

/* Bond dimension needed per bipartition (the paper's MPS compression
 * efficiency analysis, Eq. epsilon; chi = max_l chi_l): for the dense grid
 * (device, N x N, x1-major, float64, N = 2^n, 2 <= n <= 13) as the quantics
 * state of n sites, counts[l-1] (host, n-1 entries) receives chi_l(eps), the
 * least number of Schmidt values of bipartition l (sites 0..l-1 against
 * l..n-1) whose discarded tail keeps that bipartition's relative L2 error
 * within eps: sqrt(sum_{k >= chi} s_k^2) <= eps sqrt(sum_k s_k^2); at least 1,
 * 0 for a zero field.  The spectra come from the sequential decomposition of
 * qtt_from_dense (Gram eigenvalues: singular values below 1e-7 sigma_max are
 * dropped, bonds capped at chi_cap between cuts), so counts are exact while
 * chi_cap exceeds them and eps is well above 1e-7.  Errors: QTT_E_ARG for
 * null pointers, chi_cap < 1 or eps < 0; QTT_E_UNSUPPORTED for n outside
 * 2..13. */
int qtt_schmidt_counts(qtt_ctx *ctx, const double *grid, int32_t n, double eps, int32_t chi_cap,
                       int32_t *counts);

/* Dense direct numerical simulation used to verify the tensor-network solver
 * (App. D).  Fields u1, u2 are device float64 grids, N x N, x1-major
 * (u[i1 * N + i2] = u(i1 dx, i2 dx)), N = 2^n, 3 <= n <= 11, dx = 1/N, on
 * the periodic unit square; the caller owns them.  Derivatives are the
 * eighth-order central stencils (offsets 1..4); the convection is the
 * skew-symmetric form -1/2 sum_j (u_j d_j u_i + d_j(u_j u_i)), the diffusion
 * (1/Re)(d_11 + d_22) u_i.
 *
 * qtt_dns_rhs: f = C + D at u (f1, f2: device, N x N, distinct from u).
 * qtt_dns_project: in place, the divergence-free part by the Fourier
 *   projection of Eq. projection, u^ - kappa (kappa . u^) / |kappa|^2 for
 *   kappa != 0 with integer wavenumbers and the Nyquist component of kappa
 *   taken as 0 (the mean flow is kept).
 * qtt_dns_step: `steps` steps in place of the explicit Euler scheme
 *   u <- P(u + dt (C + D)) (order 1) or its RK4 extension with every stage
 *   velocity and the final combination projected (order 4).
 * Errors: QTT_E_ARG for null pointers, re <= 0 or NaN, dt not finite,
 * steps < 0 or order not 1 or 4; QTT_E_UNSUPPORTED for n outside 3..11. */
int qtt_dns_rhs(qtt_ctx *ctx, const double *u1, const double *u2, double *f1, double *f2,
                int32_t n, double re);
int qtt_dns_project(qtt_ctx *ctx, double *u1, double *u2, int32_t n);
int qtt_dns_step(qtt_ctx *ctx, double *u1, double *u2, int32_t n, double re, double dt,
                 int32_t order, int32_t steps);

/* Fidelity of Eq. fidelity between two fields of len float64 values (device,
 * any layout, the same for both): *F (host) = <a|b>^2 / (||a||^2 ||b||^2);
 * 0 when either norm is 0.  Errors: QTT_E_ARG for null pointers or len < 1. */
int qtt_fidelity(qtt_ctx *ctx, const double *a, const double *b, int64_t len, double *F);

/* Turbulent kinetic energy spectrum (Eqs. TKE): u' = u - mean (mean1,
 * mean2: device N x N fields, or both null for u' = u), u'^ = FFT(u') / N^2,
 * E(k1, k2) = 1/2 (|u1'^|^2 + |u2'^|^2), and E[k] (host, nshell entries)
 * the sum over the integer wavenumbers with round(|kappa|) = k, k = 0 ..
 * nshell - 1, nshell = round(sqrt(2) N / 2) + 1 (qtt_tke_shells).  Layout of
 * u as for the DNS; 3 <= n <= 11.  Errors: QTT_E_ARG for null fields, a single
 * null mean, a null E or nshell different from qtt_tke_shells(n);
 * QTT_E_UNSUPPORTED for n outside 3..11. */
int32_t qtt_tke_shells(int32_t n);
int qtt_tke_spectrum(qtt_ctx *ctx, const double *u1, const double *u2, const double *mean1,
                     const double *mean2, int32_t n, double *E, int32_t nshell);

/* One Euler minimisation (App. B, Eq. Theta; Eqs. first/second, big_LS):
 *   v = argmin Theta(v; a, b, h)
 * over MPS v_1, v_2 with the bonds of the guess v (in: guess, out: result,
 * centre at site 0).  Local systems
 *   C_i + mu h^2 sum_j P_i^T D_i^T D_j P_j C_j = P_i^T a_i - h P_i^T B_i(b)
 * are solved by CG on the GPU; B_i contains the skew-symmetric convection
 * through Hadamard MPOs of b and the diffusion through D_j^2.  a, b, v are
 * arrays of two MPS; the bonds of v must satisfy
 * bond[k+1] <= 4 bond[k] and bond[k] <= 4 bond[k+1]. */
int qtt_project(qtt_ctx *ctx, const qtt_mps *a, const qtt_mps *b, double h,
                const qtt_params *p, qtt_mps *v, qtt_stats *stats);

/* One RK4 step in place on u (array of two MPS; App. B, Table RK4, Eqs.
 * U1-U4): a = u/4; stage k solves Theta with h = dt/6, dt/3, dt/3, dt/6 and
 * b = u, 3 U1 + u/4, 3/2 U2 + 5/8 u, 3 U3 + u/4 (each truncated to chi);
 * u <- truncate(U1 + U2 + U3 + U4, chi).  u[i].capacity must hold the
 * bonds min(chi, 4^k, 4^(n-k)). */
int qtt_rk4_step(qtt_ctx *ctx, qtt_mps *u, const qtt_params *p, qtt_stats *stats);

/* One time step in place on u (array of two MPS) with the RK schedule of
 * the given order (App. B): order 1 is explicit Euler (Eq. euler), one
 * minimisation of Theta with (a, b, h) = (u, u, dt); order 2 is the
 * midpoint rule (Eqs. midpoint_calc, full_calc): u_mid from (u, u, dt/2),
 * then u from (u, u_mid, dt); order 4 is qtt_rk4_step.  Orders 1 and 2 start
 * every minimisation from the guess u and keep u's bond profile (no
 * truncation, no capacity beyond u's current size); order 4 needs the
 * capacity qtt_rk4_step states.  Any other order: QTT_E_ARG.  Warnings as
 * qtt_project. */
int qtt_rk_step(qtt_ctx *ctx, qtt_mps *u, const qtt_params *p, int32_t order,
                qtt_stats *stats);

/* One RK4 step (as qtt_rk4_step) of each of nflows independent flows, for
 * many flows of uneven size at once.  u holds 2 * nflows MPS (flow f:
 * u[2f], u[2f+1]), p and stats (may be NULL) nflows entries.  The flows are
 * dealt round-robin to `workers` worker contexts (0 = 4, at most 8), each
 * with its own stream and workspace (CG chunks are launched directly, not
 * replayed from graphs), and advanced concurrently after the work already
 * enqueued on the context's stream; the call returns when all flows are
 * done.  Each flow's result is bit-identical to qtt_rk4_step on it
 * alone.  Returns the most negative error over the flows (the message names
 * the flow), else the largest warning. */
int qtt_rk4_step_batched(qtt_ctx *ctx, int32_t nflows, qtt_mps *u, const qtt_params *p,
                         qtt_stats *stats, int32_t workers);

/* Kernel timing for roofline reporting.  While enabled, every launch of the
 * GEMM kernel instantiations QTT_KERNEL_GEMM_* is counted, the kernel adds
 * the flops it executed (2 M N K per batch entry; 0 when it returned early
 * because its CG solve had converged) to a device counter, and every
 * sample_every-th launch is bracketed by HIP events on the context stream.
 * Enabling starts a new window; reading synchronises the stream. */
enum {
  /* each kind covers the instantiations k_gemm<T, BM, BN, WGM, WGN, KD, SA, SB>
     for every operand storage type SA, SB */
  QTT_KERNEL_GEMM_F64_T64 = 0,   /* k_gemm<double, 64, 64, 2, 2, 16, ...>   */
  QTT_KERNEL_GEMM_F32_T64 = 1,   /* k_gemm<float, 64, 64, 2, 2, 16, ...>    */
  QTT_KERNEL_GEMM_F64_T128 = 2,  /* k_gemm<double, 128, 128, 2, 4, 32, ...> */
  QTT_KERNEL_GEMM_F32_T128 = 3   /* k_gemm<float, 128, 128, 2, 4, 32, ...>  */
};
typedef struct {
  int64_t launches;   /* launches in the window                          */
  int64_t timed;      /* launches bracketed by events                    */
  double flops;       /* flops executed by all launches                  */
  double timed_ms;    /* summed event time of the timed launches         */
} qtt_kernel_stats;

int qtt_kernel_timing(qtt_ctx *ctx, int32_t enable, int32_t sample_every);
int qtt_kernel_stats_read(qtt_ctx *ctx, int32_t kernel, qtt_kernel_stats *out);

/* Learned preconditioner of the local CG solves (an addition: the paper
 * solves the local systems of App. B, Eq. big_LS, by plain CG).  With
 * params.precond = QTT_PC_LEARNED every (alpha, beta) position of a centre
 * tensor gets a 4 x 4 block M = L L^T over the physical index, L lower
 * triangular with exp on the diagonal, from a shared-weight perceptron
 * QTT_PC_IN -> QTT_PC_WIDTH -> QTT_PC_WIDTH -> QTT_PC_OUT (ReLU; bfloat16
 * MFMA products, float64 weights) fed with the normalised diagonal block of
 * the local matrix at that position, log of its mean diagonal, the site,
 * log10(mu h^2 / dx^2), the component and the two bond sizes.  PCG runs with
 * M; afterwards the float64 residual of the result is recomputed and plain
 * CG continues from it whenever it misses cg_rtol (stats->fallbacks,
 * return QTT_W_PRECOND_FALLBACK).  QTT_PC_BLOCK_JACOBI uses the exact
 * inverse of the same diagonal blocks instead (the baseline).
 *
 * qtt_precond_config: train_per_solve > 0 turns on training: before every
 * local solve the network takes that many Adam steps (learning rate lr) on
 * the loss ||z - M A z||^2 / ||z||^2 of the solve's own operator A with a
 * fresh Gaussian probe z drawn on the device; 0 = inference only.
 * reset != 0 (or the first call) draws the weights from `seed` and clears
 * the Adam state.  Weights persist in the context. */
enum { QTT_PC_IN = 16, QTT_PC_WIDTH = 256, QTT_PC_OUT = 10 };
int qtt_precond_config(qtt_ctx *ctx, int32_t train_per_solve, double lr, uint64_t seed,
                       int32_t reset);
/* Number of parameters, Adam steps taken, probe loss of the first and of the
 * latest training step (-1 before any).  Any pointer may be NULL. */
int qtt_precond_info(qtt_ctx *ctx, int64_t *nparam, int64_t *steps, double *first_loss,
                     double *last_loss);
/* Copy the float64 parameters (W1 [W][IN], b1 [W], W2 [W][W], b2 [W],
 * W3 [OUT][W], b3 [OUT], row-major, packed in this order) to (set = 0) or
 * from (set = 1) the host array w of n = nparam doubles. */
int qtt_precond_weights(qtt_ctx *ctx, int32_t set, double *w, int64_t n);
/* Write the weights to the file `path` / read them back (the host-side
 * persistence of a trained network): an 8-byte tag "QTTPCNET", four int64
 * (nparam, QTT_PC_IN, QTT_PC_WIDTH, QTT_PC_OUT), then the nparam float64 of
 * qtt_precond_weights, host byte order.  A file that cannot be opened or
 * written, or that is not a weights file of this network, gives QTT_E_ARG
 * (load leaves the weights unchanged). */
int qtt_precond_save(qtt_ctx *ctx, const char *path);
int qtt_precond_load(qtt_ctx *ctx, const char *path);
/* Network forward and backward on given rows (device pointers): X is
 * npos x QTT_PC_IN, dY and Y are npos x QTT_PC_OUT, grad holds nparam
 * doubles.  Y = network output, grad = gradient of sum(dY * Y) with respect
 * to the parameters (layout as in qtt_precond_weights). */
int qtt_precond_grad(qtt_ctx *ctx, const double *X, int64_t npos, const double *dY, double *Y,
                     double *grad);

#ifdef __cplusplus
}
#endif

#endif /* QTT_H */
