// Conjugate-gradient vector kernels with device-resident scalars.
//
// The local systems of the sweep are solved by CG (Sec. II.C) entirely on the
// device: alpha, beta and the convergence decision never travel to the host.
// Each kernel computes its reduction as per-block partials in a fixed order
// and the last block to finish combines them (deterministic result), then
// updates the scalar state.  Once `done` is set every later kernel of the
// solve (including the matvec GEMMs, through their skip flag) returns
// immediately, so the host can enqueue iterations in chunks and check the
// flag once per chunk.
#include "qtt_internal.h"
#include "qtt_cg.h"

namespace qtt {

namespace {

constexpr int CG_THREADS = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return s;
}

// true in every thread of the last block to arrive (block-uniform)
__device__ inline bool arrive_last(CGState *st, double *part, int slot, double s0, double s1) {
  __shared__ bool last;
  if (threadIdx.x == 0) {
    part[2 * slot] = s0;
    part[2 * slot + 1] = s1;
    __threadfence();
    const unsigned prev = atomicAdd(&st->counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// fixed-order sum of the np partial pairs by the whole (last) block; the
// result is valid in every thread
__device__ inline void sum_parts(const double *part, int np, double &s0, double &s1) {
  __shared__ double sh[2][CG_THREADS / 64];
  const volatile double *vp = part;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < np; i += CG_THREADS) {
    a += vp[2 * i];
    b += vp[2 * i + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  s0 = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
  s1 = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
}

// r = rhs - q (q = A x0), p = z = M r (M = I here), rr = r.r, bnorm2 = rhs.rhs
__global__ __launch_bounds__(CG_THREADS) void k_cg_init(const double *rhs, const double *q,
                                                        double *r, double *p, int64_t n,
                                                        CGState *st, double *part) {
  __shared__ double sh[4];
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS) {
    const double ri = rhs[i] - q[i];
    r[i] = ri;
    p[i] = ri;
    a += ri * ri;
    b += rhs[i] * rhs[i];
  }
  const double sa = block_sum(a, sh);
  __syncthreads();
  const double sb = block_sum(b, sh);
  if (arrive_last(st, part, blockIdx.x, sa, sb)) {
    double rr, bn;
    sum_parts(part, gridDim.x, rr, bn);
    if (threadIdx.x == 0) {
      st->rr = rr;
      st->rz = rr;
      st->rr_new = rr;
      st->gamma = rr;
      st->first = 1;
      st->bnorm2 = bn;
      st->tol2 = st->rtol * st->rtol * bn;
      st->iters = 0;
      st->converged = 0;
      st->zero_x = (bn == 0.0) ? 1 : 0;
      st->done = (bn == 0.0 || rr <= st->tol2) ? 1 : 0;
      if (st->done) st->converged = 1;
      st->counter = 0;
    }
  }
}

// state reset before a solve (the fields cg_init does not set itself)
__global__ void k_cg_reset(CGState *st, double rtol, int maxit, int precond) {
  if (threadIdx.x != 0) return;
  st->rtol = rtol;
  st->maxit = maxit;
  st->precond = precond;
  st->done = 0;
  st->counter = 0;
}

__global__ void k_cg_zero_if(double *x, int64_t n, const CGState *st) {
  if (!st->zero_x) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// alpha = rz / (p . q)
__global__ __launch_bounds__(CG_THREADS) void k_cg_alpha(const double *p, const double *q,
                                                         int64_t n, CGState *st, double *part) {
  if (st->done) return;
  __shared__ double sh[4];
  double a = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS)
    a += p[i] * q[i];
  const double sa = block_sum(a, sh);
  if (arrive_last(st, part, blockIdx.x, sa, 0.0)) {
    double pq, dummy;
    sum_parts(part, gridDim.x, pq, dummy);
    if (threadIdx.x == 0) {
      st->pq = pq;
      st->alpha = st->rz / pq;
      st->counter = 0;
    }
  }
}

// x += alpha p, r -= alpha q, rr_new = r . r ; convergence test
__global__ __launch_bounds__(CG_THREADS) void k_cg_update(double *x, double *r, const double *p,
                                                          const double *q, int64_t n, CGState *st,
                                                          double *part) {
  if (st->done) return;
  __shared__ double sh[4];
  const double al = st->alpha;
  double a = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS) {
    x[i] += al * p[i];
    const double ri = r[i] - al * q[i];
    r[i] = ri;
    a += ri * ri;
  }
  const double sa = block_sum(a, sh);
  if (arrive_last(st, part, blockIdx.x, sa, 0.0)) {
    double rr, dummy;
    sum_parts(part, gridDim.x, rr, dummy);
    if (threadIdx.x == 0) {
      st->iters += 1;
      // plain CG: rr <- previous r.r (for beta), rr_new = rz <- new r.r (for
      // beta and the next alpha); PCG keeps rz = r.z for pcg_next
      if (!st->precond) {
        st->rr = st->rz;
        st->rz = rr;
      }
      st->rr_new = rr;
      if (!(rr == rr)) {
        st->done = 1;  // NaN: stop, not converged
      } else if (rr <= st->tol2) {
        st->done = 1;
        st->converged = 1;
      } else if (st->iters >= st->maxit) {
        st->done = 1;
      }
      st->counter = 0;
    }
  }
}

// unpreconditioned: beta = rr_new / rr, p = r + beta p
__global__ __launch_bounds__(CG_THREADS) void k_cg_pupdate(const double *r, double *p, int64_t n,
                                                           CGState *st) {
  if (st->done) return;
  const double beta = st->rr_new / st->rr;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS)
    p[i] = r[i] + beta * p[i];
}

// preconditioned: rz_new = r . z ; beta = rz_new / rz ; p = z + beta p (two kernels)
__global__ __launch_bounds__(CG_THREADS) void k_pcg_rz(const double *r, const double *z,
                                                       int64_t n, CGState *st, double *part) {
  if (st->done) return;
  __shared__ double sh[4];
  double a = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS)
    a += r[i] * z[i];
  const double sa = block_sum(a, sh);
  if (arrive_last(st, part, blockIdx.x, sa, 0.0)) {
    double rz, dummy;
    sum_parts(part, gridDim.x, rz, dummy);
    if (threadIdx.x == 0) {
      st->beta = rz / st->rz;
      st->rz = rz;
      st->rr = st->rr_new;
      st->counter = 0;
    }
  }
}

__global__ __launch_bounds__(CG_THREADS) void k_pcg_pupdate(const double *z, double *p, int64_t n,
                                                            const CGState *st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS)
    p[i] = z[i] + beta * p[i];
}

// PCG start: z = M r already computed; p = z, rz = r . z
__global__ __launch_bounds__(CG_THREADS) void k_pcg_start(const double *r, const double *z,
                                                          double *p, int64_t n, CGState *st,
                                                          double *part) {
  if (st->done) return;
  __shared__ double sh[4];
  double a = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)CG_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * CG_THREADS) {
    p[i] = z[i];
    a += r[i] * z[i];
  }
  const double sa = block_sum(a, sh);
  if (arrive_last(st, part, blockIdx.x, sa, 0.0)) {
    double rz, dummy;
    sum_parts(part, gridDim.x, rz, dummy);
    if (threadIdx.x == 0) {
      st->rz = rz;
      st->counter = 0;
    }
  }
}

inline unsigned cg_grid(int64_t n) {
  int64_t g = (n + CG_THREADS * 4 - 1) / (CG_THREADS * 4);
  if (g > 512) g = 512;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

static void chk(Ctx &c, const double *v, int64_t n, const char *w) {
  c.check_range(v, 0, n - 1, 8, w);
}

void cg_reset(Ctx &c, CGState *st, double rtol, int maxit, int precond) {
  c.check_range(st, 0, 0, sizeof(CGState), "cg state");
  hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(64), 0, c.stream, st, rtol, maxit, precond);
  HIPC(hipGetLastError());
}

void cg_init(Ctx &c, const double *rhs, const double *q, double *r, double *p, double *x,
             int64_t n, CGState *st, double *part) {
  const unsigned g = cg_grid(n);
  chk(c, rhs, n, "cg rhs");
  chk(c, q, n, "cg q");
  chk(c, r, n, "cg r");
  chk(c, p, n, "cg p");
  chk(c, x, n, "cg x");
  chk(c, part, 2 * g, "cg partials");
  c.check_range(st, 0, 0, sizeof(CGState), "cg state");
  hipLaunchKernelGGL(k_cg_init, dim3(g), dim3(CG_THREADS), 0, c.stream, rhs, q, r, p, n, st,
                     part);
  hipLaunchKernelGGL(k_cg_zero_if, dim3(g), dim3(CG_THREADS), 0, c.stream, x, n, st);
  HIPC(hipGetLastError());
}

void cg_alpha(Ctx &c, const double *p, const double *q, int64_t n, CGState *st, double *part) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, p, q, n, st,
                     part);
  HIPC(hipGetLastError());
}

void cg_update(Ctx &c, double *x, double *r, const double *p, const double *q, int64_t n,
               CGState *st, double *part) {
  hipLaunchKernelGGL(k_cg_update, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, x, r, p, q, n,
                     st, part);
  HIPC(hipGetLastError());
}

void cg_pupdate(Ctx &c, const double *r, double *p, int64_t n, CGState *st) {
  hipLaunchKernelGGL(k_cg_pupdate, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, r, p, n, st);
  HIPC(hipGetLastError());
}

void pcg_start(Ctx &c, const double *r, const double *z, double *p, int64_t n, CGState *st,
               double *part) {
  hipLaunchKernelGGL(k_pcg_start, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, r, z, p, n,
                     st, part);
  HIPC(hipGetLastError());
}

void pcg_next(Ctx &c, const double *r, const double *z, double *p, int64_t n, CGState *st,
              double *part) {
  hipLaunchKernelGGL(k_pcg_rz, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, r, z, n, st,
                     part);
  hipLaunchKernelGGL(k_pcg_pupdate, dim3(cg_grid(n)), dim3(CG_THREADS), 0, c.stream, z, p, n, st);
  HIPC(hipGetLastError());
}

}  // namespace qtt
