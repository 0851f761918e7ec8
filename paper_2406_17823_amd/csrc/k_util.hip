// Element-wise and data-movement kernels of the MPS algebra: block placement
// for MPS sums, Hadamard and MPO site products, index permutations, the
// quantics (Morton) reordering of grids, deterministic dot products.
// All are HBM-bound; grid-stride loops with unit-stride writes.
#include "qtt_internal.h"

namespace qtt {

namespace {

inline unsigned grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f32(float *p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_scale_copy(double *d, const double *s, int64_t n, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = a * s[i];
}

__global__ void k_axpy_into(double *y, const double *x, int64_t n, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

__global__ void k_permute3(double *dst, const double *src, int d0, int d1, int d2, int64_t s0,
                           int64_t s1, int64_t s2, double a) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int i2 = (int)(i % d2);
    const int64_t t = i / d2;
    const int i1 = (int)(t % d1);
    const int i0 = (int)(t / d1);
    dst[i] = a * src[i0 * s0 + i1 * s1 + i2 * s2];
  }
}

__global__ void k_place_block(double *dst, int dl, int dr, const double *src, int l, int r,
                              int ol, int orr, double a) {
  const int64_t n = (int64_t)l * 4 * r;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i % r);
    const int64_t t = i / r;
    const int w = (int)(t % 4);
    const int al = (int)(t / 4);
    dst[((int64_t)(ol + al) * 4 + w) * dr + orr + b] = a * src[i];
  }
}

// y[(al,al'), w, (be,be')] = A[al,w,be] * B[al',w,be']
__global__ void k_hadamard(double *y, const double *A, int la, int ra, const double *B, int lb,
                           int rb) {
  const int64_t R = (int64_t)ra * rb;
  const int64_t n = (int64_t)la * lb * 4 * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = i % R;
    const int64_t t = i / R;
    const int w = (int)(t % 4);
    const int64_t row = t / 4;
    const int al = (int)(row / lb), alp = (int)(row % lb);
    const int be = (int)(col / rb), bep = (int)(col % rb);
    y[i] = A[((int64_t)al * 4 + w) * ra + be] * B[((int64_t)alp * 4 + w) * rb + bep];
  }
}

// y[(a,al), w, (b,be)] = sum_w' W[a,w,w',b] x[al,w',be]
__global__ void k_mpo_core(double *y, const double *W, int wl, int wr, const double *x, int l,
                           int r) {
  const int64_t R = (int64_t)wr * r;
  const int64_t n = (int64_t)wl * l * 4 * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = i % R;
    const int64_t t = i / R;
    const int w = (int)(t % 4);
    const int64_t row = t / 4;
    const int a = (int)(row / l), al = (int)(row % l);
    const int b = (int)(col / r), be = (int)(col % r);
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      s += W[(((int64_t)a * 4 + w) * 4 + v) * wr + b] * x[((int64_t)al * 4 + v) * r + be];
    y[i] = s;
  }
}

__device__ inline int64_t morton(int x1, int x2, int n) {
  int64_t idx = 0;
  for (int k = 0; k < n; ++k) {
    const int b1 = (x1 >> (n - 1 - k)) & 1;
    const int b2 = (x2 >> (n - 1 - k)) & 1;
    idx |= (int64_t)(2 * b1 + b2) << (2 * (n - 1 - k));
  }
  return idx;
}

__global__ void k_morton_gather(double *grid, const double *vec, int n) {
  const int N = 1 << n;
  const int64_t tot = (int64_t)N * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x)
    grid[i] = vec[morton((int)(i / N), (int)(i % N), n)];
}

__global__ void k_morton_scatter(double *vec, const double *grid, int n) {
  const int N = 1 << n;
  const int64_t tot = (int64_t)N * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x)
    vec[morton((int)(i / N), (int)(i % N), n)] = grid[i];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// per-block partial sums, then one block adds them in index order
__global__ __launch_bounds__(256) void k_dot_partial(const double *x, const double *y, int64_t n,
                                                     double *part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *part, int np, double *out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_nonfinite(const double *x, int64_t n, int *flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) *flag = 1;
}

// up to four contiguous copies in one launch (blockIdx.y selects the pair)
struct CopyPairs {
  double *dst[4];
  const double *src[4];
  int64_t n[4];
};
__global__ void k_copy_pairs(CopyPairs P) {
  const int k = blockIdx.y;
  double *d = P.dst[k];
  const double *s = P.src[k];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P.n[k];
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

}  // namespace

void copy_pairs(Ctx &c, int np, double *const *dst, const double *const *src, const int64_t *n) {
  if (np < 1 || np > 4) fail(QTT_E_ARG, "copy_pairs: 1..4 copies");
  CopyPairs P{};
  int64_t mx = 0;
  for (int k = 0; k < np; ++k) {
    if (n[k] > 0) {
      c.check_range(src[k], 0, n[k] - 1, sizeof(double), "copy_pairs src");
      c.check_range(dst[k], 0, n[k] - 1, sizeof(double), "copy_pairs dst");
    }
    P.dst[k] = dst[k];
    P.src[k] = src[k];
    P.n[k] = std::max<int64_t>(n[k], 0);
    mx = std::max(mx, P.n[k]);
  }
  if (mx == 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, (mx + 255) / 256);
  hipLaunchKernelGGL(k_copy_pairs, dim3(g, np), dim3(256), 0, c.stream, P);
  HIPC(hipGetLastError());
}

void fill(Ctx &c, double *p, int64_t n, double v) {
  if (n <= 0) return;
  c.check_range(p, 0, n - 1, 8, "fill");
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, c.stream, p, n, v);
  HIPC(hipGetLastError());
}

void fill_f32(Ctx &c, float *p, int64_t n, float v) {
  if (n <= 0) return;
  c.check_range(p, 0, n - 1, 4, "fill_f32");
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, c.stream, p, n, v);
  HIPC(hipGetLastError());
}

void scale_copy(Ctx &c, double *d, const double *s, int64_t n, double a) {
  if (n <= 0) return;
  c.check_range(d, 0, n - 1, 8, "scale_copy dst");
  c.check_range(s, 0, n - 1, 8, "scale_copy src");
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, c.stream, d, s, n, a);
  HIPC(hipGetLastError());
}

void axpy_into(Ctx &c, double *y, const double *x, int64_t n, double a) {
  if (n <= 0) return;
  c.check_range(y, 0, n - 1, 8, "axpy y");
  c.check_range(x, 0, n - 1, 8, "axpy x");
  hipLaunchKernelGGL(k_axpy_into, dim3(grid_for(n)), dim3(256), 0, c.stream, y, x, n, a);
  HIPC(hipGetLastError());
}

void permute3(Ctx &c, double *dst, const double *src, int d0, int d1, int d2, int64_t s0,
              int64_t s1, int64_t s2, double a) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  if (n <= 0) return;
  c.check_range(dst, 0, n - 1, 8, "permute3 dst");
  {
    int64_t lo = 0, hi = 0;
    span(lo, hi, d0, s0);
    span(lo, hi, d1, s1);
    span(lo, hi, d2, s2);
    c.check_range(src, lo, hi, 8, "permute3 src");
  }
  hipLaunchKernelGGL(k_permute3, dim3(grid_for(n)), dim3(256), 0, c.stream, dst, src, d0, d1,
                     d2, s0, s1, s2, a);
  HIPC(hipGetLastError());
}

void place_block(Ctx &c, double *dst, int dl, int dr, const double *src, int l, int r, int ol,
                 int orr, double a) {
  const int64_t n = (int64_t)l * 4 * r;
  if (n <= 0) return;
  if (ol + l > dl || orr + r > dr) fail(QTT_E_SHAPE, "place_block: block outside core");
  c.check_range(dst, 0, (int64_t)dl * 4 * dr - 1, 8, "place_block dst");
  c.check_range(src, 0, n - 1, 8, "place_block src");
  hipLaunchKernelGGL(k_place_block, dim3(grid_for(n)), dim3(256), 0, c.stream, dst, dl, dr, src,
                     l, r, ol, orr, a);
  HIPC(hipGetLastError());
}

void hadamard_core(Ctx &c, double *y, const double *a, int la, int ra, const double *b, int lb,
                   int rb) {
  const int64_t n = (int64_t)la * lb * 4 * ra * rb;
  c.check_range(y, 0, n - 1, 8, "hadamard y");
  c.check_range(a, 0, (int64_t)la * 4 * ra - 1, 8, "hadamard a");
  c.check_range(b, 0, (int64_t)lb * 4 * rb - 1, 8, "hadamard b");
  hipLaunchKernelGGL(k_hadamard, dim3(grid_for(n)), dim3(256), 0, c.stream, y, a, la, ra, b, lb,
                     rb);
  HIPC(hipGetLastError());
}

void mpo_core(Ctx &c, double *y, const double *W, int wl, int wr, const double *x, int l, int r) {
  const int64_t n = (int64_t)wl * l * 4 * wr * r;
  c.check_range(y, 0, n - 1, 8, "mpo_core y");
  c.check_range(W, 0, (int64_t)wl * 16 * wr - 1, 8, "mpo_core W");
  c.check_range(x, 0, (int64_t)l * 4 * r - 1, 8, "mpo_core x");
  hipLaunchKernelGGL(k_mpo_core, dim3(grid_for(n)), dim3(256), 0, c.stream, y, W, wl, wr, x, l,
                     r);
  HIPC(hipGetLastError());
}

void morton_gather(Ctx &c, double *grid, const double *vec, int n) {
  const int64_t N2 = (int64_t)1 << (2 * n);
  c.check_range(grid, 0, N2 - 1, 8, "morton grid");
  c.check_range(vec, 0, N2 - 1, 8, "morton vec");
  hipLaunchKernelGGL(k_morton_gather, dim3(grid_for(N2)), dim3(256), 0, c.stream, grid, vec, n);
  HIPC(hipGetLastError());
}

void morton_scatter(Ctx &c, double *vec, const double *grid, int n) {
  const int64_t N2 = (int64_t)1 << (2 * n);
  c.check_range(grid, 0, N2 - 1, 8, "morton grid");
  c.check_range(vec, 0, N2 - 1, 8, "morton vec");
  hipLaunchKernelGGL(k_morton_scatter, dim3(grid_for(N2)), dim3(256), 0, c.stream, vec, grid, n);
  HIPC(hipGetLastError());
}

void dot(Ctx &c, const double *x, const double *y, int64_t n, double *out_dev) {
  const int np = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  double *part = c.buf("dot_partials", 1024);
  if (n > 0) {
    c.check_range(x, 0, n - 1, 8, "dot x");
    c.check_range(y, 0, n - 1, 8, "dot y");
  }
  c.check_range(out_dev, 0, 0, 8, "dot out");
  hipLaunchKernelGGL(k_dot_partial, dim3(np), dim3(256), 0, c.stream, x, y, n, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, c.stream, part, np, out_dev);
  HIPC(hipGetLastError());
}

int any_nonfinite(Ctx &c, const double *x, int64_t n) {
  int *flag = (int *)c.raw("nonfinite_flag", sizeof(int));
  HIPC(hipMemsetAsync(flag, 0, sizeof(int), c.stream));
  if (n > 0) c.check_range(x, 0, n - 1, 8, "nonfinite");
  if (n > 0)
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n)), dim3(256), 0, c.stream, x, n, flag);
  int h = 0;
  HIPC(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  c.sync();
  return h;
}

}  // namespace qtt
