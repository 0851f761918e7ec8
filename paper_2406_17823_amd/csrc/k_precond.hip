// Learned block preconditioner of the local CG solves.
//
// For component i at site d, every position (alpha, beta) of the centre
// tensor owns a 4 x 4 block over the physical index omega.  Its features come
// from the diagonal 4 x 4 block of the local matrix,
//   B(al, be) = I + mu h^2 sum_{m, m'} L_ii[al][m][al] W_ii[m][w][w'][m'] R_ii[be][m'][be],
// built from the penalty pair (i, i)'s environments and composed core.  A
// 3-layer perceptron (width 256; bfloat16 MFMA operands, float32 slice
// accumulation, float64 weights, biases and activations) maps them to the 10
// entries of a lower-triangular factor L (diagonal through exp), and the
// block of the preconditioner is M = L L^T, symmetric positive definite for
// any weights, so PCG stays valid whatever the network outputs.  Training
// minimises ||z - M A z||^2 / ||z||^2 over Gaussian probes z drawn on the
// device, with A the exact local operator; gradients flow back through the
// factor and the network in hand-written kernels, followed by Adam.
#include "qtt_internal.h"

#include <cmath>
#include <vector>

namespace qtt {

namespace {

// row-major lower triangle of a 4 x 4 matrix: t -> (r, c)
__device__ inline void tri(int t, int &r, int &c) {
  r = (t >= 6) ? 3 : (t >= 3) ? 2 : (t >= 1) ? 1 : 0;
  c = t - r * (r + 1) / 2;
}

inline unsigned grid1(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

__global__ void k_pc_features(const double *Lenv, const double *Renv, const double *W, int la,
                              int ra, int mi, int mo, double muh2, double f_site, double f_pen,
                              double f_comp, double f_la, double f_ra, double *X, double *Bblk) {
  const int64_t npos = (int64_t)la * ra;
  for (int64_t pidx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pidx < npos;
       pidx += (int64_t)gridDim.x * blockDim.x) {
    const int al = (int)(pidx / ra), be = (int)(pidx % ra);
    double B[16];
    for (int e = 0; e < 16; ++e) B[e] = 0.0;
    for (int m = 0; m < mi; ++m) {
      const double lv = Lenv[((int64_t)al * mi + m) * la + al];
      for (int mp = 0; mp < mo; ++mp) {
        const double s = lv * Renv[((int64_t)be * mo + mp) * ra + be];
        for (int e = 0; e < 16; ++e) B[e] += s * W[((int64_t)m * 16 + e) * mo + mp];
      }
    }
    for (int e = 0; e < 16; ++e) B[e] *= muh2;
    for (int w = 0; w < 4; ++w) B[w * 5] += 1.0;
    for (int e = 0; e < 16; ++e) Bblk[pidx * 16 + e] = B[e];
    const double tr = 0.25 * (B[0] + B[5] + B[10] + B[15]);
    double *x = X + pidx * PC_IN;
    for (int t = 0; t < 10; ++t) {
      int r, c;
      tri(t, r, c);
      x[t] = B[r * 4 + c] / tr;
    }
    x[10] = log(tr);
    x[11] = f_site;
    x[12] = f_pen;
    x[13] = f_comp;
    x[14] = f_la;
    x[15] = f_ra;
  }
}

// Z += b (column bias); H = relu(Z) when H is given
__global__ void k_pc_bias_act(double *Z, double *H, const double *b, int64_t rows, int cols) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double z = Z[i] + b[i % cols];
    Z[i] = z;
    if (H) H[i] = z > 0.0 ? z : 0.0;
  }
}

// Y (PC_OUT per row) -> L (16 per row, kept when Lf is given) -> M = L L^T
__global__ void k_pc_factor(const double *Y, double *M, double *Lf, int64_t rows) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < rows;
       p += (int64_t)gridDim.x * blockDim.x) {
    double L[16];
    for (int e = 0; e < 16; ++e) L[e] = 0.0;
    for (int t = 0; t < 10; ++t) {
      int r, c;
      tri(t, r, c);
      const double y = Y[p * PC_OUT + t];
      L[r * 4 + c] = (r == c) ? exp(fmax(fmin(y, 30.0), -30.0)) : y;
    }
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += L[r * 4 + k] * L[c * 4 + k];
        M[p * 16 + r * 4 + c] = s;
      }
    if (Lf)
      for (int e = 0; e < 16; ++e) Lf[p * 16 + e] = L[e];
  }
}

// exact inverse of each diagonal block (the block-Jacobi baseline)
__global__ void k_pc_block_inverse(const double *Bblk, double *M, int64_t rows) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < rows;
       p += (int64_t)gridDim.x * blockDim.x) {
    double a[16], inv[16];
    for (int e = 0; e < 16; ++e) {
      a[e] = Bblk[p * 16 + e];
      inv[e] = (e % 5 == 0) ? 1.0 : 0.0;
    }
    // Gauss-Jordan; the blocks are SPD with diagonal >= 1, no pivoting needed
    for (int c = 0; c < 4; ++c) {
      const double ip = 1.0 / a[c * 4 + c];
      for (int k = 0; k < 4; ++k) {
        a[c * 4 + k] *= ip;
        inv[c * 4 + k] *= ip;
      }
      for (int r = 0; r < 4; ++r) {
        if (r == c) continue;
        const double f = a[r * 4 + c];
        for (int k = 0; k < 4; ++k) {
          a[r * 4 + k] -= f * a[c * 4 + k];
          inv[r * 4 + k] -= f * inv[c * 4 + k];
        }
      }
    }
    for (int e = 0; e < 16; ++e) M[p * 16 + e] = inv[e];
  }
}

// z[al][w][be] = sum_w' M(al, be)[w][w'] r[al][w'][be]
__global__ void k_pc_apply(const double *M, const double *r, double *z, int la, int ra,
                           const int *skip) {
  if (skip && *skip) return;
  const int64_t npos = (int64_t)la * ra;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npos;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int al = (int)(p / ra), be = (int)(p % ra);
    double v[4];
    for (int w = 0; w < 4; ++w) v[w] = r[((int64_t)al * 4 + w) * ra + be];
    for (int w = 0; w < 4; ++w) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += M[p * 16 + w * 4 + k] * v[k];
      z[((int64_t)al * 4 + w) * ra + be] = s;
    }
  }
}

// counter-based standard normal probes: splitmix64 finaliser + Box-Muller
__device__ inline uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__global__ void k_pc_probe(double *z, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t a = mix64(seed + 2 * (uint64_t)i), b = mix64(seed + 2 * (uint64_t)i + 1);
    const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    z[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// per position p: res = z_p - M_p (Az)_p, loss += |res|^2 / zz,
// G = dloss/dM_p = -2 res (Az)_p^T / zz, dL = (G + G^T) L, and dY on the
// factor entries (times L_rr on the diagonal, the derivative of exp)
__global__ __launch_bounds__(256) void k_pc_loss_grad(const double *M, const double *Lf,
                                                      const double *z, const double *Az, int la,
                                                      int ra, const double *zz, double *dY,
                                                      double *loss) {
  const int64_t npos = (int64_t)la * ra;
  const double inv = 1.0 / *zz;
  double lsum = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npos;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int al = (int)(p / ra), be = (int)(p % ra);
    double zv[4], av[4], res[4];
    for (int w = 0; w < 4; ++w) {
      zv[w] = z[((int64_t)al * 4 + w) * ra + be];
      av[w] = Az[((int64_t)al * 4 + w) * ra + be];
    }
    for (int w = 0; w < 4; ++w) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += M[p * 16 + w * 4 + k] * av[k];
      res[w] = zv[w] - s;
      lsum += res[w] * res[w];
    }
    const double *L = Lf + p * 16;
    for (int t = 0; t < 10; ++t) {
      int r, c;
      tri(t, r, c);
      double g = 0.0;
      for (int k = 0; k < 4; ++k) g += (res[r] * av[k] + res[k] * av[r]) * L[k * 4 + c];
      g *= -2.0 * inv;
      if (r == c) g *= L[r * 4 + c];
      dY[p * PC_OUT + t] = g;
    }
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = lsum * inv;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, sh[0]);
}

// dZ = dH where Z > 0, else 0
__global__ void k_pc_relu_back(const double *Z, double *dH, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!(Z[i] > 0.0)) dH[i] = 0.0;
}

// column sums of dZ (rows x cols), two passes: partials over row chunks of
// PC_ROWS rows (block = 64 columns x 4 row lanes), then a fixed-order sum
constexpr int PC_ROWS = 1024;
__global__ __launch_bounds__(256) void k_pc_colsum_part(const double *dZ, int64_t rows, int cols,
                                                        double *part) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int lane_r = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * PC_ROWS;
  const int64_t r1 = r0 + PC_ROWS < rows ? r0 + PC_ROWS : rows;
  double s = 0.0;
  if (c < cols)
    for (int64_t r = r0 + lane_r; r < r1; r += 4) s += dZ[r * cols + c];
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64 && c < cols)
    part[(int64_t)blockIdx.y * cols + c] =
        (sh[threadIdx.x] + sh[threadIdx.x + 64]) + (sh[threadIdx.x + 128] + sh[threadIdx.x + 192]);
}

__global__ void k_pc_colsum_fin(const double *part, int nchunk, int cols, double *db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += part[(int64_t)k * cols + c];
  db[c] = s;
}

__global__ void k_pc_adam(double *w, const double *g, double *m, double *v, int64_t n, double lr,
                          double b1, double b2, double bc1, double bc2, double eps) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrt(vi / bc2) + eps);
  }
}

// host-side counter-based normal stream for the initial weights
struct HostNormal {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t x = s;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
  }
  double operator()() {
    const double u1 = ((double)(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// C (rows x kout) = A (rows x kin) W^T, W row-major kout x kin
void lin_fwd(Ctx &c, const double *A, int64_t rows, int kin, const double *W, int kout, double *C) {
  Gemm q;
  q.M = (int)rows;
  q.N = kout;
  q.K = kin;
  q.A = A;
  q.sAm = kin;
  q.sAk = 1;
  q.B = W;
  q.sBk = 1;
  q.sBn = kin;
  q.C = C;
  q.sCm = kout;
  q.sCn = 1;
  gemm_bf16(c, q);
}

// dW (kout x kin) = dZ^T A
void lin_wgrad(Ctx &c, const double *dZ, int64_t rows, int kout, const double *A, int kin,
               double *dW) {
  Gemm q;
  q.M = kout;
  q.N = kin;
  q.K = (int)rows;
  q.A = dZ;
  q.sAm = 1;
  q.sAk = kout;
  q.B = A;
  q.sBk = kin;
  q.sBn = 1;
  q.C = dW;
  q.sCm = kin;
  q.sCn = 1;
  gemm_bf16(c, q);
}

// dA (rows x kin) = dZ W
void lin_agrad(Ctx &c, const double *dZ, int64_t rows, int kout, const double *W, int kin,
               double *dA) {
  Gemm q;
  q.M = (int)rows;
  q.N = kin;
  q.K = kout;
  q.A = dZ;
  q.sAm = kout;
  q.sAk = 1;
  q.B = W;
  q.sBk = kin;
  q.sBn = 1;
  q.C = dA;
  q.sCm = kin;
  q.sCn = 1;
  gemm_bf16(c, q);
}

void colsum(Ctx &c, const double *dZ, int64_t rows, int cols, double *db) {
  const int nchunk = (int)((rows + PC_ROWS - 1) / PC_ROWS);
  double *part = c.buf("pc_colpart", (int64_t)nchunk * cols);
  c.check_range(dZ, 0, rows * cols - 1, 8, "pc colsum dZ");
  c.check_range(db, 0, cols - 1, 8, "pc colsum db");
  hipLaunchKernelGGL(k_pc_colsum_part, dim3((cols + 63) / 64, nchunk), dim3(256), 0, c.stream, dZ,
                     rows, cols, part);
  hipLaunchKernelGGL(k_pc_colsum_fin, dim3((cols + 255) / 256), dim3(256), 0, c.stream, part,
                     nchunk, cols, db);
  HIPC(hipGetLastError());
}

// activations for `rows` rows (grows the named buffers; contents not kept)
void act_buffers(Ctx &c, int64_t rows) {
  PrecondNet &net = c.pc;
  net.Z1 = c.buf("pc_Z1", rows * PC_W);
  net.H1 = c.buf("pc_H1", rows * PC_W);
  net.Z2 = c.buf("pc_Z2", rows * PC_W);
  net.H2 = c.buf("pc_H2", rows * PC_W);
  net.Y = c.buf("pc_Y", rows * PC_OUT);
  net.Lf = c.buf("pc_L", rows * 16);
  net.dY = c.buf("pc_dY", rows * PC_OUT);
  net.act_rows = rows;
}

// backward from dY (rows x PC_OUT) into grad (nparam), activations stored
void backward(Ctx &c, const double *X, int64_t rows, const double *dY, double *grad) {
  PrecondNet &net = c.pc;
  double *dH2 = c.buf("pc_dH2", rows * PC_W), *dH1 = c.buf("pc_dH1", rows * PC_W);
  lin_wgrad(c, dY, rows, PC_OUT, net.H2, PC_W, grad + net.off[4]);
  colsum(c, dY, rows, PC_OUT, grad + net.off[5]);
  lin_agrad(c, dY, rows, PC_OUT, net.w + net.off[4], PC_W, dH2);
  hipLaunchKernelGGL(k_pc_relu_back, dim3(grid1(rows * PC_W)), dim3(256), 0, c.stream, net.Z2,
                     dH2, rows * PC_W);
  lin_wgrad(c, dH2, rows, PC_W, net.H1, PC_W, grad + net.off[2]);
  colsum(c, dH2, rows, PC_W, grad + net.off[3]);
  lin_agrad(c, dH2, rows, PC_W, net.w + net.off[2], PC_W, dH1);
  hipLaunchKernelGGL(k_pc_relu_back, dim3(grid1(rows * PC_W)), dim3(256), 0, c.stream, net.Z1,
                     dH1, rows * PC_W);
  lin_wgrad(c, dH1, rows, PC_W, X, PC_IN, grad + net.off[0]);
  colsum(c, dH1, rows, PC_W, grad + net.off[1]);
  HIPC(hipGetLastError());
}

}  // namespace

namespace {
// initial weights from net.seed: He-scaled hidden layers and a small output
// layer, so that L starts near the identity and M near I; Adam state cleared
void upload_initial(Ctx &c) {
  PrecondNet &net = c.pc;
  std::vector<double> h(net.nparam, 0.0);
  HostNormal gauss{net.seed};
  const int64_t n0 = (int64_t)PC_W * PC_IN, n2 = (int64_t)PC_W * PC_W, n4 = (int64_t)PC_OUT * PC_W;
  for (int64_t i = 0; i < n0; ++i) h[net.off[0] + i] = gauss() * std::sqrt(2.0 / PC_IN);
  for (int64_t i = 0; i < n2; ++i) h[net.off[2] + i] = gauss() * std::sqrt(2.0 / PC_W);
  for (int64_t i = 0; i < n4; ++i) h[net.off[4] + i] = gauss() * 1e-3;
  HIPC(hipMemcpy(net.w, h.data(), net.nparam * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemset(net.g, 0, net.nparam * sizeof(double)));
  HIPC(hipMemset(net.m, 0, net.nparam * sizeof(double)));
  HIPC(hipMemset(net.v, 0, net.nparam * sizeof(double)));
  HIPC(hipMemset(net.loss_dev, 0, sizeof(double)));
  net.steps = 0;
  net.probe_ctr = 0;
  net.first_loss = net.last_loss = -1.0;
}
}  // namespace

void pc_init(Ctx &c) {
  PrecondNet &net = c.pc;
  if (net.ready) return;
  const int64_t sizes[6] = {(int64_t)PC_W * PC_IN, PC_W, (int64_t)PC_W * PC_W, PC_W,
                            (int64_t)PC_OUT * PC_W, PC_OUT};
  int64_t tot = 0;
  for (int k = 0; k < 6; ++k) {
    net.off[k] = tot;
    tot += sizes[k];
  }
  if (tot != net.param_count()) fail(QTT_E_ARG, "preconditioner parameter layout");
  net.nparam = tot;
  net.w = c.alloc_owned(tot);
  net.g = c.alloc_owned(tot);
  net.m = c.alloc_owned(tot);
  net.v = c.alloc_owned(tot);
  net.loss_dev = c.alloc_owned(1);
  upload_initial(c);
  net.ready = true;
}

void pc_reset(Ctx &c, uint64_t seed) {
  c.pc.seed = seed;
  if (!c.pc.ready) pc_init(c);
  else upload_initial(c);
}

void pc_features(Ctx &c, const double *Lenv, const double *Renv, const Mpo &Wii, int d, int la,
                 int ra, double mu_h2, double pen_scale, int n, int comp, double *X,
                 double *Bblk) {
  const int mi = Wii.bond[d], mo = Wii.bond[d + 1];
  const int64_t npos = (int64_t)la * ra;
  c.check_range(Lenv, 0, (int64_t)la * mi * la - 1, 8, "pc Lenv");
  c.check_range(Renv, 0, (int64_t)ra * mo * ra - 1, 8, "pc Renv");
  c.check_range(Wii.fwd + Wii.off(d), 0, (int64_t)mi * 16 * mo - 1, 8, "pc W");
  c.check_range(X, 0, npos * PC_IN - 1, 8, "pc X");
  c.check_range(Bblk, 0, npos * 16 - 1, 8, "pc B");
  const double f_site = (double)d / std::max(1, n - 1);
  const double f_pen = std::log10(std::max(pen_scale, 1e-30)) / 3.0;
  hipLaunchKernelGGL(k_pc_features, dim3(grid1(npos)), dim3(256), 0, c.stream, Lenv, Renv,
                     Wii.fwd + Wii.off(d), la, ra, mi, mo, mu_h2, f_site, f_pen, (double)comp,
                     std::log2((double)la) / 8.0, std::log2((double)ra) / 8.0, X, Bblk);
  HIPC(hipGetLastError());
}

void pc_forward(Ctx &c, const double *X, int64_t npos, double *M, bool keep) {
  PrecondNet &net = c.pc;
  if (!net.ready) fail(QTT_E_ARG, "preconditioner network not initialised");
  if (npos <= 0) return;
  act_buffers(c, npos);
  c.check_range(X, 0, npos * PC_IN - 1, 8, "pc forward X");
  c.check_range(M, 0, npos * 16 - 1, 8, "pc forward M");
  lin_fwd(c, X, npos, PC_IN, net.w + net.off[0], PC_W, net.Z1);
  hipLaunchKernelGGL(k_pc_bias_act, dim3(grid1(npos * PC_W)), dim3(256), 0, c.stream, net.Z1,
                     net.H1, net.w + net.off[1], npos, PC_W);
  lin_fwd(c, net.H1, npos, PC_W, net.w + net.off[2], PC_W, net.Z2);
  hipLaunchKernelGGL(k_pc_bias_act, dim3(grid1(npos * PC_W)), dim3(256), 0, c.stream, net.Z2,
                     net.H2, net.w + net.off[3], npos, PC_W);
  lin_fwd(c, net.H2, npos, PC_W, net.w + net.off[4], PC_OUT, net.Y);
  hipLaunchKernelGGL(k_pc_bias_act, dim3(grid1(npos * PC_OUT)), dim3(256), 0, c.stream, net.Y,
                     (double *)nullptr, net.w + net.off[5], npos, PC_OUT);
  hipLaunchKernelGGL(k_pc_factor, dim3(grid1(npos)), dim3(256), 0, c.stream, net.Y, M,
                     keep ? net.Lf : (double *)nullptr, npos);
  HIPC(hipGetLastError());
}

void pc_block_inverse(Ctx &c, const double *Bblk, double *M, int64_t npos) {
  if (npos <= 0) return;
  c.check_range(Bblk, 0, npos * 16 - 1, 8, "pc B");
  c.check_range(M, 0, npos * 16 - 1, 8, "pc M");
  hipLaunchKernelGGL(k_pc_block_inverse, dim3(grid1(npos)), dim3(256), 0, c.stream, Bblk, M,
                     npos);
  HIPC(hipGetLastError());
}

void pc_apply(Ctx &c, const double *M, const double *r, double *z, int la, int ra,
              const int *skip) {
  const int64_t npos = (int64_t)la * ra;
  if (npos <= 0) return;
  c.check_range(M, 0, npos * 16 - 1, 8, "pc apply M");
  c.check_range(r, 0, npos * 4 - 1, 8, "pc apply r");
  c.check_range(z, 0, npos * 4 - 1, 8, "pc apply z");
  hipLaunchKernelGGL(k_pc_apply, dim3(grid1(npos)), dim3(256), 0, c.stream, M, r, z, la, ra,
                     skip);
  HIPC(hipGetLastError());
}

void pc_probe(Ctx &c, double *z, int64_t n, uint64_t seed) {
  c.check_range(z, 0, n - 1, 8, "pc probe");
  hipLaunchKernelGGL(k_pc_probe, dim3(grid1(n)), dim3(256), 0, c.stream, z, n, seed);
  HIPC(hipGetLastError());
}

void pc_loss_grad(Ctx &c, const double *M, int64_t row0, const double *z, const double *Az,
                  int la, int ra, const double *zz) {
  PrecondNet &net = c.pc;
  const int64_t npos = (int64_t)la * ra;
  if (npos <= 0) return;
  if (row0 < 0 || row0 + npos > net.act_rows) fail(QTT_E_ARG, "pc loss: rows outside activations");
  c.check_range(M, row0 * 16, (row0 + npos) * 16 - 1, 8, "pc loss M");
  c.check_range(z, 0, npos * 4 - 1, 8, "pc loss z");
  c.check_range(Az, 0, npos * 4 - 1, 8, "pc loss Az");
  c.check_range(zz, 0, 0, 8, "pc loss zz");
  hipLaunchKernelGGL(k_pc_loss_grad, dim3(grid1(npos)), dim3(256), 0, c.stream, M + row0 * 16,
                     net.Lf + row0 * 16, z, Az, la, ra, zz, net.dY + row0 * PC_OUT, net.loss_dev);
  HIPC(hipGetLastError());
}

void pc_backward_adam(Ctx &c, const double *X, int64_t npos) {
  PrecondNet &net = c.pc;
  if (npos != net.act_rows) fail(QTT_E_ARG, "pc backward: rows differ from the forward pass");
  backward(c, X, npos, net.dY, net.g);
  net.steps += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double bc1 = 1.0 - std::pow(b1, (double)net.steps);
  const double bc2 = 1.0 - std::pow(b2, (double)net.steps);
  hipLaunchKernelGGL(k_pc_adam, dim3(grid1(net.nparam)), dim3(256), 0, c.stream, net.w, net.g,
                     net.m, net.v, net.nparam, net.lr, b1, b2, bc1, bc2, 1e-8);
  HIPC(hipGetLastError());
}

void pc_net_grad(Ctx &c, const double *X, int64_t npos, const double *dY, double *Y,
                 double *grad) {
  PrecondNet &net = c.pc;
  if (!net.ready) fail(QTT_E_ARG, "preconditioner network not initialised");
  if (npos <= 0) fail(QTT_E_ARG, "pc grad: npos < 1");
  double *M = c.buf("pc_Mgrad", npos * 16);
  pc_forward(c, X, npos, M, true);
  c.check_range(Y, 0, npos * PC_OUT - 1, 8, "pc grad Y");
  c.check_range(dY, 0, npos * PC_OUT - 1, 8, "pc grad dY");
  c.check_range(grad, 0, net.nparam - 1, 8, "pc grad out");
  HIPC(hipMemcpyAsync(Y, net.Y, npos * PC_OUT * sizeof(double), hipMemcpyDeviceToDevice,
                      c.stream));
  backward(c, X, npos, dY, grad);
}

}  // namespace qtt
