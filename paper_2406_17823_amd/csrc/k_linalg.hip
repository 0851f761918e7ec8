// Small dense float64 factorisations of the MPS algebra, one workgroup per
// matrix, several matrices per launch (the two velocity components, several
// flows).
//
//  * Householder QR with explicit Q and a non-negative diagonal of R: the
//    centre shifts of the sweep and the left-to-right pass of TT-rounding.
//  (the SVD of the right-to-left pass of TT-rounding is in k_svd.hip)
//
// The working matrix lives column-major in a workspace slice in HBM/L2 so
// that a wave64 reads one column with unit stride; reductions along a column
// are wave-level (DPP/shuffle), the Householder vector is staged in LDS.
#include "qtt_internal.h"

namespace qtt {

namespace {

constexpr int LA_THREADS = 1024;
constexpr int LA_WAVES = LA_THREADS / 64;
constexpr int MAX_BATCH = 8;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct QRDesc {
  const double *A;
  int m, n;
  int64_t ars, acs;
  double *Q;
  int64_t qrs, qcs;
  double *R;
  int64_t rrs, rcs;
  double *W;  // m*n + m*k doubles of workspace
};
struct QRBatch {
  int count;
  QRDesc d[MAX_BATCH];
};

// dynamic LDS: v[m], tau[k], 2 scalars
__global__ __launch_bounds__(LA_THREADS) void k_qr(QRBatch batch) {
  extern __shared__ double lds[];
  QRDesc D = batch.d[blockIdx.x];
  const int m = D.m, n = D.n, k = min(m, n);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *v = lds;
  double *tau = lds + m;
  double *scal = tau + k;
  double *W = D.W;               // column-major m x n
  double *Qw = D.W + (int64_t)m * n;  // column-major m x k

  for (int64_t idx = tid; idx < (int64_t)m * n; idx += LA_THREADS) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    W[idx] = D.A[i * D.ars + j * D.acs];
  }
  __syncthreads();

  for (int j = 0; j < k; ++j) {
    double *wj = W + (int64_t)j * m;
    if (wave == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) s += wj[i] * wj[i];
      s = wave_sum(s);
      if (lane == 0) scal[0] = s;
    }
    __syncthreads();
    const double xnorm2 = scal[0];
    const double alpha = wj[j];
    double t = 0.0, beta = alpha, sc = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    for (int i = j + tid; i < m; i += LA_THREADS) v[i] = (i == j) ? 1.0 : wj[i] * sc;
    __syncthreads();
    // apply H_j = I - t v v^T to the trailing columns, one wave per column
    if (t != 0.0) {
      for (int cidx = j + 1 + wave; cidx < n; cidx += LA_WAVES) {
        double *wc = W + (int64_t)cidx * m;
        double s = 0.0;
        for (int i = j + lane; i < m; i += 64) s += v[i] * wc[i];
        s = wave_sum(s) * t;
        for (int i = j + lane; i < m; i += 64) wc[i] -= s * v[i];
      }
    }
    __syncthreads();
    // store R_jj and the reflector below the diagonal
    for (int i = j + tid; i < m; i += LA_THREADS) wj[i] = (i == j) ? beta : v[i];
    if (tid == 0) tau[j] = t;
    __syncthreads();
  }

  // Q = H_0 ... H_{k-1} [I_k; 0], accumulated backwards
  for (int64_t idx = tid; idx < (int64_t)m * k; idx += LA_THREADS) {
    const int i = (int)(idx % m), c = (int)(idx / m);
    Qw[idx] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double *wj = W + (int64_t)j * m;
    for (int i = j + tid; i < m; i += LA_THREADS) v[i] = (i == j) ? 1.0 : wj[i];
    __syncthreads();
    const double t = tau[j];
    if (t != 0.0) {
      for (int cidx = j + wave; cidx < k; cidx += LA_WAVES) {
        double *qc = Qw + (int64_t)cidx * m;
        double s = 0.0;
        for (int i = j + lane; i < m; i += 64) s += v[i] * qc[i];
        s = wave_sum(s) * t;
        for (int i = j + lane; i < m; i += 64) qc[i] -= s * v[i];
      }
    }
    __syncthreads();
  }

  // sign convention: diag(R) >= 0
  for (int64_t idx = tid; idx < (int64_t)m * k; idx += LA_THREADS) {
    const int i = (int)(idx % m), c = (int)(idx / m);
    const double s = (W[(int64_t)c * m + c] < 0.0) ? -1.0 : 1.0;
    D.Q[i * D.qrs + c * D.qcs] = s * Qw[idx];
  }
  for (int64_t idx = tid; idx < (int64_t)k * n; idx += LA_THREADS) {
    const int r = (int)(idx % k), c = (int)(idx / k);
    const double s = (W[(int64_t)r * m + r] < 0.0) ? -1.0 : 1.0;
    D.R[r * D.rrs + c * D.rcs] = (c >= r) ? s * W[(int64_t)c * m + r] : 0.0;
  }
}

}  // namespace

void qr_batch(Ctx &c, int count, const ConstMatView *A, const MatView *Q, const MatView *R) {
  for (int base = 0; base < count; base += MAX_BATCH) {
    const int cnt = std::min(MAX_BATCH, count - base);
    QRBatch b{};
    b.count = cnt;
    int64_t ws = 0;
    int maxm = 0, maxk = 0;
    for (int i = 0; i < cnt; ++i) {
      const int m = A[base + i].rows, n = A[base + i].cols;
      if (Q[base + i].rows != m || Q[base + i].cols != std::min(m, n) ||
          R[base + i].rows != std::min(m, n) || R[base + i].cols != n)
        fail(QTT_E_SHAPE, "qr_batch: output shapes");
      ws += (int64_t)m * n + (int64_t)m * std::min(m, n);
      maxm = std::max(maxm, m);
      maxk = std::max(maxk, std::min(m, n));
    }
    double *W = c.buf("qr_work", ws);
    int64_t o = 0;
    for (int i = 0; i < cnt; ++i) {
      const ConstMatView &a = A[base + i];
      const MatView &q = Q[base + i];
      const MatView &r = R[base + i];
      {
        int64_t lo = 0, hi = 0;
        span(lo, hi, a.rows, a.rs);
        span(lo, hi, a.cols, a.cs);
        c.check_range(a.p, lo, hi, 8, "qr A");
        lo = hi = 0;
        span(lo, hi, q.rows, q.rs);
        span(lo, hi, q.cols, q.cs);
        c.check_range(q.p, lo, hi, 8, "qr Q");
        lo = hi = 0;
        span(lo, hi, r.rows, r.rs);
        span(lo, hi, r.cols, r.cs);
        c.check_range(r.p, lo, hi, 8, "qr R");
      }
      b.d[i] = QRDesc{a.p, a.rows, a.cols, a.rs, a.cs, q.p, q.rs, q.cs, r.p, r.rs, r.cs, W + o};
      o += (int64_t)a.rows * a.cols + (int64_t)a.rows * std::min(a.rows, a.cols);
    }
    const size_t lds = sizeof(double) * (maxm + maxk + 2);
    if (lds > 160 * 1024) fail(QTT_E_UNSUPPORTED, "qr_batch: matrix too tall for LDS");
    hipLaunchKernelGGL(k_qr, dim3(cnt), dim3(LA_THREADS), lds, c.stream, b);
    HIPC(hipGetLastError());
  }
}

}  // namespace qtt
