// Small dense float64 factorisations of the MPS algebra, one workgroup per
// matrix, several matrices per launch (the two velocity components, several
// flows).
//
//  * Householder QR with explicit Q and a non-negative diagonal of R: the
//    centre shifts of the sweep and the left-to-right pass of TT-rounding.
//  * One-sided (Hestenes) Jacobi SVD with round-robin pair ordering and
//    singular values sorted in descending order: the right-to-left pass of
//    TT-rounding and the Gram eigen-decompositions of the input compression.
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

struct SVDDesc {
  const double *A;
  int m, n;
  int64_t ars, acs;
  double *U;
  int64_t urs, ucs;
  double *S;
  double *V;
  int64_t vrs, vcs;
  double *W;  // m*n + n*n doubles
};
struct SVDBatch {
  int count;
  SVDDesc d[MAX_BATCH];
};

// dynamic LDS: sigma[n], rank[n] (as double), counter
__global__ __launch_bounds__(LA_THREADS) void k_svd(SVDBatch batch) {
  extern __shared__ double lds[];
  SVDDesc D = batch.d[blockIdx.x];
  const int m = D.m, n = D.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *W = D.W;                        // m x n column-major
  double *Vw = D.W + (int64_t)m * n;      // n x n column-major
  double *sig = lds;
  int *rank = (int *)(lds + n);
  int *counter = rank + n + 1;

  for (int64_t idx = tid; idx < (int64_t)m * n; idx += LA_THREADS) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    W[idx] = D.A[i * D.ars + j * D.acs];
  }
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += LA_THREADS) {
    const int i = (int)(idx % n), j = (int)(idx / n);
    Vw[idx] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) *counter = 0;
  __syncthreads();

  const int np = n + (n & 1);   // even number of players; index n is a dummy
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 60 && np > 1; ++sweep) {
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      for (int pr = wave; pr < np / 2; pr += LA_WAVES) {
        int p, q;
        if (pr == 0) {
          p = np - 1;
          q = rnd;
        } else {
          p = (rnd + pr) % (np - 1);
          q = (rnd - pr + np - 1) % (np - 1);
        }
        if (p >= n || q >= n) continue;
        double *wp = W + (int64_t)p * m;
        double *wq = W + (int64_t)q * m;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < m; i += 64) {
          const double x = wp[i], y = wq[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
          for (int i = lane; i < m; i += 64) {
            const double x = wp[i], y = wq[i];
            wp[i] = cs * x - sn * y;
            wq[i] = sn * x + cs * y;
          }
          double *vp = Vw + (int64_t)p * n;
          double *vq = Vw + (int64_t)q * n;
          for (int i = lane; i < n; i += 64) {
            const double x = vp[i], y = vq[i];
            vp[i] = cs * x - sn * y;
            vq[i] = sn * x + cs * y;
          }
          if (lane == 0) atomicAdd(counter, 1);
        }
      }
      __syncthreads();
    }
    const int rot = *counter;
    __syncthreads();
    if (tid == 0) *counter = 0;
    __syncthreads();
    if (rot == 0) break;
  }

  // singular values = column norms, ranked in descending order (ties by index)
  for (int j = wave; j < n; j += LA_WAVES) {
    const double *wj = W + (int64_t)j * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += wj[i] * wj[i];
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < n; j += LA_THREADS) {
    const double sj = sig[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig[i];
      r += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
    rank[j] = r;
  }
  __syncthreads();
  for (int j = tid; j < n; j += LA_THREADS) D.S[rank[j]] = sig[j];
  for (int64_t idx = tid; idx < (int64_t)m * n; idx += LA_THREADS) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    const double s = sig[j];
    D.U[i * D.urs + rank[j] * D.ucs] = (s > 0.0) ? W[idx] / s : 0.0;
  }
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += LA_THREADS) {
    const int i = (int)(idx % n), j = (int)(idx / n);
    D.V[i * D.vrs + rank[j] * D.vcs] = Vw[idx];
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

void svd_batch(Ctx &c, int count, const ConstMatView *A, const MatView *U, double *const *S,
               const MatView *V) {
  for (int base = 0; base < count; base += MAX_BATCH) {
    const int cnt = std::min(MAX_BATCH, count - base);
    SVDBatch b{};
    b.count = cnt;
    int64_t ws = 0;
    int maxn = 0;
    for (int i = 0; i < cnt; ++i) {
      const int m = A[base + i].rows, n = A[base + i].cols;
      if (m < n) fail(QTT_E_SHAPE, "svd_batch: needs rows >= cols");
      if (U[base + i].rows != m || U[base + i].cols != n || V[base + i].rows != n ||
          V[base + i].cols != n)
        fail(QTT_E_SHAPE, "svd_batch: output shapes");
      ws += (int64_t)m * n + (int64_t)n * n;
      maxn = std::max(maxn, n);
    }
    double *W = c.buf("svd_work", ws);
    int64_t o = 0;
    for (int i = 0; i < cnt; ++i) {
      const ConstMatView &a = A[base + i];
      {
        int64_t lo = 0, hi = 0;
        span(lo, hi, a.rows, a.rs);
        span(lo, hi, a.cols, a.cs);
        c.check_range(a.p, lo, hi, 8, "svd A");
        lo = hi = 0;
        span(lo, hi, U[base + i].rows, U[base + i].rs);
        span(lo, hi, U[base + i].cols, U[base + i].cs);
        c.check_range(U[base + i].p, lo, hi, 8, "svd U");
        lo = hi = 0;
        span(lo, hi, V[base + i].rows, V[base + i].rs);
        span(lo, hi, V[base + i].cols, V[base + i].cs);
        c.check_range(V[base + i].p, lo, hi, 8, "svd V");
        c.check_range(S[base + i], 0, a.cols - 1, 8, "svd S");
      }
      b.d[i] = SVDDesc{a.p, a.rows, a.cols, a.rs, a.cs, U[base + i].p, U[base + i].rs,
                       U[base + i].cs, S[base + i], V[base + i].p, V[base + i].rs,
                       V[base + i].cs, W + o};
      o += (int64_t)a.rows * a.cols + (int64_t)a.cols * a.cols;
    }
    const size_t lds = sizeof(double) * (2 * maxn + 4);
    hipLaunchKernelGGL(k_svd, dim3(cnt), dim3(LA_THREADS), lds, c.stream, b);
    HIPC(hipGetLastError());
  }
}

}  // namespace qtt
