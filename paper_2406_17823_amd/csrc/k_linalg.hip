// Small dense float64 factorisations of the MPS algebra, one workgroup per
// matrix, several matrices per launch (the two velocity components, several
// flows).
//
//  * Householder QR with explicit Q and a non-negative diagonal of R: the
//    centre shifts of the sweep and the left-to-right pass of TT-rounding.
//    Small matrices take one workgroup each; larger ones (up to the
//    2048 x 512 unfoldings of a four-term RK4 sum at chi = 128) use the blocked
//    form: a panel of QR_NB columns is factorised by one workgroup per
//    matrix, its reflectors are aggregated into I - V T V^T (compact WY), and
//    the trailing columns and the explicit Q are updated by a block-reflector
//    kernel on float64 MFMAs (one workgroup per 32-column tile).
//  (the SVD of the right-to-left pass of TT-rounding is in k_svd.hip)
//
// The working matrix lives column-major in a workspace slice in HBM/L2 so
// that a wave64 reads one column with unit stride; reductions along a column
// are wave-level (DPP/shuffle), the Householder vector is staged in LDS.
#include <mutex>
#include <utility>

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

// ---------------------------------------------------------------- blocked QR
constexpr int QR_NB = 16;
constexpr int QR_REG_MAXROWS = 4;  // rows per thread of the register-resident panel, at most

typedef double d4v __attribute__((ext_vector_type(4)));

struct QrbDesc {
  const double *A;
  int64_t ars, acs;
  double *W;    // m x n column-major working matrix (R above, reflectors below)
  double *V;    // m x k column-major: reflector c in column c (1 at row c, 0 above)
  double *VT;   // m x k: panel p's columns hold V_p T_p
  double *VTt;  // m x k: panel p's columns hold V_p T_p^T
  double *Qw;   // m x k column-major explicit Q (before the sign fix)
  double *T;    // QR_NB x QR_NB: the current panel's T (upper triangular)
  double *Q;
  int64_t qrs, qcs;
  double *R;
  int64_t rrs, rcs;
  int m, n, k;
};
struct QrbBatch {
  int count;
  QrbDesc d[MAX_BATCH];
};

__global__ void k_qrb_load(QrbBatch B) {
  const QrbDesc &D = B.d[blockIdx.y];
  const int64_t tot = (int64_t)D.m * D.n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % D.m), j = (int)(idx / D.m);
    D.W[idx] = D.A[i * D.ars + j * D.acs];
  }
  const int64_t tq = (int64_t)D.m * D.k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tq;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % D.m), j = (int)(idx / D.m);
    D.Qw[idx] = (i == j) ? 1.0 : 0.0;
  }
}

// sum of nv per-thread values over the workgroup; result in red[0..nv)
// (valid after return in every thread)
__device__ inline void block_sum_vec(const double (&vals)[QR_NB], int nv,
                                     double (*sh)[QR_NB + 1], double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < QR_NB; ++t) {
    if (t < nv) {
      const double s = wave_sum(vals[t]);
      if (lane == 0) sh[wave][t] = s;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
    for (int w = 0; w < LA_WAVES; ++w) s += sh[w][threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();
}

// factorise columns [j0, j0 + jb) of each matrix (rows j0..m); every thread
// owns the rows r = tid + LA_THREADS * s throughout, so reflector entries
// are produced and consumed by the same thread
__global__ __launch_bounds__(LA_THREADS) void k_qrb_panel(QrbBatch B, int j0) {
  const QrbDesc &D = B.d[blockIdx.x];
  const int m = D.m, k = D.k;
  const int jb = min(QR_NB, k - j0);
  if (jb <= 0) return;
  const int tid = threadIdx.x;
  __shared__ double sh[LA_WAVES][QR_NB + 1];
  __shared__ double red[QR_NB + 1];
  __shared__ double T[QR_NB][QR_NB + 1];
  double *W = D.W, *V = D.V;
  for (int i = 0; i < jb; ++i) {
    const int c = j0 + i;
    double *wc = W + (int64_t)c * m;
    double part = 0.0;
    for (int r = tid; r < m; r += LA_THREADS)
      if (r > c) part += wc[r] * wc[r];
    part = wave_sum(part);
    if ((tid & 63) == 0) sh[tid >> 6][0] = part;
    __syncthreads();
    if (tid == 0) {
      double s2 = 0.0;
      for (int w = 0; w < LA_WAVES; ++w) s2 += sh[w][0];
      red[QR_NB] = s2;
    }
    __syncthreads();
    const double xnorm2 = red[QR_NB];
    const double alpha = wc[c];
    double tau = 0.0, beta = alpha, sc = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha before row c is overwritten
    // reflector: column c of V (zeros on rows j0..c-1), below-diagonal part of W
    double d[QR_NB];
#pragma unroll
    for (int t = 0; t < QR_NB; ++t) d[t] = 0.0;
    for (int r = tid; r < m; r += LA_THREADS) {
      if (r < j0) continue;
      double v = 0.0;
      if (r == c) {
        v = 1.0;
        wc[r] = beta;
      } else if (r > c) {
        v = wc[r] * sc;
        wc[r] = v;
      }
      V[(int64_t)c * m + r] = v;
      if (r >= c) {
#pragma unroll
        for (int t = 0; t < QR_NB; ++t)
          if (t < jb && t != i) d[t] += v * W[(int64_t)(j0 + t) * m + r];
      }
    }
    block_sum_vec(d, jb, sh, red);
    // H_c on the panel's trailing columns
    for (int r = tid; r < m; r += LA_THREADS) {
      if (r < c) continue;
      const double v = V[(int64_t)c * m + r];
      for (int t = i + 1; t < jb; ++t) W[(int64_t)(j0 + t) * m + r] -= tau * red[t] * v;
    }
    // T[0:i, i] = -tau T[0:i, 0:i] (V_{0:i}^T v_c), T[i][i] = tau
    if (tid < i) {
      double s = 0.0;
      for (int u = tid; u < i; ++u) s += T[tid][u] * red[u];
      T[tid][i] = -tau * s;
    }
    if (tid == 0) T[i][i] = tau;
    __syncthreads();
  }
  // T_p for the aggregation kernel
  for (int e = tid; e < QR_NB * QR_NB; e += LA_THREADS) {
    const int t = e / QR_NB, u = e % QR_NB;
    D.T[e] = (t < jb && u < jb && u >= t) ? T[t][u] : 0.0;
  }
}

// sum over the 64 lanes of a wave of 16 values at once: four butterfly
// steps halve the values each lane holds (17 exchanges instead of 16 x 6);
// on return lane l holds the total of value (l >> 2) & 15
__device__ inline double wave_sum16(const double (&v)[16], int lane) {
  double a[8], b[4], c[2];
  const bool h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1, h3 = (lane >> 3) & 1, h2 = (lane >> 2) & 1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double keep = h5 ? v[j + 8] : v[j], send = h5 ? v[j] : v[j + 8];
    a[j] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double keep = h4 ? a[j + 4] : a[j], send = h4 ? a[j] : a[j + 4];
    b[j] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double keep = h3 ? b[j + 2] : b[j], send = h3 ? b[j] : b[j + 2];
    c[j] = keep + __shfl_xor(send, 8, 64);
  }
  double d = (h2 ? c[1] : c[0]) + __shfl_xor(h2 ? c[0] : c[1], 4, 64);
  d += __shfl_xor(d, 2, 64);
  d += __shfl_xor(d, 1, 64);
  return d;
}

// register-resident panel for m <= ROWS * 64 NW: thread tid holds
// rows r = tid + 64 NW s of the panel's columns, so a column step touches
// HBM/L2 not at all.  One reduction per column: with x the entries of
// column i below row c = j0 + i, the sums S[t] = sum_{r > c} x_r P[r][t]
// over all 16 panel columns give |x|^2 (t = i), the products of the new
// reflector v = (1, x / (alpha - beta)) with the trailing columns
// (P[c][t] + S[t] / (alpha - beta), t > i) and with the earlier reflectors
// (the same expression, t < i, for the next column of T); row c itself is
// published through LDS by its owner.  Two barriers per column; the LDS
// words read after the second are double-buffered by column parity.
// Register columns are selected with compile-time indices and a predicate,
// never indexed by i.
// (ROWS = 1, 2 or 4 with 8 waves: the per-thread work of a column step
// scales with ROWS, so the panel of a short matrix spreads over the waves)
// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): a loop
// whose index is a compile-time constant in every step (the unroller does not
// take loops with barriers and a run-time exit)
template <typename F, int... Is>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

template <int NW, int ROWS>
__device__ void qrb_panel_reg(const QrbDesc &D, int j0) {
  constexpr int NT = 64 * NW;
  const int m = D.m, k = D.k;
  const int jb = min(QR_NB, k - j0);
  if (jb <= 0 || m > ROWS * NT) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double sh[NW][QR_NB];
  __shared__ double red[2][QR_NB];
  __shared__ double rowc[2][QR_NB];
  __shared__ double T[QR_NB][QR_NB + 1];
  __shared__ double Y[QR_NB][QR_NB + 1];  // Y[u][i] = v_u . v_i, u < i
  __shared__ double taus[QR_NB];
  double P[ROWS][QR_NB];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = tid + NT * s;
#pragma unroll
    for (int t = 0; t < QR_NB; ++t)
      P[s][t] = (r >= j0 && r < m && t < jb) ? D.W[(int64_t)(j0 + t) * m + r] : 0.0;
  }
  // one column step; with one row per thread the steps are expanded with a
  // compile-time column index, so the register columns are selected directly
  // (more rows per thread would spill so expanded); jb < 16 only for a
  // matrix's last panel
  auto column_step = [&](auto I_) __attribute__((always_inline)) {
    const int i = I_;
    if (i >= jb) return;
    const int c = j0 + i, bf = i & 1;
    double pc[ROWS];
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      pc[s] = 0.0;
#pragma unroll
      for (int t = 0; t < QR_NB; ++t)
        if (t == i) pc[s] = P[s][t];
    }
    double d[QR_NB];
#pragma unroll
    for (int t = 0; t < QR_NB; ++t) d[t] = 0.0;
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int r = tid + NT * s;
      if (r > c && r < m) {
#pragma unroll
        for (int t = 0; t < QR_NB; ++t) d[t] += pc[s] * P[s][t];
      }
      if (r == c) {
#pragma unroll
        for (int t = 0; t < QR_NB; ++t) rowc[bf][t] = P[s][t];
      }
    }
    static_assert(QR_NB == 16, "wave_sum16 reduces 16 columns");
    {
      const double sum = wave_sum16(d, lane);
      if ((lane & 3) == 0) sh[wave][lane >> 2] = sum;
    }
    __syncthreads();
    if (tid < QR_NB) {
      double s2 = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s2 += sh[w][tid];
      red[bf][tid] = s2;
    }
    __syncthreads();
    const double xnorm2 = red[bf][i];
    const double alpha = rowc[bf][i];
    double tau = 0.0, beta = alpha, sc = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    // tau (v^T column t) for the trailing columns
    double w[QR_NB];
#pragma unroll
    for (int t = 0; t < QR_NB; ++t) w[t] = tau * (rowc[bf][t] + sc * red[bf][t]);
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int r = tid + NT * s;
      if (r < c || r >= m) continue;
      const double v = (r == c) ? 1.0 : pc[s] * sc;
#pragma unroll
      for (int t = 0; t < QR_NB; ++t) {
        if (t == i) P[s][t] = (r == c) ? beta : v;
        else if (t > i && t < jb) P[s][t] -= w[t] * v;
      }
    }
    // the products of the earlier reflectors with this one and tau, for T
    if (tid < i) Y[tid][i] = rowc[bf][tid] + sc * red[bf][tid];
    if (tid == 0) taus[i] = tau;
  };
  if constexpr (ROWS == 1) {
    static_for<QR_NB>(column_step);
  } else {
    for (int i = 0; i < jb; ++i) column_step(i);
  }
  __syncthreads();
  // T (upper triangular) after the column loop, off its critical path:
  // T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] Y[0:i, i]; row t of T
  // depends only on row t, so thread t forms it alone, in registers
  if (tid < QR_NB) {
    double Tr[QR_NB];
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) {
      double val = 0.0;
      if (i < jb) {
        if (i == tid) {
          val = taus[i];
        } else if (i > tid) {
          double s2 = 0.0;
#pragma unroll
          for (int u = 0; u < i; ++u)
            if (u >= tid) s2 += Tr[u] * Y[u][i];
          val = -taus[i] * s2;
        }
      }
      Tr[i] = val;
    }
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) T[tid][i] = Tr[i];
  }
  __syncthreads();
  // write back: W panel (R entries and reflectors), V (unit diagonal, zeros
  // above), V T and V T^T of the thread's rows (T upper triangular, read
  // from LDS on and above its diagonal only), T
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = tid + NT * s;
    if (r < j0 || r >= m) continue;
    double v[QR_NB];
#pragma unroll
    for (int t = 0; t < QR_NB; ++t) {
      const int c = j0 + t;
      v[t] = (t >= jb || r < c) ? 0.0 : (r == c ? 1.0 : P[s][t]);
      if (t < jb) {
        D.W[(int64_t)c * m + r] = P[s][t];
        D.V[(int64_t)c * m + r] = v[t];
      }
    }
#pragma unroll
    for (int t = 0; t < QR_NB; ++t) {
      if (t >= jb) continue;
      double a = 0.0, bt = 0.0;
#pragma unroll
      for (int u = 0; u < QR_NB; ++u) {
        if (u <= t) a += v[u] * T[u][t];
        if (u >= t && u < jb) bt += v[u] * T[t][u];
      }
      D.VT[(int64_t)(j0 + t) * m + r] = a;
      D.VTt[(int64_t)(j0 + t) * m + r] = bt;
    }
  }
  for (int e = tid; e < QR_NB * QR_NB; e += NT) {
    const int t = e / QR_NB, u = e % QR_NB;
    D.T[e] = (t < jb && u < jb && u >= t) ? T[t][u] : 0.0;
  }
}

template <int NW, int ROWS>
__global__ __launch_bounds__(64 * NW) void k_qrb_panel_reg(QrbBatch B, int j0) {
  qrb_panel_reg<NW, ROWS>(B.d[blockIdx.x], j0);
}

// VT = V_p T_p and VTt = V_p T_p^T on rows j0..m (one thread per row and column)
__global__ void k_qrb_vt(QrbBatch B, int j0) {
  const QrbDesc &D = B.d[blockIdx.y];
  const int m = D.m;
  const int jb = min(QR_NB, D.k - j0);
  if (jb <= 0) return;
  const int64_t tot = (int64_t)(m - j0) * jb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = j0 + (int)(e % (m - j0)), t = (int)(e / (m - j0));
    double a = 0.0, b = 0.0;
    for (int s = 0; s < jb; ++s) {
      const double v = D.V[(int64_t)(j0 + s) * m + r];
      if (s <= t) a += v * D.T[s * QR_NB + t];
      if (s >= t) b += v * D.T[t * QR_NB + s];
    }
    D.VT[(int64_t)(j0 + t) * m + r] = a;
    D.VTt[(int64_t)(j0 + t) * m + r] = b;
  }
}

// Block reflector applied to one 32-column tile X[j0:m, c0:c0+32) of one
// matrix: X -= U (V_p^T X), with U = V_p T_p^T for the trailing columns of
// the working matrix (which = 0) and U = V_p T_p for the explicit Q (which =
// 1).  Both products run on float64 MFMAs inside one 8-wave workgroup: Z =
// V_p^T X (16 x 32) with the rows dealt to the waves and the partials summed
// in wave order through LDS, then X^T -= Z^T U^T on 16-row tiles (lanes along
// rows, so X is read and written in 128-byte column segments), the loads of
// a batch of tiles issued before their MFMAs.  One launch per panel replaces
// two GEMMs, a split-K reduction and their launch gaps.
constexpr int QA_COLS = 32, QA_THREADS = 512, QA_WAVES = QA_THREADS / 64, QA_BATCH = 4;

// X[j0:m, c0:c0+nc) -= U (V_p^T X) for one 32-column tile (see above)
__device__ void qrb_apply_tile(const QrbDesc &D, int j0, int jb, double *X, const double *U,
                               int c0, int nc, double (*Zs)[QR_NB][QA_COLS + 1]) {
  const int m = D.m;
  const int R = m - j0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // Z = V_p^T X: A[t][k] = V[j0 + k][j0 + t], B[k][c] = X[j0 + k][c0 + c]
  d4v z[2] = {d4v{0.0, 0.0, 0.0, 0.0}, d4v{0.0, 0.0, 0.0, 0.0}};
#pragma unroll 8
  for (int k0 = 4 * wave; k0 < R; k0 += 4 * QA_WAVES) {
    const int kr = k0 + lk;
    const int64_t r = j0 + kr;
    const bool rv = kr < R;
    const double a = (rv && li < jb) ? D.V[(int64_t)(j0 + li) * m + r] : 0.0;
    const double b0 = (rv && li < nc) ? X[(int64_t)(c0 + li) * m + r] : 0.0;
    const double b1 = (rv && 16 + li < nc) ? X[(int64_t)(c0 + 16 + li) * m + r] : 0.0;
    z[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, z[0], 0, 0, 0);
    if (nc > 16) z[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, z[1], 0, 0, 0);
  }
  // D register q: row 4 q + lane / 16, column lane % 16
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) Zs[wave][4 * q + lk][16 * h + li] = z[h][q];
  __syncthreads();
  for (int e = threadIdx.x; e < QR_NB * QA_COLS; e += QA_THREADS) {
    const int t = e / QA_COLS, cc = e % QA_COLS;
    double sum = Zs[0][t][cc];
#pragma unroll
    for (int w = 1; w < QA_WAVES; ++w) sum += Zs[w][t][cc];
    Zs[0][t][cc] = sum;
  }
  __syncthreads();
  // X^T[c][r] -= sum_t Z[t][c] U[r][t]: A[c][t] = Z[t][c] (LDS), B[t][r] = U[r][t]
  const int ntiles = ((R + 15) / 16) * 2;
  for (int base = wave; base < ntiles; base += QA_WAVES * QA_BATCH) {
    double ub[QA_BATCH][4], xo[QA_BATCH][4];
#pragma unroll
    for (int j = 0; j < QA_BATCH; ++j) {
      const int task = base + j * QA_WAVES;
      const int rt = task >> 1, h = task & 1;
      const int r = j0 + 16 * rt + li;
      const bool ok = task < ntiles && 16 * h < nc && r < m;
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0) {
        const int t = 4 * t0 + lk;
        ub[j][t0] = (ok && t < jb) ? U[(int64_t)(j0 + t) * m + r] : 0.0;
        const int cc = 16 * h + 4 * t0 + lk;
        xo[j][t0] = (ok && cc < nc) ? X[(int64_t)(c0 + cc) * m + r] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < QA_BATCH; ++j) {
      const int task = base + j * QA_WAVES;
      const int rt = task >> 1, h = task & 1;
      const int r = j0 + 16 * rt + li;
      // wave-uniform skip: every lane takes part in the MFMAs (rows past m
      // carry zeros and are not stored)
      if (!(task < ntiles && 16 * h < nc)) continue;
      d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Zs[0][4 * t0 + lk][16 * h + li], ub[j][t0], acc,
                                                   0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = 16 * h + 4 * q + lk;
        if (r < m && cc < nc) X[(int64_t)(c0 + cc) * m + r] = xo[j][q] - acc[q];
      }
    }
  }
}

__global__ __launch_bounds__(QA_THREADS) void k_qrb_apply(QrbBatch B, int j0, int which) {
  const QrbDesc &D = B.d[blockIdx.y];
  const int jb = min(QR_NB, D.k - j0);
  if (jb <= 0) return;
  double *X;
  const double *U;
  int cbeg, cend;
  if (which == 0) {
    X = D.W;
    U = D.VTt;
    cbeg = j0 + jb;
    cend = D.n;
  } else {
    if (!D.Q) return;
    X = D.Qw;
    U = D.VT;
    cbeg = j0;
    cend = D.k;
  }
  const int c0 = cbeg + (int)blockIdx.x * QA_COLS;
  if (c0 >= cend) return;
  __shared__ double Zs[QA_WAVES][QR_NB][QA_COLS + 1];
  qrb_apply_tile(D, j0, jb, X, U, c0, min(QA_COLS, cend - c0), Zs);
}

// trailing update of panel j0 (as k_qrb_apply, which = 0) with look-ahead:
// workgroup 0 of each matrix owns the first 32 trailing columns, which hold
// the next panel, so once its tile is updated (its own writes, visible to
// the workgroup after the barrier) it factors that panel in the same launch
// while the other workgroups finish the trailing columns; one launch per
// panel instead of two.  The next panel's writes (its columns of W, V, VT,
// VTt and T) are disjoint from what the other workgroups read (panel j0's
// columns of V and VTt, their own columns of W).
template <int ROWS>
__global__ __launch_bounds__(QA_THREADS) void k_qrb_apply_la(QrbBatch B, int j0) {
  const QrbDesc &D = B.d[blockIdx.y];
  const int jb = min(QR_NB, D.k - j0);
  if (jb <= 0) return;
  const int cbeg = j0 + jb, cend = D.n;
  const int c0 = cbeg + (int)blockIdx.x * QA_COLS;
  if (c0 >= cend) return;
  __shared__ double Zs[QA_WAVES][QR_NB][QA_COLS + 1];
  qrb_apply_tile(D, j0, jb, D.W, D.VTt, c0, min(QA_COLS, cend - c0), Zs);
  if (blockIdx.x != 0 || j0 + QR_NB >= D.k) return;
  __syncthreads();
  qrb_panel_reg<QA_THREADS / 64, ROWS>(D, j0 + QR_NB);
}

// explicit Q = H_0 H_1 ... [I; 0] in one launch: the columns of Q are
// independent, so each workgroup takes its tile of FQ_COLS = 16 columns
// through every panel's block reflector, last panel first (a panel whose rows
// start at or right of the tile's last column leaves it unchanged and is
// skipped); narrower tiles than the trailing updates' put twice the
// workgroups on this chain of dependent panel steps.  The tile's own global
// writes are visible to the whole workgroup after the barrier; the arithmetic
// per column is that of one apply launch per panel.
constexpr int FQ_COLS = 16;
__global__ __launch_bounds__(QA_THREADS) void k_qrb_formq(QrbBatch B) {
  const QrbDesc &D = B.d[blockIdx.y];
  if (!D.Q) return;
  const int c0 = (int)blockIdx.x * FQ_COLS;
  if (c0 >= D.k) return;
  const int nc = min(FQ_COLS, D.k - c0);
  __shared__ double Zs[QA_WAVES][QR_NB][QA_COLS + 1];
  for (int j0 = ((D.k - 1) / QR_NB) * QR_NB; j0 >= 0; j0 -= QR_NB) {
    if (j0 >= c0 + nc) continue;
    // columns left of j0 are zero in rows j0.. (untouched by this panel)
    const int cs = max(c0, j0);
    qrb_apply_tile(D, j0, min(QR_NB, D.k - j0), D.Qw, D.VT, cs, c0 + nc - cs, Zs);
    __syncthreads();
  }
}

// explicit Q as k_qrb_formq, with the workgroup's tile of NCOL columns of Q
// resident in LDS from [I; 0] to the end (matrices of at most MAXM rows: 16
// columns up to 1024 rows, 8 up to 2048): a panel step reads its V_p and
// V_p T_p columns from HBM/L2 but the tile only from LDS, so the chain of
// panel steps no longer waits on the tile's own global stores and reloads.
// Columns left of a panel's first row are zero in that panel's rows, so they
// take part with Z = 0 and stay exactly unchanged.  Tile layout: row-major,
// leading dimension NCOL + 1.  With 8 columns the MFMAs' upper 8 columns
// carry zeros.
template <int NCOL, int MAXM>
__global__ __launch_bounds__(QA_THREADS) void k_qrb_formq_lds(QrbBatch B) {
  static_assert(NCOL == 16 || NCOL == 8, "tiles of 16 or 8 columns");
  constexpr int LD = NCOL + 1, NQ = NCOL / 4;
  // 16-row tiles of the update per wave, at most
  constexpr int TASKS = (MAXM / 16 + QA_WAVES - 1) / QA_WAVES;
  const QrbDesc &D = B.d[blockIdx.y];
  if (!D.Q) return;
  const int c0 = (int)blockIdx.x * NCOL;
  if (c0 >= D.k) return;
  const int nc = min(NCOL, D.k - c0), m = D.m;
  extern __shared__ double Xs[];
  __shared__ double Zs[QA_WAVES][QR_NB][NCOL + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // the wave's V_p operands of the V_p^T X product (k0 = 4 wave + 32 i): up to
  // 512 rows they are loaded one panel step ahead, under the current step's
  // update (more rows would not fit the registers)
  constexpr bool PF = MAXM <= 512;
  constexpr int KITER = MAXM / (4 * QA_WAVES);
  double va[PF ? KITER : 1];
  auto load_v = [&](int j0) {
    const int jb = min(QR_NB, D.k - j0), R = m - j0;
#pragma unroll
    for (int i = 0; i < (PF ? KITER : 1); ++i) {
      const int kr = 4 * wave + 32 * i + lk;
      va[i] = (kr < R && li < jb) ? D.V[(int64_t)(j0 + li) * m + j0 + kr] : 0.0;
    }
  };
  const int jfirst = ((min(D.k, c0 + nc) - 1) / QR_NB) * QR_NB;
  if (PF) load_v(jfirst);
  for (int e = tid; e < m * NCOL; e += QA_THREADS) {
    const int r = e / NCOL, cc = e % NCOL;
    Xs[r * LD + cc] = (cc < nc && r == c0 + cc) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j0 = jfirst; j0 >= 0; j0 -= QR_NB) {
    const int jb = min(QR_NB, D.k - j0), R = m - j0;
    // the wave's operands of U = V_p T_p for the update below, issued first
    // (they do not depend on Z): 16-row tile rt = wave + QA_WAVES j
    const int ntiles = (R + 15) / 16;
    double ub[TASKS][4];
#pragma unroll
    for (int j = 0; j < TASKS; ++j) {
      const int rt = wave + j * QA_WAVES;
      const int r = j0 + 16 * rt + li;
      const bool ok = rt < ntiles && r < m;
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0) {
        const int t = 4 * t0 + lk;
        ub[j][t0] = (ok && t < jb) ? D.VT[(int64_t)(j0 + t) * m + r] : 0.0;
      }
    }
    // Z = V_p^T X: A[t][k] = V[j0 + k][j0 + t], B[k][c] = X[j0 + k][c]
    d4v z = d4v{0.0, 0.0, 0.0, 0.0};
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < KITER; ++i) {
        const int k0 = 4 * wave + 32 * i;
        if (k0 < R) {  // wave-uniform
          const int kr = k0 + lk, r = j0 + kr;
          const double b = (kr < R && li < NCOL) ? Xs[r * LD + li] : 0.0;
          z = __builtin_amdgcn_mfma_f64_16x16x4f64(va[i], b, z, 0, 0, 0);
        }
      }
      // the next panel step's operands (independent of this step's results)
      if (j0 >= QR_NB) load_v(j0 - QR_NB);
    } else {
#pragma unroll 8
      for (int k0 = 4 * wave; k0 < R; k0 += 4 * QA_WAVES) {
        const int kr = k0 + lk, r = j0 + kr;
        const bool rv = kr < R;
        const double a = (rv && li < jb) ? D.V[(int64_t)(j0 + li) * m + r] : 0.0;
        const double b = (rv && li < NCOL) ? Xs[r * LD + li] : 0.0;
        z = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, z, 0, 0, 0);
      }
    }
    // D register q: row 4 q + lane / 16, column lane % 16; waves summed in
    // wave order
    if (li < NCOL)
#pragma unroll
      for (int q = 0; q < 4; ++q) Zs[wave][4 * q + lk][li] = z[q];
    __syncthreads();
    if (tid < QR_NB * NCOL) {
      const int t = tid / NCOL, cc = tid % NCOL;
      double sum = Zs[0][t][cc];
#pragma unroll
      for (int w = 1; w < QA_WAVES; ++w) sum += Zs[w][t][cc];
      Zs[0][t][cc] = sum;
    }
    __syncthreads();
    // X^T[c][r] -= sum_t Z[t][c] U[r][t] on 16-row tiles (U = V_p T_p):
    // A[c][t] = Z[t][c], B[t][r] = U[r][t]
#pragma unroll
    for (int j = 0; j < TASKS; ++j) {
      const int rt = wave + j * QA_WAVES;
      if (rt >= ntiles) break;  // wave-uniform
      const int r = j0 + 16 * rt + li;
      double xo[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) xo[q] = r < m ? Xs[r * LD + 4 * q + lk] : 0.0;
      d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(li < NCOL ? Zs[0][4 * t0 + lk][li] : 0.0,
                                                   ub[j][t0], acc, 0, 0, 0);
      if (r < m)
#pragma unroll
        for (int q = 0; q < NQ; ++q) Xs[r * LD + 4 * q + lk] = xo[q] - acc[q];
    }
    __syncthreads();
  }
  // the tile back to the column-major Q workspace (consecutive threads on
  // consecutive rows)
  for (int e = tid; e < m * nc; e += QA_THREADS) {
    const int cc = e / m, r = e - cc * m;
    D.Qw[(int64_t)(c0 + cc) * m + r] = Xs[r * LD + cc];
  }
}

// dynamic LDS of k_qrb_formq_lds<ncol, .> for matrices of at most m rows
size_t fql_lds(int ncol, int m) { return (size_t)m * (ncol + 1) * sizeof(double); }

// whether k_qrb_formq_lds may take its row limits (the LDS opt-in, once per
// process)
std::mutex g_fql_mutex;
int g_fql_ok = -1;
bool fql_enabled() {
  std::lock_guard<std::mutex> lock(g_fql_mutex);
  if (g_fql_ok < 0) {
    g_fql_ok = hipFuncSetAttribute((const void *)k_qrb_formq_lds<16, 512>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)fql_lds(16, 512)) == hipSuccess &&
               hipFuncSetAttribute((const void *)k_qrb_formq_lds<16, 1024>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)fql_lds(16, 1024)) == hipSuccess &&
               hipFuncSetAttribute((const void *)k_qrb_formq_lds<8, 2048>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)fql_lds(8, 2048)) == hipSuccess;
    if (!g_fql_ok) (void)hipGetLastError();
  }
  return g_fql_ok == 1;
}

// sign convention diag(R) >= 0; Q (m x k) and R (k x n) into the caller views
__global__ void k_qrb_finish(QrbBatch B) {
  const QrbDesc &D = B.d[blockIdx.y];
  const int m = D.m, n = D.n, k = D.k;
  const int64_t tq = (int64_t)m * k, tr = (int64_t)k * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tq + tr;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < tq) {
      if (!D.Q) continue;  // R only
      const int i = (int)(idx % m), c = (int)(idx / m);
      const double s = (D.W[(int64_t)c * m + c] < 0.0) ? -1.0 : 1.0;
      D.Q[i * D.qrs + c * D.qcs] = s * D.Qw[idx];
    } else {
      const int64_t e = idx - tq;
      const int r = (int)(e % k), c = (int)(e / k);
      const double s = (D.W[(int64_t)r * m + r] < 0.0) ? -1.0 : 1.0;
      D.R[r * D.rrs + c * D.rcs] = (c >= r) ? s * D.W[(int64_t)c * m + r] : 0.0;
    }
  }
}

}  // namespace

namespace {

bool qr_use_blocked(int m, int n) {
  const int k = std::min(m, n);
  return k > 2 * QR_NB;
}

// blocked Householder QR of cnt matrices (all taking the blocked path)
void qr_blocked(Ctx &c, int cnt, const ConstMatView *A, const MatView *Q, const MatView *R) {
  QrbBatch b{};
  b.count = cnt;
  int64_t ws = 0;
  int kmax = 0, nmax = 0;
  for (int i = 0; i < cnt; ++i) {
    const int m = A[i].rows, n = A[i].cols, k = std::min(m, n);
    ws += (int64_t)m * n + 4 * (int64_t)m * k + QR_NB * QR_NB;
    kmax = std::max(kmax, k);
    nmax = std::max(nmax, n);
  }
  double *Wb = c.buf("qrb_work", ws);
  int64_t o = 0;
  int64_t elems = 0;
  for (int i = 0; i < cnt; ++i) {
    const int m = A[i].rows, n = A[i].cols, k = std::min(m, n);
    QrbDesc &D = b.d[i];
    D.A = A[i].p;
    D.ars = A[i].rs;
    D.acs = A[i].cs;
    D.m = m;
    D.n = n;
    D.k = k;
    D.W = Wb + o;
    o += (int64_t)m * n;
    D.V = Wb + o;
    o += (int64_t)m * k;
    D.VT = Wb + o;
    o += (int64_t)m * k;
    D.VTt = Wb + o;
    o += (int64_t)m * k;
    D.Qw = Wb + o;
    o += (int64_t)m * k;
    D.T = Wb + o;
    o += QR_NB * QR_NB;
    D.Q = Q[i].p;
    D.qrs = Q[i].rs;
    D.qcs = Q[i].cs;
    D.R = R[i].p;
    D.rrs = R[i].rs;
    D.rcs = R[i].cs;
    elems = std::max(elems, (int64_t)m * n + (int64_t)m * k);
  }
  const unsigned g = (unsigned)std::min<int64_t>(1024, (elems + 255) / 256);
  hipLaunchKernelGGL(k_qrb_load, dim3(g, cnt), dim3(256), 0, c.stream, b);
  HIPC(hipGetLastError());
  int mmax = 0;
  for (int i = 0; i < cnt; ++i) mmax = std::max(mmax, b.d[i].m);
  if (mmax <= 512 * QR_REG_MAXROWS) {
    // register panels: the first panel alone, then one launch per panel for
    // its trailing update and the factorisation of the next panel
    const int rows = mmax <= 512 ? 1 : (mmax <= 1024 ? 2 : 4);
    if (rows == 1)
      hipLaunchKernelGGL((k_qrb_panel_reg<8, 1>), dim3(cnt), dim3(512), 0, c.stream, b, 0);
    else if (rows == 2)
      hipLaunchKernelGGL((k_qrb_panel_reg<8, 2>), dim3(cnt), dim3(512), 0, c.stream, b, 0);
    else
      hipLaunchKernelGGL((k_qrb_panel_reg<8, 4>), dim3(cnt), dim3(512), 0, c.stream, b, 0);
    HIPC(hipGetLastError());
    for (int j0 = 0; j0 < kmax; j0 += QR_NB) {
      int tiles = 0;
      for (int i = 0; i < cnt; ++i) {
        const QrbDesc &D = b.d[i];
        const int jb = std::min(QR_NB, D.k - j0);
        const int nt = D.n - j0 - std::max(jb, 0);
        if (jb > 0 && nt > 0) tiles = std::max(tiles, (nt + QA_COLS - 1) / QA_COLS);
      }
      if (tiles == 0) continue;
      if (rows == 1)
        hipLaunchKernelGGL((k_qrb_apply_la<1>), dim3(tiles, cnt), dim3(QA_THREADS), 0, c.stream,
                           b, j0);
      else if (rows == 2)
        hipLaunchKernelGGL((k_qrb_apply_la<2>), dim3(tiles, cnt), dim3(QA_THREADS), 0, c.stream,
                           b, j0);
      else
        hipLaunchKernelGGL((k_qrb_apply_la<4>), dim3(tiles, cnt), dim3(QA_THREADS), 0, c.stream,
                           b, j0);
      HIPC(hipGetLastError());
    }
  } else {
    for (int j0 = 0; j0 < kmax; j0 += QR_NB) {
      // matrices taller than the register panel: panel in HBM, V T by a second kernel
      hipLaunchKernelGGL(k_qrb_panel, dim3(cnt), dim3(LA_THREADS), 0, c.stream, b, j0);
      int64_t rows = 0;
      for (int i = 0; i < cnt; ++i) rows = std::max<int64_t>(rows, (int64_t)(b.d[i].m - j0) * QR_NB);
      const unsigned gv = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (rows + 255) / 256));
      hipLaunchKernelGGL(k_qrb_vt, dim3(gv, cnt), dim3(256), 0, c.stream, b, j0);
      HIPC(hipGetLastError());
      // trailing columns: W[j0:m, j0+jb:n] -= (V_p T_p^T)(V_p^T W[j0:m, j0+jb:n])
      int tiles = 0;
      for (int i = 0; i < cnt; ++i) {
        const QrbDesc &D = b.d[i];
        const int jb = std::min(QR_NB, D.k - j0);
        const int nt = D.n - j0 - std::max(jb, 0);
        if (jb > 0 && nt > 0) tiles = std::max(tiles, (nt + QA_COLS - 1) / QA_COLS);
      }
      if (tiles > 0) {
        hipLaunchKernelGGL(k_qrb_apply, dim3(tiles, cnt), dim3(QA_THREADS), 0, c.stream, b, j0,
                           0);
        HIPC(hipGetLastError());
      }
    }
  }
  // Q = H_0 ... [I; 0], panels applied last to first (not for R-only requests):
  // Q[j0:m, j0:k] -= (V_p T_p)(V_p^T Q[j0:m, j0:k]), all panels in one launch
  {
    const bool lds = mmax <= 2048 && fql_enabled();
    const int ncol = !lds ? FQ_COLS : (mmax <= 1024 ? 16 : 8);
    int tiles = 0;
    for (int i = 0; i < cnt; ++i)
      if (b.d[i].Q) tiles = std::max(tiles, (b.d[i].k + ncol - 1) / ncol);
    if (tiles > 0) {
      if (lds && mmax <= 512)
        hipLaunchKernelGGL((k_qrb_formq_lds<16, 512>), dim3(tiles, cnt), dim3(QA_THREADS),
                           fql_lds(16, mmax), c.stream, b);
      else if (lds && ncol == 16)
        hipLaunchKernelGGL((k_qrb_formq_lds<16, 1024>), dim3(tiles, cnt), dim3(QA_THREADS),
                           fql_lds(16, mmax), c.stream, b);
      else if (lds)
        hipLaunchKernelGGL((k_qrb_formq_lds<8, 2048>), dim3(tiles, cnt), dim3(QA_THREADS),
                           fql_lds(8, mmax), c.stream, b);
      else
        hipLaunchKernelGGL(k_qrb_formq, dim3(tiles, cnt), dim3(QA_THREADS), 0, c.stream, b);
      HIPC(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(k_qrb_finish, dim3(g, cnt), dim3(256), 0, c.stream, b);
  HIPC(hipGetLastError());
}

}  // namespace

void qr_batch(Ctx &c, int count, const ConstMatView *A, const MatView *Q, const MatView *R) {
  // large matrices: blocked path (after the same shape and range checks)
  {
    std::vector<ConstMatView> bA;
    std::vector<MatView> bQ, bR;
    std::vector<ConstMatView> sA;
    std::vector<MatView> sQ, sR;
    for (int i = 0; i < count; ++i) {
      const int m = A[i].rows, n = A[i].cols;
      if (Q[i].rows != m || Q[i].cols != std::min(m, n) || R[i].rows != std::min(m, n) ||
          R[i].cols != n)
        fail(QTT_E_SHAPE, "qr_batch: output shapes");
      int64_t lo = 0, hi = 0;
      span(lo, hi, A[i].rows, A[i].rs);
      span(lo, hi, A[i].cols, A[i].cs);
      c.check_range(A[i].p, lo, hi, 8, "qr A");
      if (Q[i].p) {
        lo = hi = 0;
        span(lo, hi, Q[i].rows, Q[i].rs);
        span(lo, hi, Q[i].cols, Q[i].cs);
        c.check_range(Q[i].p, lo, hi, 8, "qr Q");
      }
      lo = hi = 0;
      span(lo, hi, R[i].rows, R[i].rs);
      span(lo, hi, R[i].cols, R[i].cs);
      c.check_range(R[i].p, lo, hi, 8, "qr R");
      if (qr_use_blocked(m, n)) {
        bA.push_back(A[i]);
        bQ.push_back(Q[i]);
        bR.push_back(R[i]);
      } else {
        sA.push_back(A[i]);
        sQ.push_back(Q[i]);
        sR.push_back(R[i]);
      }
    }
    for (size_t b0 = 0; b0 < bA.size(); b0 += MAX_BATCH) {
      const int cnt = (int)std::min<size_t>(MAX_BATCH, bA.size() - b0);
      qr_blocked(c, cnt, bA.data() + b0, bQ.data() + b0, bR.data() + b0);
    }
    if (sA.empty()) return;
    // the single-workgroup kernel always forms Q: R-only requests get scratch
    int64_t qscr = 0;
    for (const MatView &q : sQ)
      if (!q.p) qscr += (int64_t)q.rows * q.cols;
    if (qscr > 0) {
      double *qs = c.buf("qr_Qscratch", qscr);
      for (MatView &q : sQ)
        if (!q.p) {
          q = MatView{qs, q.rows, q.cols, q.cols, 1};
          qs += (int64_t)q.rows * q.cols;
        }
      qr_batch(c, (int)sA.size(), sA.data(), sQ.data(), sR.data());
      return;
    }
    if ((int)sA.size() != count) {
      qr_batch(c, (int)sA.size(), sA.data(), sQ.data(), sR.data());
      return;
    }
  }
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
