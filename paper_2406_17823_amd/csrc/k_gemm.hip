// Strided batched GEMM on CDNA4 matrix cores.
//
// Every tensor-network contraction of the library (environment updates,
// local right-hand sides, the penalty matvec, QR/SVD factor products) is
// expressed as C[b1,b2](m,n) = alpha sum_k A(m,k) B(k,n) + beta C with
// arbitrary element strides, so that no tensor is ever transposed in HBM.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup (4 wave64s in a 2 x 2
// arrangement, 32 x 32 per wave = 2 x 2 blocks of 16 x 16), K staged through
// LDS in slices of 16.  The loader picks the thread-to-element map from the
// operand's unit-stride dimension so that global loads stay coalesced.
// float64: v_mfma_f64_16x16x4_f64; float32: v_mfma_f32_16x16x4_f32 with
// float64 operands rounded to float32 on the way into LDS.
#include "qtt_internal.h"

namespace qtt {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int MT = 64, NT = 64, KT = 16, PADM = 1;

struct GemmK {
  int M, N, K, B1, B2, tm, tn;
  const double *A;
  int64_t sAm, sAk, sAb1, sAb2;
  const double *B;
  int64_t sBk, sBn, sBb1, sBb2;
  double *C;
  int64_t sCm, sCn, sCb1, sCb2;
  double alpha, beta;
  const int *skip;
  double *flop_ctr;
  double flops;
};

template <typename T>
__device__ inline void mfma_step(const T (*As)[MT + PADM], const T (*Bs)[NT + PADM], int lane,
                                 int wm, int wn, d4v (&acc)[2][2]);

template <>
__device__ inline void mfma_step<double>(const double (*As)[MT + PADM],
                                         const double (*Bs)[NT + PADM], int lane, int wm, int wn,
                                         d4v (&acc)[2][2]) {
#pragma unroll
  for (int kq = 0; kq < KT / 4; ++kq) {
    const int kk = kq * 4 + (lane >> 4);
    double a0 = As[kk][wm * 32 + (lane & 15)];
    double a1 = As[kk][wm * 32 + 16 + (lane & 15)];
    double b0 = Bs[kk][wn * 32 + (lane & 15)];
    double b1 = Bs[kk][wn * 32 + 16 + (lane & 15)];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

template <>
__device__ inline void mfma_step<float>(const float (*As)[MT + PADM], const float (*Bs)[NT + PADM],
                                        int lane, int wm, int wn, d4v (&acc)[2][2]) {
  f4v f[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      f[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kq = 0; kq < KT / 4; ++kq) {
    const int kk = kq * 4 + (lane >> 4);
    float a0 = As[kk][wm * 32 + (lane & 15)];
    float a1 = As[kk][wm * 32 + 16 + (lane & 15)];
    float b0 = Bs[kk][wn * 32 + (lane & 15)];
    float b1 = Bs[kk][wn * 32 + 16 + (lane & 15)];
    f[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, f[0][0], 0, 0, 0);
    f[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, f[0][1], 0, 0, 0);
    f[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, f[1][0], 0, 0, 0);
    f[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, f[1][1], 0, 0, 0);
  }
  // the K slice is accumulated in float32, slices are summed in float64
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)f[i][j][r];
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm(GemmK g) {
  if (g.skip && *g.skip) return;
  if (g.flop_ctr && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(g.flop_ctr, g.flops);
  __shared__ T As[KT][MT + PADM];
  __shared__ T Bs[KT][NT + PADM];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  int64_t bid = blockIdx.x;
  const int tiles = g.tm * g.tn;
  const int t = (int)(bid % tiles);
  const int64_t bb = bid / tiles;
  const int b1 = (int)(bb % g.B1);
  const int b2 = (int)(bb / g.B1);
  const int m0 = (t % g.tm) * MT;
  const int n0 = (t / g.tm) * NT;

  const double *A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const double *B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  double *C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
  const bool a_m_unit = (g.sAm == 1);
  const bool b_n_unit = (g.sBn == 1);

  d4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < g.K; k0 += KT) {
#pragma unroll
    for (int i = 0; i < (MT * KT) / 256; ++i) {
      const int idx = tid + 256 * i;
      int mm, kk;
      if (a_m_unit) {
        mm = idx & (MT - 1);
        kk = idx / MT;
      } else {
        mm = idx / KT;
        kk = idx & (KT - 1);
      }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < g.M && gk < g.K) v = A[gm * g.sAm + gk * g.sAk];
      As[kk][mm] = (T)v;
    }
#pragma unroll
    for (int i = 0; i < (NT * KT) / 256; ++i) {
      const int idx = tid + 256 * i;
      int nn, kk;
      if (b_n_unit) {
        nn = idx & (NT - 1);
        kk = idx / NT;
      } else {
        nn = idx / KT;
        kk = idx & (KT - 1);
      }
      const int gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < g.N && gk < g.K) v = B[gk * g.sBk + gn * g.sBn];
      Bs[kk][nn] = (T)v;
    }
    __syncthreads();
    mfma_step<T>(As, Bs, lane, wm, wn, acc);
    __syncthreads();
  }

  // D(16x16): lane l holds column l % 16.  float32 16x16x4: register r is row
  // 4*(l/16) + r; float64 16x16x4: register r is row 4*r + l/16.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (sizeof(T) == 8) ? (4 * r + (lane >> 4)) : ((lane >> 4) * 4 + r);
        const int gm = m0 + wm * 32 + i * 16 + row;
        const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          double *cp = C + gm * g.sCm + gn * g.sCn;
          double v = g.alpha * acc[i][j][r];
          if (g.beta != 0.0) v += g.beta * *cp;
          *cp = v;
        }
      }
}

template <typename T>
void launch(Ctx &c, const Gemm &q) {
  if (q.M <= 0 || q.N <= 0 || q.B1 <= 0 || q.B2 <= 0) return;
  GemmK g;
  g.M = q.M;
  g.N = q.N;
  g.K = q.K;
  g.B1 = q.B1;
  g.B2 = q.B2;
  g.tm = (q.M + MT - 1) / MT;
  g.tn = (q.N + NT - 1) / NT;
  g.A = q.A;
  g.sAm = q.sAm;
  g.sAk = q.sAk;
  g.sAb1 = q.sAb1;
  g.sAb2 = q.sAb2;
  g.B = q.B;
  g.sBk = q.sBk;
  g.sBn = q.sBn;
  g.sBb1 = q.sBb1;
  g.sBb2 = q.sBb2;
  g.C = q.C;
  g.sCm = q.sCm;
  g.sCn = q.sCn;
  g.sCb1 = q.sCb1;
  g.sCb2 = q.sCb2;
  g.alpha = q.alpha;
  g.beta = q.beta;
  g.skip = q.skip;
  {
    int64_t lo = 0, hi = 0;
    span(lo, hi, q.M, q.sAm);
    span(lo, hi, q.K, q.sAk);
    span(lo, hi, q.B1, q.sAb1);
    span(lo, hi, q.B2, q.sAb2);
    if (q.K > 0) c.check_range(q.A, lo, hi, sizeof(double), "gemm A");
    lo = hi = 0;
    span(lo, hi, q.K, q.sBk);
    span(lo, hi, q.N, q.sBn);
    span(lo, hi, q.B1, q.sBb1);
    span(lo, hi, q.B2, q.sBb2);
    if (q.K > 0) c.check_range(q.B, lo, hi, sizeof(double), "gemm B");
    lo = hi = 0;
    span(lo, hi, q.M, q.sCm);
    span(lo, hi, q.N, q.sCn);
    span(lo, hi, q.B1, q.sCb1);
    span(lo, hi, q.B2, q.sCb2);
    c.check_range(q.C, lo, hi, sizeof(double), "gemm C");
  }
  const int64_t blocks = (int64_t)g.tm * g.tn * g.B1 * g.B2;
  if (blocks > 0x7fffffffLL) fail(QTT_E_UNSUPPORTED, "gemm grid too large");
  const int kind = (sizeof(T) == 8) ? 0 : 1;
  g.flop_ctr = nullptr;
  g.flops = 2.0 * q.M * (double)q.N * q.K * q.B1 * q.B2;
  bool timed = false;
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (c.kt.on) {
    g.flop_ctr = c.kt.flop_ctr + kind;
    timed = (c.kt.launches[kind] % c.kt.every) == 0;
    c.kt.launches[kind] += 1;
    if (timed) {
      if (c.kt.pending[kind].size() >= 16384) c.resolve_events();
      ev.first = c.take_event();
      ev.second = c.take_event();
      HIPC(hipEventRecord(ev.first, c.stream));
    }
  }
  hipLaunchKernelGGL(k_gemm<T>, dim3((unsigned)blocks), dim3(256), 0, c.stream, g);
  HIPC(hipGetLastError());
  if (timed) {
    HIPC(hipEventRecord(ev.second, c.stream));
    c.kt.pending[kind].push_back(ev);
  }
}

}  // namespace

void gemm(Ctx &c, const Gemm &g) { launch<double>(c, g); }
void gemm_f32(Ctx &c, const Gemm &g) { launch<float>(c, g); }

}  // namespace qtt
