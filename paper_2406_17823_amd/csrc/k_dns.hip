// Dense direct numerical simulation on the periodic unit square (App. D)
// and the two comparison measures of the verification section: the fidelity
// (Eq. fidelity) and the turbulent kinetic energy spectrum (Eqs. TKE).
//
// Grid fields are N x N float64, x1-major (U[i1 * N + i2]), N = 2^n.
// * k_dns_stage: eighth-order central differences (Fornberg's weights,
//   offsets 1..4) of a 32 x 32 tile staged in LDS with a periodic halo of
//   4; skew-symmetric convection -1/2 (u_j d_j u_i + d_j(u_j u_i)) plus
//   diffusion (1/Re) lap u_i, fused with the Runge-Kutta bookkeeping
//   (stage sum and the intermediate velocity, written packed as u1 + i u2
//   for the transform).
// * The projection onto divergence-free fields (Eq. projection) by a 2D
//   FFT of the packed pair: radix-2 rows in LDS with a twiddle table, a
//   tiled transpose, rows again; the projector u^ - kappa (kappa . u^) /
//   |kappa|^2 separates the two real fields from Z(k) and conj Z(-k); the
//   Nyquist component of kappa is 0, so the projected pair is again the
//   transform of two real fields and the inverse unpacks it exactly.  The
//   second forward row transform, the projector and the first inverse row
//   transform run in one kernel on the rows k2 and -k2 (five passes over
//   the spectrum per projection).
// * TKE shells: |u1^|^2 + |u2^|^2 summed over k and -k equals |Z(k)|^2 +
//   |Z(-k)|^2, so the shell sum of E is sum |Z(k)|^2 / (2 N^4); partial
//   sums per row and shell, reduced per shell in a fixed order.
// All kernels are HBM-bound streaming passes (the stencil reads each value
// once per tile plus the halo); every grid is guarded for N < 32.
#include "qtt_internal.h"

#include <cmath>

namespace qtt {

namespace {

constexpr int TILE = 32, HALO = 4, TW = TILE + 2 * HALO;

struct StageArgs {
  const double *w1, *w2;  // stage argument (the right-hand side is taken there)
  const double *u1, *u2;  // field at the start of the step
  double *acc1, *acc2;    // stage sum of right-hand sides
  double2 *z;             // packed intermediate velocity u + gz * (acc or F)
  double *f1, *f2;        // right-hand side only (rhs_only)
  double inv_dx, inv_dx2, inv_re;
  double acc_w, gz;
  int acc_mode;           // 0: no stage sum, 1: acc = F, 2: acc += acc_w F
  int z_from_acc;         // 1: z = u + gz acc (after the update), 0: z = u + gz F
  int rhs_only;
  int n;
};

__global__ __launch_bounds__(256) void k_dns_stage(StageArgs A) {
  __shared__ double s1[TW][TW + 1], s2[TW][TW + 1];
  const int N = 1 << A.n, mask = N - 1;
  const int i0 = blockIdx.y * TILE, j0 = blockIdx.x * TILE;
  const int tid = threadIdx.y * TILE + threadIdx.x;
  for (int idx = tid; idx < TW * TW; idx += 256) {
    const int lr = idx / TW, lc = idx - lr * TW;
    const int64_t g = (int64_t)((i0 - HALO + lr) & mask) * N + ((j0 - HALO + lc) & mask);
    s1[lr][lc] = A.w1[g];
    s2[lr][lc] = A.w2[g];
  }
  __syncthreads();
  const double w1[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
  const double w2[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  const double w20 = -205.0 / 72.0;
  const int lc = threadIdx.x + HALO, gj = j0 + threadIdx.x;
  for (int rr = threadIdx.y; rr < TILE; rr += 8) {
    const int gi = i0 + rr;
    if (gi >= N || gj >= N) continue;
    const int lr = rr + HALO;
    const double a = s1[lr][lc], b = s2[lr][lc];
    // axis 0 (i1): rows; axis 1 (i2): columns
    double d0a = 0, d0b = 0, d1a = 0, d1b = 0;        // d_j u_i
    double d0aa = 0, d0ab = 0, d1ab = 0, d1bb = 0;    // d_j (u_j u_i)
    double l_a = 2.0 * w20 * a, l_b = 2.0 * w20 * b;  // both axes' centre weight
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
      const double ap = s1[lr + m][lc], am = s1[lr - m][lc];
      const double bp = s2[lr + m][lc], bm = s2[lr - m][lc];
      const double aq = s1[lr][lc + m], an = s1[lr][lc - m];
      const double bq = s2[lr][lc + m], bn = s2[lr][lc - m];
      const double c1 = w1[m - 1], c2 = w2[m - 1];
      d0a += c1 * (ap - am);
      d0b += c1 * (bp - bm);
      d1a += c1 * (aq - an);
      d1b += c1 * (bq - bn);
      d0aa += c1 * (ap * ap - am * am);
      d0ab += c1 * (ap * bp - am * bm);
      d1ab += c1 * (bq * aq - bn * an);
      d1bb += c1 * (bq * bq - bn * bn);
      l_a += c2 * ((ap + am) + (aq + an));
      l_b += c2 * ((bp + bm) + (bq + bn));
    }
    const double f1 = -0.5 * A.inv_dx * ((a * d0a + b * d1a) + (d0aa + d1ab)) + A.inv_re * A.inv_dx2 * l_a;
    const double f2 = -0.5 * A.inv_dx * ((a * d0b + b * d1b) + (d0ab + d1bb)) + A.inv_re * A.inv_dx2 * l_b;
    const int64_t g = (int64_t)gi * N + gj;
    if (A.rhs_only) {
      A.f1[g] = f1;
      A.f2[g] = f2;
      continue;
    }
    double s1v = f1, s2v = f2;
    if (A.acc_mode == 1) {
      A.acc1[g] = f1;
      A.acc2[g] = f2;
    } else if (A.acc_mode == 2) {
      s1v = A.acc1[g] + A.acc_w * f1;
      s2v = A.acc2[g] + A.acc_w * f2;
      A.acc1[g] = s1v;
      A.acc2[g] = s2v;
    }
    const double q1 = A.z_from_acc ? s1v : f1, q2 = A.z_from_acc ? s2v : f2;
    A.z[g] = make_double2(A.u1[g] + A.gz * q1, A.u2[g] + A.gz * q2);
  }
}

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 w) {
  return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// twiddle table of one transform length: tw[k] = exp(-2 pi i k / N), k < N/2
__global__ void k_twiddles(double2 *tw, int n) {
  const int N = 1 << n;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N / 2; k += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(2.0 * k / N, &sn, &cs);
    tw[k] = make_double2(cs, -sn);
  }
}

// R consecutive radix-2 decimation-in-time stages starting at span `half`,
// in registers: thread t takes the 2^R elements i + m half of one group;
// stage r pairs m and m + 2^r (bit r of m clear) with the twiddle of the
// element's position q in its group of 2^(r+1) half, exp(-+2 pi i q / (2^(r+1) half)).
template <int R>
__device__ inline void fused_stages(double2 *s, const double2 *twg, double tsg, int N, int half,
                                    int tid, int nth) {
  constexpr int E = 1 << R;
  for (int t = tid; t < (N >> R); t += nth) {
    const int pos = t & (half - 1);
    const int i = ((t - pos) << R) + pos;
    double2 a[E];
#pragma unroll
    for (int m = 0; m < E; ++m) a[m] = s[i + m * half];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int span = 1 << r, stride = N / ((2 << r) * half);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        if (m & span) continue;
        const double2 w0 = twg[(pos + (m & (span - 1)) * half) * stride];
        const double2 b = cmul(a[m + span], make_double2(w0.x, tsg * w0.y));
        a[m + span] = csub(a[m], b);
        a[m] = cadd(a[m], b);
      }
    }
#pragma unroll
    for (int m = 0; m < E; ++m) s[i + m * half] = a[m];
  }
}

// One radix-2 transform per row, in LDS: bit-reversed load, log2 N
// butterfly stages (fused in pairs), natural-order result.  IN: 0 packed complex, 1 two real
// fields (minus optional means) packed as re + i im.  OUT: 0 packed complex,
// 1 two real fields (re, im) times scale, 2 the row's TKE shell partials.
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_fft_rows(const double2 *zin, const double *ra,
                                                  const double *rb, const double *ma,
                                                  const double *mb, double2 *zout, double *oa,
                                                  double *ob, double scale, double *part,
                                                  int nshell, int n, int inverse,
                                                  const double2 *twg) {
  extern __shared__ double2 sm[];
  const int N = 1 << n, H = N >> 1;
  double2 *s = sm;
  const int64_t base = (int64_t)blockIdx.x * N;
  // twg[k] = exp(-2 pi i k / N), read through the caches (every block reads
  // the same table); the inverse takes the conjugate
  const double tsg = inverse ? -1.0 : 1.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double2 v;
    if (IN == 0) {
      v = zin[base + j];
    } else {
      v.x = ra[base + j] - (ma ? ma[base + j] : 0.0);
      v.y = rb[base + j] - (mb ? mb[base + j] : 0.0);
    }
    s[__brev((unsigned)j) >> (32 - n)] = v;
  }
  __syncthreads();
  // groups of R radix-2 stages (spans half .. 2^(R-1) half) in registers on
  // the 2^R elements i + m half: the operations of R separate stages, one
  // LDS round trip and one barrier per group (R = 3, 3, 3, 2 for n = 11)
  for (int half = 1, rem = n; rem > 0;) {
    const int R = (rem == 4 || rem == 2) ? 2 : (rem >= 3 ? 3 : 1);
    if (R == 3) fused_stages<3>(s, twg, tsg, N, half, threadIdx.x, blockDim.x);
    else if (R == 2) fused_stages<2>(s, twg, tsg, N, half, threadIdx.x, blockDim.x);
    else fused_stages<1>(s, twg, tsg, N, half, threadIdx.x, blockDim.x);
    __syncthreads();
    half <<= R;
    rem -= R;
  }
  if (OUT == 0) {
    for (int j = threadIdx.x; j < N; j += blockDim.x) zout[base + j] = s[j];
  } else if (OUT == 1) {
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      oa[base + j] = s[j].x * scale;
      ob[base + j] = s[j].y * scale;
    }
  } else {
    // row index = wavenumber along the row's transform of the first pass
    const int64_t f = blockIdx.x < (unsigned)H ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - N;
    const int64_t f2 = 4 * f * f;
    for (int sh = threadIdx.x; sh < nshell; sh += blockDim.x) {
      // columns a = |k| in [0, N/2] with round(sqrt(a^2 + f^2)) = sh:
      // (2 sh - 1)^2 <= 4 (a^2 + f^2) < (2 sh + 1)^2
      const int64_t lo2 = sh == 0 ? INT64_MIN : (int64_t)(2 * sh - 1) * (2 * sh - 1) - f2;
      const int64_t hi2 = (int64_t)(2 * sh + 1) * (2 * sh + 1) - f2;
      double acc = 0.0;
      if (hi2 > 0) {
        int64_t alo = 0;
        if (lo2 > 0) {
          alo = (int64_t)ceil(0.5 * sqrt((double)lo2));
          for (int it = 0; it < 4 && 4 * alo * alo < lo2; ++it) ++alo;
          for (int it = 0; it < 4 && alo > 0 && 4 * (alo - 1) * (alo - 1) >= lo2; ++it) --alo;
        }
        int64_t ahi = (int64_t)floor(0.5 * sqrt((double)hi2));
        for (int it = 0; it < 4 && ahi >= 0 && 4 * ahi * ahi >= hi2; ++it) --ahi;
        for (int it = 0; it < 4 && 4 * (ahi + 1) * (ahi + 1) < hi2; ++it) ++ahi;
        if (ahi > H) ahi = H;
        for (int64_t a = alo; a <= ahi; ++a) {
          const double2 v = s[a];
          acc += v.x * v.x + v.y * v.y;
          if (a != 0 && a != H) {
            const double2 u = s[N - a];
            acc += u.x * u.x + u.y * u.y;
          }
        }
      }
      part[(int64_t)blockIdx.x * nshell + sh] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_transpose_c(const double2 *in, double2 *out, int N) {
  __shared__ double2 t[TILE][TILE + 1];
  const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
  for (int r = threadIdx.y; r < TILE; r += 8) {
    const int gi = by + r, gj = bx + threadIdx.x;
    if (gi < N && gj < N) t[r][threadIdx.x] = in[(int64_t)gi * N + gj];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < TILE; r += 8) {
    const int gi = bx + r, gj = by + threadIdx.x;
    if (gi < N && gj < N) out[(int64_t)gi * N + gj] = t[threadIdx.x][r];
  }
}

// Projector on the transposed spectrum T[k2][k1] of the packed pair,
// written to out (out of place: each output reads the mirror mode -k).
// Projected Z(k) from A = Z(k) and M = Z(-k) of the packed pair, kappa = (k1, k2)
__device__ inline double2 proj_mode(double2 A, double2 M, double k1, double k2) {
  const double kk = k1 * k1 + k2 * k2;
  if (kk == 0.0) return A;
  const double2 B = make_double2(M.x, -M.y);  // conj Z(-k)
  const double2 a1 = make_double2(0.5 * (A.x + B.x), 0.5 * (A.y + B.y));  // u1^
  const double2 a2 = make_double2(0.5 * (A.y - B.y), -0.5 * (A.x - B.x)); // u2^
  const double2 sc = make_double2((k1 * a1.x + k2 * a2.x) / kk, (k1 * a1.y + k2 * a2.y) / kk);
  const double2 p1 = make_double2(a1.x - k1 * sc.x, a1.y - k1 * sc.y);
  const double2 p2 = make_double2(a2.x - k2 * sc.x, a2.y - k2 * sc.y);
  return make_double2(p1.x - p2.y, p1.y + p2.x);
}

// signed wavenumber of an FFT index, the Nyquist index as 0
__device__ inline double wn(int idx, int N) {
  const int H = N >> 1;
  return idx == H ? 0.0 : (double)(idx < H ? idx : idx - N);
}

// Rows r and N - r (one row when they coincide) of the half-transformed
// packed pair, T[k2][i1]: forward transforms along i1, the projector on
// every pair of modes (k, -k), which both lie in these rows, an in-place
// bit-reversal permutation and the inverse transforms; written to out in
// the same layout.  Replaces a row-transform pass, the projector pass and
// a second row-transform pass.
__global__ __launch_bounds__(512) void k_fft_project_pair(const double2 *T, double2 *out, int n,
                                                          const double2 *twg) {
  extern __shared__ double2 sm[];
  const int N = 1 << n, H = N >> 1, mask = N - 1;
  const int r0 = blockIdx.x, r1 = (N - r0) & mask;
  const bool two = r0 != r1;
  double2 *s0 = sm, *s1 = two ? sm + N : sm;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const int jr = __brev((unsigned)j) >> (32 - n);
    s0[jr] = T[(int64_t)r0 * N + j];
    if (two) s1[jr] = T[(int64_t)r1 * N + j];
  }
  __syncthreads();
  // the two rows are transformed concurrently, each by half of the workgroup
  const int hq = threadIdx.x >= (blockDim.x >> 1), htid = threadIdx.x - hq * (blockDim.x >> 1);
  const int hn = blockDim.x >> 1;
  double2 *sq = hq ? s1 : s0;
  const bool act = two || hq == 0;
  for (int half = 1, rem = n; rem > 0;) {
    const int R = (rem == 4 || rem == 2) ? 2 : (rem >= 3 ? 3 : 1);
    if (act) {
      if (R == 3) fused_stages<3>(sq, twg, 1.0, N, half, htid, hn);
      else if (R == 2) fused_stages<2>(sq, twg, 1.0, N, half, htid, hn);
      else fused_stages<1>(sq, twg, 1.0, N, half, htid, hn);
    }
    __syncthreads();
    half <<= R;
    rem -= R;
  }
  // projector: each thread owns a mode and its mirror (reads and writes
  // only that pair)
  const double k2a = wn(r0, N), k2b = wn(r1, N);
  if (two) {
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      const int m = (N - c) & mask;
      const double2 A = s0[c], M = s1[m];
      s0[c] = proj_mode(A, M, wn(c, N), k2a);
      s1[m] = proj_mode(M, A, wn(m, N), k2b);
    }
  } else {
    for (int c = threadIdx.x; c <= H; c += blockDim.x) {
      const int m = (N - c) & mask;
      const double2 A = s0[c], M = s0[m];
      s0[c] = proj_mode(A, M, wn(c, N), k2a);
      if (m != c) s0[m] = proj_mode(M, A, wn(m, N), k2a);
    }
  }
  __syncthreads();
  for (int q = 0; q < (two ? 2 : 1); ++q) {
    double2 *s = q ? s1 : s0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      const int jr = __brev((unsigned)j) >> (32 - n);
      if (j < jr) {
        const double2 t = s[j];
        s[j] = s[jr];
        s[jr] = t;
      }
    }
  }
  __syncthreads();
  for (int half = 1, rem = n; rem > 0;) {
    const int R = (rem == 4 || rem == 2) ? 2 : (rem >= 3 ? 3 : 1);
    if (act) {
      if (R == 3) fused_stages<3>(sq, twg, -1.0, N, half, htid, hn);
      else if (R == 2) fused_stages<2>(sq, twg, -1.0, N, half, htid, hn);
      else fused_stages<1>(sq, twg, -1.0, N, half, htid, hn);
    }
    __syncthreads();
    half <<= R;
    rem -= R;
  }
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    out[(int64_t)r0 * N + j] = s0[j];
    if (two) out[(int64_t)r1 * N + j] = s1[j];
  }
}

// E[sh] = scale * sum over rows of part[row][sh], rows in a fixed order:
// 64 shells per block, 4 row groups combined in LDS.
__global__ __launch_bounds__(256) void k_shell_reduce(const double *part, int rows, int nshell,
                                                      double *out, double scale) {
  __shared__ double sh[4][64];
  const int s = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  double acc = 0.0;
  if (s < nshell)
    for (int r = g; r < rows; r += 4) acc += part[(int64_t)r * nshell + s];
  sh[g][threadIdx.x & 63] = acc;
  __syncthreads();
  if (g == 0 && s < nshell)
    out[s] = scale * ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]));
}

inline unsigned blocks_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

void check_n(int n, const char *what) {
  if (n < 3 || n > 11) fail(QTT_E_UNSUPPORTED, std::string(what) + ": n must be 3..11");
}

struct DnsBufs {
  double *w1, *w2, *acc1, *acc2;
  double2 *Z, *T;
  double2 *tw;  // twiddles of length N, written at every call
};

DnsBufs dns_bufs(Ctx &c, int n) {
  const int64_t NN = (int64_t)1 << (2 * n);
  DnsBufs b;
  b.w1 = c.buf("dns_w1", NN);
  b.w2 = c.buf("dns_w2", NN);
  b.acc1 = c.buf("dns_acc1", NN);
  b.acc2 = c.buf("dns_acc2", NN);
  b.Z = (double2 *)c.buf("dns_z", 2 * NN);
  b.T = (double2 *)c.buf("dns_t", 2 * NN);
  b.tw = (double2 *)c.buf("dns_tw", (int64_t)1 << n);
  c.check_range(b.tw, 0, ((int64_t)1 << (n - 1)) - 1, 16, "twiddles");
  hipLaunchKernelGGL(k_twiddles, dim3(((1 << (n - 1)) + 255) / 256), dim3(256), 0, c.stream, b.tw, n);
  HIPC(hipGetLastError());
  return b;
}

template <int IN, int OUT>
void fft_rows(Ctx &c, int n, const double2 *zin, const double *ra, const double *rb,
              const double *ma, const double *mb, double2 *zout, double *oa, double *ob,
              double scale, double *part, int nshell, int inverse, const double2 *tw) {
  const int N = 1 << n;
  c.check_range(tw, 0, N / 2 - 1, 16, "fft twiddles");
  const int64_t NN = (int64_t)N * N;
  if (IN == 0) c.check_range(zin, 0, NN - 1, 16, "fft in");
  if (IN == 1) {
    c.check_range(ra, 0, NN - 1, 8, "fft in re");
    c.check_range(rb, 0, NN - 1, 8, "fft in im");
    if (ma) c.check_range(ma, 0, NN - 1, 8, "fft mean re");
    if (mb) c.check_range(mb, 0, NN - 1, 8, "fft mean im");
  }
  if (OUT == 0) c.check_range(zout, 0, NN - 1, 16, "fft out");
  if (OUT == 1) {
    c.check_range(oa, 0, NN - 1, 8, "fft out re");
    c.check_range(ob, 0, NN - 1, 8, "fft out im");
  }
  if (OUT == 2) c.check_range(part, 0, (int64_t)N * nshell - 1, 8, "fft shell partials");
  const size_t lds = (size_t)N * sizeof(double2);
  const int threads = std::min(256, std::max(64, N / 2));
  hipLaunchKernelGGL((k_fft_rows<IN, OUT>), dim3(N), dim3(threads), lds, c.stream, zin, ra, rb, ma,
                     mb, zout, oa, ob, scale, part, nshell, n, inverse, tw);
  HIPC(hipGetLastError());
}

void transpose(Ctx &c, int n, const double2 *in, double2 *out) {
  const int N = 1 << n;
  c.check_range(in, 0, (int64_t)N * N - 1, 16, "transpose in");
  c.check_range(out, 0, (int64_t)N * N - 1, 16, "transpose out");
  const unsigned g = (unsigned)((N + TILE - 1) / TILE);
  hipLaunchKernelGGL(k_transpose_c, dim3(g, g), dim3(TILE, 8), 0, c.stream, in, out, N);
  HIPC(hipGetLastError());
}

// Z (packed u1* + i u2*) -> divergence-free (o1, o2); Z and T are clobbered.
void project_pair(Ctx &c, int n, DnsBufs &b) {
  const int N = 1 << n;
  const int64_t NN = (int64_t)N * N;
  c.check_range(b.T, 0, NN - 1, 16, "project in");
  c.check_range(b.Z, 0, NN - 1, 16, "project out");
  c.check_range(b.tw, 0, N / 2 - 1, 16, "project twiddles");
  hipLaunchKernelGGL(k_fft_project_pair, dim3(N / 2 + 1), dim3(512), (size_t)2 * N * sizeof(double2),
                     c.stream, b.T, b.Z, n, b.tw);
  HIPC(hipGetLastError());
}

// Z (packed u1* + i u2*) -> divergence-free (o1, o2); Z and T are clobbered.
void project_packed(Ctx &c, int n, DnsBufs &b, double *o1, double *o2) {
  const int N = 1 << n;
  const int64_t NN = (int64_t)N * N;
  fft_rows<0, 0>(c, n, b.Z, nullptr, nullptr, nullptr, nullptr, b.Z, nullptr, nullptr, 1.0,
                 nullptr, 0, 0, b.tw);
  transpose(c, n, b.Z, b.T);
  project_pair(c, n, b);
  transpose(c, n, b.Z, b.T);
  fft_rows<0, 1>(c, n, b.T, nullptr, nullptr, nullptr, nullptr, nullptr, o1, o2,
                 1.0 / (double)NN, nullptr, 0, 1, b.tw);
}

void stage(Ctx &c, int n, StageArgs A) {
  const int N = 1 << n;
  const int64_t NN = (int64_t)N * N;
  A.n = n;
  A.inv_dx = (double)N;
  A.inv_dx2 = (double)N * (double)N;
  c.check_range(A.w1, 0, NN - 1, 8, "dns w1");
  c.check_range(A.w2, 0, NN - 1, 8, "dns w2");
  if (A.rhs_only) {
    c.check_range(A.f1, 0, NN - 1, 8, "dns f1");
    c.check_range(A.f2, 0, NN - 1, 8, "dns f2");
  } else {
    c.check_range(A.u1, 0, NN - 1, 8, "dns u1");
    c.check_range(A.u2, 0, NN - 1, 8, "dns u2");
    c.check_range(A.z, 0, NN - 1, 16, "dns z");
    if (A.acc_mode) {
      c.check_range(A.acc1, 0, NN - 1, 8, "dns acc1");
      c.check_range(A.acc2, 0, NN - 1, 8, "dns acc2");
    }
  }
  const unsigned g = (unsigned)((N + TILE - 1) / TILE);
  hipLaunchKernelGGL(k_dns_stage, dim3(g, g), dim3(TILE, 8), 0, c.stream, A);
  HIPC(hipGetLastError());
}

StageArgs stage_args(const double *w1, const double *w2, const double *u1, const double *u2,
                     DnsBufs &b, double re) {
  StageArgs A{};
  A.w1 = w1;
  A.w2 = w2;
  A.u1 = u1;
  A.u2 = u2;
  A.acc1 = b.acc1;
  A.acc2 = b.acc2;
  A.z = b.Z;
  A.inv_re = 1.0 / re;
  return A;
}

}  // namespace

void dns_rhs(Ctx &c, const double *u1, const double *u2, double *f1, double *f2, int n,
             double re) {
  check_n(n, "dns_rhs");
  StageArgs A{};
  A.w1 = u1;
  A.w2 = u2;
  A.f1 = f1;
  A.f2 = f2;
  A.inv_re = 1.0 / re;
  A.rhs_only = 1;
  stage(c, n, A);
}

void dns_project(Ctx &c, double *u1, double *u2, int n) {
  check_n(n, "dns_project");
  DnsBufs b = dns_bufs(c, n);
  const int N = 1 << n;
  const int64_t NN = (int64_t)N * N;
  fft_rows<1, 0>(c, n, nullptr, u1, u2, nullptr, nullptr, b.Z, nullptr, nullptr, 1.0, nullptr, 0,
                 0, b.tw);
  transpose(c, n, b.Z, b.T);
  project_pair(c, n, b);
  transpose(c, n, b.Z, b.T);
  fft_rows<0, 1>(c, n, b.T, nullptr, nullptr, nullptr, nullptr, nullptr, u1, u2,
                 1.0 / (double)NN, nullptr, 0, 1, b.tw);
}

void dns_step(Ctx &c, double *u1, double *u2, int n, double re, double dt, int order,
              int steps) {
  check_n(n, "dns_step");
  DnsBufs b = dns_bufs(c, n);
  for (int s = 0; s < steps; ++s) {
    if (order == 1) {
      StageArgs A = stage_args(u1, u2, u1, u2, b, re);
      A.gz = dt;
      stage(c, n, A);
      project_packed(c, n, b, u1, u2);
      continue;
    }
    // classical RK4, every stage velocity projected
    StageArgs A = stage_args(u1, u2, u1, u2, b, re);
    A.acc_mode = 1;
    A.gz = 0.5 * dt;
    stage(c, n, A);
    project_packed(c, n, b, b.w1, b.w2);
    A = stage_args(b.w1, b.w2, u1, u2, b, re);
    A.acc_mode = 2;
    A.acc_w = 2.0;
    A.gz = 0.5 * dt;
    stage(c, n, A);
    project_packed(c, n, b, b.w1, b.w2);
    A = stage_args(b.w1, b.w2, u1, u2, b, re);
    A.acc_mode = 2;
    A.acc_w = 2.0;
    A.gz = dt;
    stage(c, n, A);
    project_packed(c, n, b, b.w1, b.w2);
    A = stage_args(b.w1, b.w2, u1, u2, b, re);
    A.acc_mode = 2;
    A.acc_w = 1.0;
    A.z_from_acc = 1;
    A.gz = dt / 6.0;
    stage(c, n, A);
    project_packed(c, n, b, u1, u2);
  }
}

int tke_shells(int n) { return (int)std::llround(std::sqrt(2.0) * (double)(1 << (n - 1))) + 1; }

void dns_tke(Ctx &c, const double *u1, const double *u2, const double *m1, const double *m2,
             int n, double *E_dev) {
  check_n(n, "tke_spectrum");
  const int N = 1 << n, S = tke_shells(n);
  DnsBufs b = dns_bufs(c, n);
  double *part = c.buf("dns_shell_part", (int64_t)N * S);
  fft_rows<1, 0>(c, n, nullptr, u1, u2, m1, m2, b.Z, nullptr, nullptr, 1.0, nullptr, 0, 0, b.tw);
  transpose(c, n, b.Z, b.T);
  fft_rows<0, 2>(c, n, b.T, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 1.0,
                 part, S, 0, b.tw);
  c.check_range(E_dev, 0, S - 1, 8, "tke out");
  const double NN = (double)N * (double)N;
  hipLaunchKernelGGL(k_shell_reduce, dim3((S + 63) / 64), dim3(256), 0, c.stream, part, N, S,
                     E_dev, 1.0 / (2.0 * NN * NN));
  HIPC(hipGetLastError());
}

void fidelity(Ctx &c, const double *a, const double *b, int64_t len, double *out_dev3) {
  dot(c, a, b, len, out_dev3);
  dot(c, a, a, len, out_dev3 + 1);
  dot(c, b, b, len, out_dev3 + 2);
}

}  // namespace qtt
