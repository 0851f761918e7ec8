// Batched one-sided block-Jacobi SVD (float64) for the truncation sweeps.
//
// A (m x n, m >= n) is orthogonalised column-wise: A V = W with W's columns
// mutually orthogonal, sigma_j = ||w_j||, u_j = w_j / sigma_j.  The columns
// are split into blocks of b; every outer round pairs the blocks with a
// round-robin schedule and one 1024-thread workgroup takes one block pair:
// its 2b columns are staged in LDS, one Jacobi sweep over all column pairs of
// the block pair runs there (one wave per pair and LDS-resident reductions),
// the accumulated 2b x 2b rotation is applied to the matching columns of V
// in HBM, and the columns go back.  Pairs of one round touch disjoint
// columns, so a round is one launch with (#pairs x #matrices) workgroups.
// Matrices with n <= 2b are one block pair and converge inside one launch.
// Rotations are counted per matrix; a sweep without rotations ends the
// iteration (the host reads the counters once per outer sweep).
#include "qtt_internal.h"

#include <cstdio>
#include <cstdlib>
#include <mutex>

namespace qtt {

namespace {

constexpr int SV_THREADS = 1024;
constexpr int SV_WAVES = SV_THREADS / 64;
// larger matrices: blocks of SV_BQ columns (halved when a block pair of m rows
// does not fit LDS), a block pair per SVB_THREADS-thread
// workgroup; matrices with at most SV_SINGLE columns are one block pair
constexpr int SV_BQ = 16, SVB_THREADS = 512, SV_SINGLE = 64;
constexpr int SV_MAXB = 8;
// rotation threshold on the cosine between two columns: sqrt(m) units of
// roundoff (the level at which computed column products stop carrying
// information, as in the one-sided Jacobi literature); a fixed tighter
// threshold sits below the noise of m-term sums and never stops rotating
constexpr double SV_EPS = 1.1102230246251565e-16;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Jacobi rotation (cs, sn, t = sn / cs, the smaller angle) that zeroes the
// off-diagonal of the symmetric 2 x 2 block [al ga; ga be], ga != 0.  With
// a = be - al, b = 2 ga and r = sqrt(a^2 + b^2) the tangent is
// sgn * |b| / (|a| + r) and 1 / cos^2 = 2 r / (|a| + r) (the half-angle form),
// so cs = q m and sn = p m with q = |a| + r, p = sgn |b|, m = 1 / sqrt(2 r q):
// one square root and one reciprocal square root, no division, on the chain.
// a and b are first scaled by a power of two (exact) into [0.5, 1), so
// a^2 + b^2 neither overflows nor underflows.  The reciprocal square root is
// the hardware estimate refined by three Newton steps (quadratic convergence
// to the rounding level from any estimate within 2^-10).  The sign convention
// of the quotient form is kept: a = 0 takes the positive tangent.
__device__ inline void jacobi_rotation(double al, double be, double ga, double &cs, double &sn,
                                       double &t) {
  double a = be - al, b = 2.0 * ga;
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(a), fabs(b)));
  a = __builtin_amdgcn_ldexp(a, -e);
  b = __builtin_amdgcn_ldexp(b, -e);
  const double r = sqrt(fma(a, a, b * b));
  const double q = fabs(a) + r;
  const bool neg = (a != 0.0) & ((a < 0.0) != (b < 0.0));
  const double p = neg ? -fabs(b) : fabs(b);
  const double x = 2.0 * r * q;
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 3; ++i) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  cs = q * y;
  sn = p * y;
  t = sn * (2.0 * r * y);
}

struct SvMat {
  const double *A;
  int m, n;
  int64_t ars, acs;
  double *W;   // m x n column-major
  double *V;   // n x n column-major
  int *count;  // rotations of the current sweep
  double *fro2;  // squared Frobenius norm of A (invariant under the rotations)
  int accumulate;  // accumulate the rotations into V (0: V is not wanted)
  int b;       // block width
  int nb;      // blocks
  int single;  // n <= 2b: whole matrix is one block pair
  int first;   // first workgroup of this matrix in a round launch
  double *U;
  int64_t urs, ucs;
  double *S;
  double *Vout;
  int64_t vrs, vcs;
};
struct SvBatch {
  int count;
  SvMat d[SV_MAXB];
};

__global__ __launch_bounds__(SV_THREADS) void k_sv_init(SvBatch B) {
  const SvMat &D = B.d[blockIdx.x];
  __shared__ double part[SV_WAVES];
  double ss = 0.0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)D.m * D.n; idx += SV_THREADS) {
    const int i = (int)(idx % D.m), j = (int)(idx / D.m);
    const double a = D.A[i * D.ars + j * D.acs];
    D.W[idx] = a;
    ss += a * a;
  }
  ss = wave_sum(ss);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < SV_WAVES; ++w) t += part[w];
    *D.fro2 = t;
  }
  for (int64_t idx = threadIdx.x; idx < (int64_t)D.n * D.n; idx += SV_THREADS) {
    const int i = (int)(idx % D.n), j = (int)(idx / D.n);
    D.V[idx] = (i == j) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) *D.count = 0;
}

// sum over a 16-lane group of a wave
__device__ inline double grp16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}

// one Jacobi sweep over the column pairs of the nc LDS columns; returns the
// number of rotations (valid in every thread after the final barrier).  A
// pair is handled by a group of 16 lanes (NT / 16 pairs at once), so its
// three column products need four exchange steps, not six.
// Columns whose squared norm is below floor2 are numerically zero (pure
// roundoff); rotating them against each other never converges and changes
// nothing above the noise, so such pairs are skipped.
template <int NT>
__device__ int inner_sweep(double *cols, int m, int nc, double *Wacc, int *rot, double floor2) {
  const double tol = sqrt((double)m) * SV_EPS;
  constexpr int NG = NT / 16;
  const int gl = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int np = nc + (nc & 1);
  if (threadIdx.x == 0) *rot = 0;
  __syncthreads();
  for (int r = 0; r < np - 1; ++r) {
    for (int pr = grp; pr < np / 2; pr += NG) {
      int p, q;
      if (pr == 0) {
        p = np - 1;
        q = r;
      } else {
        p = (r + pr) % (np - 1);
        q = (r - pr + np - 1) % (np - 1);
      }
      if (p >= nc || q >= nc) continue;
      if (p > q) {
        const int t = p;
        p = q;
        q = t;
      }
      double *cp = cols + (int64_t)p * m;
      double *cq = cols + (int64_t)q * m;
      double al = 0.0, be = 0.0, ga = 0.0;
      for (int i = gl; i < m; i += 16) {
        const double x = cp[i], y = cq[i];
        al += x * x;
        be += y * y;
        ga += x * y;
      }
      al = grp16_sum(al);
      be = grp16_sum(be);
      ga = grp16_sum(ga);
      if (ga != 0.0 && al > floor2 && be > floor2 && fabs(ga) > tol * sqrt(al * be)) {
        double cs, sn, t;
        jacobi_rotation(al, be, ga, cs, sn, t);
        for (int i = gl; i < m; i += 16) {
          const double x = cp[i], y = cq[i];
          cp[i] = cs * x - sn * y;
          cq[i] = sn * x + cs * y;
        }
        double *wp = Wacc + p * nc, *wq = Wacc + q * nc;
        for (int i = gl; i < nc; i += 16) {
          const double x = wp[i], y = wq[i];
          wp[i] = cs * x - sn * y;
          wq[i] = sn * x + cs * y;
        }
        if (gl == 0) atomicAdd(rot, 1);
      }
    }
    __syncthreads();
  }
  return *rot;
}

// LDS: cols[nc][m], Wacc[nc][nc] (column-major: Wacc[c * nc + k]), colidx[nc], rot
// NT = 1024 for matrices that are one block pair (the sweep repeats inside
// the launch), NT = SVB_THREADS for block pairs of 2 SV_BQ columns
template <int NT>
__global__ __launch_bounds__(NT) void k_sv_round(SvBatch B, int round) {
  extern __shared__ double lds[];
  // which matrix and which pair
  int mi = 0;
  for (int i = 1; i < B.count; ++i)
    if ((int)blockIdx.x >= B.d[i].first) mi = i;
  const SvMat &D = B.d[mi];
  const int t = (int)blockIdx.x - D.first;
  const int m = D.m, n = D.n, b = D.b;
  int blk[2];
  int nblk;
  if (D.single) {
    blk[0] = 0;
    nblk = 1;
  } else {
    const int nbp = D.nb + (D.nb & 1);
    int P, Q;
    if (t == 0) {
      P = nbp - 1;
      Q = round;
    } else {
      P = (round + t) % (nbp - 1);
      Q = (round - t + nbp - 1) % (nbp - 1);
    }
    nblk = 0;
    if (P < D.nb) blk[nblk++] = P;
    if (Q < D.nb) blk[nblk++] = Q;
    if (nblk == 2 && blk[0] > blk[1]) {
      const int x = blk[0];
      blk[0] = blk[1];
      blk[1] = x;
    }
  }
  // column list
  __shared__ int colidx[2 * 64];
  __shared__ int rot;
  int nc = 0;
  if (D.single) {
    nc = n;
  } else {
    for (int k = 0; k < nblk; ++k) {
      const int c0 = blk[k] * b, c1 = min(c0 + b, n);
      nc += c1 - c0;
    }
  }
  if (threadIdx.x == 0) {
    int o = 0;
    if (D.single) {
      for (int c = 0; c < n; ++c) colidx[o++] = c;
    } else {
      for (int k = 0; k < nblk; ++k)
        for (int c = blk[k] * b; c < min(blk[k] * b + b, n); ++c) colidx[o++] = c;
    }
  }
  double *cols = lds;
  double *Wacc = lds + (int64_t)nc * m;
  // numerically zero columns: norm below 4 sqrt(m) eps ||A||_F
  const double fl = 4.0 * sqrt((double)m) * SV_EPS;
  const double floor2 = fl * fl * *D.fro2;
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < (int64_t)nc * m; idx += NT) {
    const int k = (int)(idx / m), i = (int)(idx % m);
    cols[idx] = D.W[(int64_t)colidx[k] * m + i];
  }
  for (int idx = threadIdx.x; idx < nc * nc; idx += NT)
    Wacc[idx] = ((idx / nc) == (idx % nc)) ? 1.0 : 0.0;
  __syncthreads();

  int total = 0, any = 0;
  if (D.single) {
    int last = 1;
    for (int s = 0; s < 60 && last > 0; ++s) {
      last = inner_sweep<NT>(cols, m, nc, Wacc, &rot, floor2);
      any += last;
      __syncthreads();
    }
    total = last;
  } else {
    total = inner_sweep<NT>(cols, m, nc, Wacc, &rot, floor2);
    any = total;
  }
  __syncthreads();
  // columns back to HBM
  for (int64_t idx = threadIdx.x; idx < (int64_t)nc * m; idx += NT) {
    const int k = (int)(idx / m), i = (int)(idx % m);
    D.W[(int64_t)colidx[k] * m + i] = cols[idx];
  }
  // V[:, cols] <- V[:, cols] Wacc, staged through the LDS the columns used
  // (n <= m, so the n x nc slice fits)
  if (any > 0 && D.accumulate) {
    __syncthreads();
    double *Vl = cols;
    for (int64_t idx = threadIdx.x; idx < (int64_t)nc * n; idx += NT) {
      const int k = (int)(idx / n), i = (int)(idx % n);
      Vl[idx] = D.V[(int64_t)colidx[k] * n + i];
    }
    __syncthreads();
    for (int64_t idx = threadIdx.x; idx < (int64_t)nc * n; idx += NT) {
      const int cc = (int)(idx / n), i = (int)(idx % n);
      double s = 0.0;
      for (int k = 0; k < nc; ++k) s += Vl[(int64_t)k * n + i] * Wacc[cc * nc + k];
      D.V[(int64_t)colidx[cc] * n + i] = s;
    }
  }
  if (threadIdx.x == 0) {
    if (D.single) *D.count = total;
    else if (total > 0) atomicAdd(D.count, total);
  }
}

// ---- Gram-matrix form of a block-pair round (blocked matrices)
//
// Same outer schedule, rotation angles and threshold test as k_sv_round
// (the inner sweep of outer rounds past the first takes only the pairs
// across the two blocks, see below), organised around the Gram matrix of
// the block pair: its NC
// column slots (m rows, zero-padded to a multiple of 16 rows; empty slots
// are zero columns and never rotate) are staged row-major in LDS, G = X^T X
// is formed with float64 MFMAs, and the inner sweep runs on G as two-sided
// Jacobi: the NC/2 disjoint rotations of an inner round act on G as
// G <- R^T G R, 2 x 2 block by 2 x 2 block, with the rotated diagonal in the
// stable form a_pp - t a_pq, a_qq + t a_pq (the off-diagonal of the pair set
// to zero).  These are the column inner products the one-sided method would
// recompute after each rotation.  The accumulated rotation J (NC x NC) is
// applied to the columns, and to V, once per round with MFMAs.  An inner
// round costs O(NC^2) LDS work instead of O(m NC), so a round is bound by
// the two m x NC x NC products rather than by 31 dependent column passes.
constexpr int SVG_THREADS = 512;
constexpr int SVG_WAVES = SVG_THREADS / 64;
// V slots held in registers per thread while the sweep runs (the V loads are
// issued before the Gram product and consumed after it)
constexpr int SVG_VREG = 40;

typedef double d4v __attribute__((ext_vector_type(4)));

// rows x NC (row-major, leading dimension NC + 1, rows a multiple of 16)
// <- itself times J (NC x NC, same layout); each wave owns whole 16-row
// blocks, reads them completely before overwriting them
template <int NC>
__device__ void svg_apply_j(double *Xs, const double *J, int rows, int wave, int lane) {
  constexpr int LD = NC + 1, NT16 = NC / 16;
  for (int rb = wave; rb < rows / 16; rb += SVG_WAVES) {
    d4v acc[NT16];
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < NC; k0 += 4) {
      const int kk = k0 + (lane >> 4);
      // A[i][k] = X[16 rb + i][k]: lane supplies i = lane % 16, k = lane / 16
      const double a = Xs[(rb * 16 + (lane & 15)) * LD + kk];
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const double b = J[kk * LD + t * 16 + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    // D register r is row 4 r + lane / 16, column lane % 16
#pragma unroll
    for (int t = 0; t < NT16; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Xs[(rb * 16 + 4 * r + (lane >> 4)) * LD + t * 16 + (lane & 15)] = acc[t][r];
  }
}

// column slots of a column-major m x n matrix (slot c holds column colidx[c],
// -1: zero) into rows 0..mp of the row-major LDS block, rows >= m zero.  A
// thread takes row i of every slot (consecutive threads, consecutive rows:
// coalesced column reads), UNR slots' loads issued before their LDS stores
// (no index division)
template <int NC, int UNR>
__device__ void svg_stage(double *Xs, const double *src, int m, int mp, const int *colidx,
                          int tid) {
  static_assert(NC % UNR == 0, "whole slot groups");
  constexpr int LD = NC + 1;
  for (int i = tid; i < mp; i += SVG_THREADS) {
#pragma unroll
    for (int c0 = 0; c0 < NC; c0 += UNR) {
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int gc = colidx[c0 + u];
        v[u] = (gc >= 0 && i < m) ? src[(int64_t)gc * m + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) Xs[i * LD + c0 + u] = v[u];
    }
  }
}

// the LDS block's first m rows back to the slots' columns (column by column,
// consecutive threads on consecutive rows)
template <int NC>
__device__ void svg_unstage(double *dst, const double *Xs, int m, const int *colidx, int tid) {
  constexpr int LD = NC + 1;
  for (int c = 0; c < NC; ++c) {
    const int gc = colidx[c];
    if (gc < 0) continue;
    for (int i = tid; i < m; i += SVG_THREADS) dst[(int64_t)gc * m + i] = Xs[i * LD + c];
  }
}

// ACC: the launch accumulates rotations into V for some matrix (else the V
// registers are not allocated and the staging issues all NC slots' loads at
// once)
template <int NC, bool ACC>
__global__ __launch_bounds__(SVG_THREADS) void k_svg_round(SvBatch B, int round) {
  static_assert(NC == 16 || NC == 32, "block pairs of 16 or 32 column slots");
  constexpr int LD = NC + 1, P = NC / 2, NT16 = NC / 16;
  extern __shared__ double lds[];
  int mi = 0;
  for (int i = 1; i < B.count; ++i)
    if ((int)blockIdx.x >= B.d[i].first) mi = i;
  const SvMat &D = B.d[mi];
  const int tw = (int)blockIdx.x - D.first;
  const int m = D.m, n = D.n, b = D.b;
  const int mp = (m + 15) & ~15;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int colidx[NC];
  __shared__ double rc[P], rs[P], rt[P];
  __shared__ int rf[P];
  __shared__ int rot;
  if (tid == 0) {
    int o = 0;
    if (D.single) {
      for (int c = 0; c < n; ++c) colidx[o++] = c;
    } else {
      const int nbp = D.nb + (D.nb & 1);
      int blk[2] = {0, 0};
      if (tw == 0) {
        blk[0] = nbp - 1;
        blk[1] = round;
      } else {
        blk[0] = (round + tw) % (nbp - 1);
        blk[1] = (round - tw + nbp - 1) % (nbp - 1);
      }
      if (blk[0] > blk[1]) {
        const int x = blk[0];
        blk[0] = blk[1];
        blk[1] = x;
      }
      for (int k = 0; k < 2; ++k)
        if (blk[k] < D.nb)
          for (int c = blk[k] * b; c < min(blk[k] * b + b, n); ++c) colidx[o++] = c;
    }
    while (o < NC) colidx[o++] = -1;
    rot = 0;
  }
  double *Xs = lds;
  double *G = Xs + (int64_t)mp * LD;
  double *J = G + NC * LD;
  double *Gp = J + NC * LD;
  const double fl = 4.0 * sqrt((double)m) * SV_EPS;
  const double floor2 = fl * fl * *D.fro2;
  const double tol2 = (double)m * SV_EPS * SV_EPS;
  __syncthreads();
  // V slots of the pair: loads issued now into registers when they fit
  const int np16 = (n + 15) & ~15;
  constexpr int VREG = ACC ? SVG_VREG : 1;
  const bool vreg = ACC && D.accumulate && np16 * NC <= SVG_VREG * SVG_THREADS;
  double vr[VREG];
#pragma unroll
  for (int u = 0; u < VREG; ++u) {
    const int idx = tid + u * SVG_THREADS;
    vr[u] = 0.0;
    if (vreg && idx < np16 * NC) {
      const int c = idx / np16, i = idx - c * np16;
      const int gc = colidx[c];
      if (gc >= 0 && i < n) vr[u] = D.V[(int64_t)gc * n + i];
    }
  }
  svg_stage<NC, ACC ? 8 : NC>(Xs, D.W, m, mp, colidx, tid);
  for (int idx = tid; idx < NC * NC; idx += SVG_THREADS) {
    const int i = idx / NC, j = idx - i * NC;
    J[i * LD + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // G = X^T X: 16 x 16 tiles of the upper block triangle (1 or 3), the rows
  // split in two halves: waves 0.. take the first half into G, waves 4.. the
  // second into Gp, then G += Gp (fixed order)
  {
    constexpr int NTILE = NT16 * (NT16 + 1) / 2;
    const int half = wave / 4, wt = wave % 4;
    int ta = -1, tb = -1;
    if (wt < NTILE) {
      ta = (wt == 2) ? 1 : 0;
      tb = (wt == 0) ? 0 : 1;
    }
    const int kh = (mp / 16) * 8;  // first half: rows [0, kh), a multiple of 8
    const int klo = half ? kh : 0, khi = half ? mp : kh;
    if (ta >= 0) {
      // two accumulators (rows k0..k0+3 and k0+4..k0+7 of each 8) so that
      // consecutive MFMAs do not wait on each other
      d4v acc = d4v{0.0, 0.0, 0.0, 0.0}, acc2 = d4v{0.0, 0.0, 0.0, 0.0};
      for (int k0 = klo; k0 < khi; k0 += 8) {
        const int k = k0 + (lane >> 4);
        // A[i][k] = X[k][16 ta + i], B[k][j] = X[k][16 tb + j]
        const double a = Xs[k * LD + ta * 16 + (lane & 15)];
        const double bb = Xs[k * LD + tb * 16 + (lane & 15)];
        const double a2 = Xs[(k + 4) * LD + ta * 16 + (lane & 15)];
        const double bb2 = Xs[(k + 4) * LD + tb * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bb2, acc2, 0, 0, 0);
      }
      acc += acc2;
      // diagonal tiles keep their upper triangle, mirrored: G exactly symmetric
      double *Gh = half ? Gp : G;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = ta * 16 + 4 * r + (lane >> 4), gj = tb * 16 + (lane & 15);
        if (ta != tb || gi <= gj) {
          Gh[gi * LD + gj] = acc[r];
          Gh[gj * LD + gi] = acc[r];
        }
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < NC * NC; idx += SVG_THREADS) {
    const int i = idx / NC, j = idx - i * NC;
    G[i * LD + j] += Gp[i * LD + j];
  }
  __syncthreads();
  // one inner sweep over the slot pairs, rounds of P disjoint pairs.  Round 0
  // of an outer sweep (and a matrix that is one block pair) takes every pair:
  // NC - 1 rounds of the round-robin, pair k of inner round r being
  // (r, NC - 1) for k = 0, else {(r + k), (r - k)} modulo NC - 1 (one
  // conditional step each: both stay within one period).  The other outer
  // rounds take only the pairs across the two blocks: P rounds, pair k of
  // round r being (k, P + (k + r) mod P).  A block meets every other block
  // once per outer sweep but takes part in every round, so its own pairs were
  // otherwise swept in each of them; in round 0 every block is in exactly one
  // pair, so each column pair is still tested at least once per outer sweep
  // and a sweep without rotations still means every pair passed the
  // threshold test.  Every thread derives the pairs it needs without an LDS
  // round trip.
  // Phase A: P threads compute the rotations from G.  Phase B: every thread
  // updates its 2 x 2 block of G (thread (k1, k2), k1 <= k2) and its row pair
  // of J (row k1, pair k2), all loads issued before any store; a pair that
  // did not rotate has cs = 1, sn = 0, t = 0, which leaves its entries
  // unchanged exactly, so the updates need no branch on it.
  static_assert(NC * P <= SVG_THREADS, "one G block and one J row pair per thread");
  static_assert((P & (P - 1)) == 0, "cross-block schedule modulo a power of two");
  const bool full = D.single || round == 0;
  const int nr = full ? NC - 1 : P;
  auto pair_of = [full](int r, int k, int &p, int &q) {
    if (!full) {
      p = k;
      q = P + ((k + r) & (P - 1));
    } else if (k == 0) {
      p = r;
      q = NC - 1;
    } else {
      int x = r + k, y = r - k;
      x -= (x >= NC - 1) ? NC - 1 : 0;
      y += (y < 0) ? NC - 1 : 0;
      p = min(x, y);
      q = max(x, y);
    }
  };
  const int k1 = tid / P, k2 = tid - k1 * P;
  const bool gdo = tid < P * P && k1 <= k2, jdo = tid < NC * P;
  for (int r = 0; r < nr; ++r) {
    if (tid < P) {
      int p, q;
      pair_of(r, tid, p, q);
      const double al = G[p * LD + p], be = G[q * LD + q], ga = G[p * LD + q];
      double cs = 1.0, sn = 0.0, tt = 0.0;
      int f = 0;
      // |cos| > tol without a square root (al, be > 0 past the floor test)
      if (ga != 0.0 && al > floor2 && be > floor2 && ga * ga > tol2 * (al * be)) {
        jacobi_rotation(al, be, ga, cs, sn, tt);
        f = 1;
        atomicAdd(&rot, 1);
      }
      rc[tid] = cs;
      rs[tid] = sn;
      rt[tid] = tt;
      rf[tid] = f;
    }
    __syncthreads();
    // G <- R^T G R and J <- J R
    int pa = 0, qa = 0, pb, qb;
    pair_of(r, k2, pb, qb);
    if (gdo) pair_of(r, k1, pa, qa);
    const double cb = rc[k2], sb = rs[k2];
    double x = 0.0, y = 0.0, g11 = 0.0, g12 = 0.0, g21 = 0.0, g22 = 0.0, ca = 1.0, sa = 0.0,
           ta = 0.0;
    int fa = 0;
    if (jdo) {
      x = J[k1 * LD + pb];
      y = J[k1 * LD + qb];
    }
    if (gdo) {
      g11 = G[pa * LD + pb];
      g12 = G[pa * LD + qb];
      g21 = G[qa * LD + pb];
      g22 = G[qa * LD + qb];
      ca = rc[k1];
      sa = rs[k1];
      ta = rt[k1];
      fa = rf[k1];
    }
    if (jdo) {
      J[k1 * LD + pb] = cb * x - sb * y;
      J[k1 * LD + qb] = sb * x + cb * y;
    }
    if (gdo) {
      double n11, n12, n21, n22;
      if (k1 == k2) {
        // the pair's own block: stable diagonal, off-diagonal zeroed
        n11 = g11 - ta * g12;
        n22 = g22 + ta * g12;
        n12 = fa ? 0.0 : g12;
        n21 = n12;
      } else {
        // columns (pb, qb) rotated, then rows (pa, qa)
        const double h11 = cb * g11 - sb * g12, h12 = sb * g11 + cb * g12;
        const double h21 = cb * g21 - sb * g22, h22 = sb * g21 + cb * g22;
        n11 = ca * h11 - sa * h21;
        n21 = sa * h11 + ca * h21;
        n12 = ca * h12 - sa * h22;
        n22 = sa * h12 + ca * h22;
      }
      // the mirrored entries too (for the own block the same addresses,
      // written with the same values)
      G[pa * LD + pb] = n11;
      G[pb * LD + pa] = n11;
      G[pa * LD + qb] = n12;
      G[qb * LD + pa] = n12;
      G[qa * LD + pb] = n21;
      G[pb * LD + qa] = n21;
      G[qa * LD + qb] = n22;
      G[qb * LD + qa] = n22;
    }
    __syncthreads();
  }
  const int total = rot;
  if (total == 0) return;  // J = I: columns and V unchanged
  svg_apply_j<NC>(Xs, J, mp, wave, lane);
  __syncthreads();
  svg_unstage<NC>(D.W, Xs, m, colidx, tid);
  if (ACC && D.accumulate) {
    // V[:, cols] (n x NC) <- V[:, cols] J through the same LDS rows (n <= m)
    __syncthreads();
    if (vreg) {
#pragma unroll
      for (int u = 0; u < VREG; ++u) {
        const int idx = tid + u * SVG_THREADS;
        if (idx < np16 * NC) {
          const int c = idx / np16, i = idx - c * np16;
          Xs[i * LD + c] = vr[u];
        }
      }
    } else {
      svg_stage<NC, 8>(Xs, D.V, n, np16, colidx, tid);
    }
    __syncthreads();
    svg_apply_j<NC>(Xs, J, np16, wave, lane);
    __syncthreads();
    svg_unstage<NC>(D.V, Xs, n, colidx, tid);
  }
  if (tid == 0) atomicAdd(D.count, total);
}

// LDS of a k_svg_round<nc> launch for matrices of at most m rows: the
// row-major block, G, J and the second half's G
size_t svg_lds(int nc, int m) {
  const size_t mp = (size_t)((m + 15) & ~15);
  return (mp * (nc + 1) + 3 * (size_t)nc * (nc + 1)) * sizeof(double);
}

// singular values, descending order, outputs
__global__ __launch_bounds__(SV_THREADS) void k_sv_finish(SvBatch B) {
  extern __shared__ double lds[];
  const SvMat &D = B.d[blockIdx.x];
  const int m = D.m, n = D.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double *sig = lds;
  int *rank = (int *)(lds + n);
  for (int j = wave; j < n; j += SV_WAVES) {
    const double *wj = D.W + (int64_t)j * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += wj[i] * wj[i];
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += SV_THREADS) {
    const double sj = sig[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig[i];
      r += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
    rank[j] = r;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += SV_THREADS) D.S[rank[j]] = sig[j];
  for (int64_t idx = threadIdx.x; idx < (int64_t)m * n; idx += SV_THREADS) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    const double s = sig[j];
    D.U[i * D.urs + rank[j] * D.ucs] = (s > 0.0) ? D.W[idx] / s : 0.0;
  }
  if (D.accumulate)
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += SV_THREADS) {
      const int i = (int)(idx % n), j = (int)(idx / n);
      D.Vout[i * D.vrs + rank[j] * D.vcs] = D.V[idx];
    }
}

// dynamic LDS available to k_sv_round: the device's per-workgroup maximum
// minus the kernel's static LDS (opted in once per process)
size_t g_lds_limit = 0;

std::mutex g_lds_mutex;

size_t sv_lds_limit(Ctx &c) {
  std::lock_guard<std::mutex> lock(g_lds_mutex);
  if (g_lds_limit) return g_lds_limit;
  int maxsh = 0;
  HIPC(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device));
  size_t stat = 0;
  const void *kerns[6] = {(const void *)k_sv_round<SV_THREADS>,
                          (const void *)k_sv_round<SVB_THREADS>,
                          (const void *)k_svg_round<32, true>,
                          (const void *)k_svg_round<16, true>,
                          (const void *)k_svg_round<32, false>,
                          (const void *)k_svg_round<16, false>};
  for (const void *k : kerns) {
    hipFuncAttributes fa;
    HIPC(hipFuncGetAttributes(&fa, k));
    stat = std::max(stat, (size_t)fa.sharedSizeBytes);
  }
  size_t lim = (size_t)maxsh > stat + 256 ? (size_t)maxsh - stat - 256 : 32768;
  if (lim > 65536 - stat - 256) {
    for (const void *k : kerns)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
          hipSuccess) {
        (void)hipGetLastError();
        lim = 65536 - stat - 256;
      }
  }
  g_lds_limit = lim;
  const char *vb = std::getenv("QTT_VERBOSE");
  if (vb && vb[0] == '1')
    std::fprintf(stderr, "[qtt] svd: device LDS per workgroup %d, static %zu, dynamic limit %zu\n",
                 maxsh, stat, lim);
  return lim;
}

bool sv_verbose() {
  static const bool v = [] {
    const char *e = std::getenv("QTT_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

}  // namespace

namespace {

// dst view <- src (rows x cols, row-major packed)
__global__ void k_sv_copy_view(double *dst, int64_t drs, int64_t dcs, const double *src, int rows,
                               int cols) {
  const int64_t tot = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    dst[i * drs + j * dcs] = src[e];
  }
}

void svd_jacobi(Ctx &c, int count, const ConstMatView *A, const MatView *U, double *const *S,
                const MatView *V);

}  // namespace

// Matrices with more than SVQ_MIN columns are first brought to a square
// triangular factor by Householder QR steps, and the one-sided Jacobi runs
// on its transpose, whose columns start much closer to orthogonal than A's
// (and, for tall A, are shorter).  Each further QR of the previous R^T cuts
// the sweeps on truncation unfoldings again (16 -> 9 -> 8 on a four-term RK4
// sum), and the number of steps decides which singular vectors come out of
// the Jacobi as its normalised columns, free of accumulated rotations:
//   U and V wanted:  A = Q1 R1, X = R1^T = U_X S V_X^T, A = (Q1 V_X) S U_X^T:
//                    V = U_X, U = Q1 V_X with the rotations accumulated;
//   U only (null V): R1^T = Q2 R2, X = R2^T: A = (Q1 U_X) S (Q2 V_X)^T,
//                    U = Q1 U_X;
//   V only (null U): R2^T = Q3 R3, X = R3^T: A = (Q1 Q3 V_X) S (Q2 U_X)^T,
//                    V = Q2 U_X.
// Q factors that are not used are not formed.
constexpr int SVQ_MIN = 32;

void svd_batch(Ctx &c, int count, const ConstMatView *A, const MatView *U, double *const *S,
               const MatView *V) {
  std::vector<int> qi, di;
  for (int i = 0; i < count; ++i) {
    if (A[i].rows < A[i].cols) fail(QTT_E_SHAPE, "svd_batch: needs rows >= cols");
    if (U[i].rows != A[i].rows || U[i].cols != A[i].cols || V[i].rows != A[i].cols ||
        V[i].cols != A[i].cols)
      fail(QTT_E_SHAPE, "svd_batch: output shapes");
    if (!U[i].p && !V[i].p) fail(QTT_E_ARG, "svd_batch: neither U nor V requested");
    (A[i].cols > SVQ_MIN ? qi : di).push_back(i);
  }
  if (!di.empty()) {
    std::vector<ConstMatView> a;
    std::vector<MatView> u, v;
    std::vector<double *> s;
    int64_t scratch = 0;
    for (int i : di)
      if (!U[i].p) scratch += (int64_t)A[i].rows * A[i].cols;
    double *Us = scratch ? c.buf("svd_Uscratch", scratch) : nullptr;
    for (int i : di) {
      a.push_back(A[i]);
      if (U[i].p) {
        u.push_back(U[i]);
      } else {
        u.push_back(MatView{Us, A[i].rows, A[i].cols, A[i].cols, 1});
        Us += (int64_t)A[i].rows * A[i].cols;
      }
      v.push_back(V[i]);
      s.push_back(S[i]);
    }
    svd_jacobi(c, (int)di.size(), a.data(), u.data(), s.data(), v.data());
  }
  if (qi.empty()) return;
  const int cnt = (int)qi.size();
  // number of QR steps per matrix (1: U and V, 2: U only, 3: V only)
  std::vector<int> steps(cnt);
  int64_t qs = 0, ns = 0;
  for (int k = 0; k < cnt; ++k) {
    const int i = qi[k];
    steps[k] = (U[i].p && V[i].p) ? 1 : (U[i].p ? 2 : 3);
    qs += (int64_t)A[i].rows * A[i].cols;
    ns += (int64_t)A[i].cols * A[i].cols;
  }
  double *Qb = c.buf("svq_Q", qs);     // Q1 (steps 1, 2)
  double *Q2b = c.buf("svq_Q2", ns);   // Q2 (step 3)
  double *Rb[2] = {c.buf("svq_R", ns), c.buf("svq_R2", ns)};  // R factors, ping-pong
  double *UXb = c.buf("svq_UX", ns);
  double *VXb = c.buf("svq_VX", ns);
  std::vector<int64_t> qo(cnt), no(cnt);
  {
    int64_t o1 = 0, o2 = 0;
    for (int k = 0; k < cnt; ++k) {
      qo[k] = o1;
      no[k] = o2;
      o1 += (int64_t)A[qi[k]].rows * A[qi[k]].cols;
      o2 += (int64_t)A[qi[k]].cols * A[qi[k]].cols;
    }
  }
  // QR step t (0-based) of every matrix that takes it; R of step t goes to Rb[t % 2]
  for (int t = 0; t < 3; ++t) {
    std::vector<ConstMatView> a;
    std::vector<MatView> q, r;
    for (int k = 0; k < cnt; ++k) {
      if (steps[k] <= t) continue;
      const int i = qi[k];
      const int m = A[i].rows, n = A[i].cols;
      double *R = Rb[t % 2] + no[k];
      if (t == 0) {
        a.push_back(A[i]);
        q.push_back(MatView{steps[k] <= 2 ? Qb + qo[k] : nullptr, m, n, n, 1});
      } else {
        a.push_back(ConstMatView{Rb[(t - 1) % 2] + no[k], n, n, 1, n});  // previous R^T
        q.push_back(MatView{(t == 1 && steps[k] == 3) ? Q2b + no[k] : nullptr, n, n, n, 1});
      }
      r.push_back(MatView{R, n, n, n, 1});
    }
    if (!a.empty()) qr_batch(c, (int)a.size(), a.data(), q.data(), r.data());
  }
  // one Jacobi batch over all of them: X = (last R)^T
  std::vector<ConstMatView> x;
  std::vector<MatView> ux, vx;
  std::vector<double *> s;
  for (int k = 0; k < cnt; ++k) {
    const int n = A[qi[k]].cols;
    x.push_back(ConstMatView{Rb[(steps[k] - 1) % 2] + no[k], n, n, 1, n});
    ux.push_back(MatView{UXb + no[k], n, n, n, 1});
    vx.push_back(MatView{steps[k] == 1 ? VXb + no[k] : nullptr, n, n, n, 1});
    s.push_back(S[qi[k]]);
  }
  svd_jacobi(c, cnt, x.data(), ux.data(), s.data(), vx.data());
  for (int k = 0; k < cnt; ++k) {
    const int i = qi[k];
    const int m = A[i].rows, n = A[i].cols;
    if (steps[k] == 1) {
      // V = U_X (copied into the caller's view)
      int64_t lo = 0, hi = 0;
      span(lo, hi, n, V[i].rs);
      span(lo, hi, n, V[i].cs);
      c.check_range(V[i].p, lo, hi, 8, "svd V");
      c.check_range(ux[k].p, 0, (int64_t)n * n - 1, 8, "svd UX");
      const unsigned g = (unsigned)std::min<int64_t>(1024, ((int64_t)n * n + 255) / 256);
      hipLaunchKernelGGL(k_sv_copy_view, dim3(g), dim3(256), 0, c.stream, V[i].p, V[i].rs,
                         V[i].cs, (const double *)ux[k].p, n, n);
      HIPC(hipGetLastError());
    }
    Gemm gq;  // U = Q1 V_X (1 step), U = Q1 U_X (2), V = Q2 U_X (3)
    gq.K = n;
    gq.N = n;
    gq.sAk = 1;
    gq.sBn = 1;
    gq.sBk = n;
    if (steps[k] == 3) {
      gq.M = n;
      gq.A = Q2b + no[k];
      gq.sAm = n;
      gq.B = ux[k].p;
      gq.C = V[i].p;
      gq.sCm = V[i].rs;
      gq.sCn = V[i].cs;
    } else {
      gq.M = m;
      gq.A = Qb + qo[k];
      gq.sAm = n;
      gq.B = steps[k] == 1 ? vx[k].p : ux[k].p;
      gq.C = U[i].p;
      gq.sCm = U[i].rs;
      gq.sCn = U[i].cs;
    }
    gemm(c, gq);
  }
}

namespace {

void svd_jacobi_group(Ctx &c, int count, const ConstMatView *A, const MatView *U,
                      double *const *S, const MatView *V, bool single_group) {
  const size_t SV_LDS_LIMIT = sv_lds_limit(c);
  for (int base = 0; base < count; base += SV_MAXB) {
    const int cnt = std::min(SV_MAXB, count - base);
    SvBatch B{};
    B.count = cnt;
    int64_t ws = 0;
    // blocked matrices take the Gram-matrix rounds when the tallest of the
    // launch fits LDS with 32 (else 16) column slots
    int gram_nc = 0;
    if (!single_group) {
      int mmax = 0;
      for (int i = 0; i < cnt; ++i) mmax = std::max(mmax, A[base + i].rows);
      if (svg_lds(32, mmax) <= SV_LDS_LIMIT) gram_nc = 32;
      else if (svg_lds(16, mmax) <= SV_LDS_LIMIT) gram_nc = 16;
    }
    size_t lds_round = 0, lds_fin = 0;
    for (int i = 0; i < cnt; ++i) {
      const ConstMatView &a = A[base + i];
      const int m = a.rows, n = a.cols;
      if (m < n) fail(QTT_E_SHAPE, "svd_batch: needs rows >= cols");
      if (U[base + i].rows != m || U[base + i].cols != n || V[base + i].rows != n ||
          V[base + i].cols != n)
        fail(QTT_E_SHAPE, "svd_batch: output shapes");
      {
        int64_t lo = 0, hi = 0;
        span(lo, hi, a.rows, a.rs);
        span(lo, hi, a.cols, a.cs);
        c.check_range(a.p, lo, hi, 8, "svd A");
        lo = hi = 0;
        span(lo, hi, U[base + i].rows, U[base + i].rs);
        span(lo, hi, U[base + i].cols, U[base + i].cs);
        c.check_range(U[base + i].p, lo, hi, 8, "svd U");
        if (V[base + i].p) {
          lo = hi = 0;
          span(lo, hi, V[base + i].rows, V[base + i].rs);
          span(lo, hi, V[base + i].cols, V[base + i].cs);
          c.check_range(V[base + i].p, lo, hi, 8, "svd V");
        }
        c.check_range(S[base + i], 0, n - 1, 8, "svd S");
      }
      // one block pair when the whole matrix fits LDS, else blocks of SV_BQ
      // (Gram rounds: NC / 2 for the whole launch)
      const bool one = n <= SV_SINGLE && (size_t)n * (m + n) * 8 <= SV_LDS_LIMIT;
      if (one != single_group) fail(QTT_E_ARG, "svd_batch: block-pair grouping");
      int b = one ? (n + 1) / 2 : (gram_nc ? gram_nc / 2 : SV_BQ);
      while (!one && !gram_nc && b > 4 && (size_t)(2 * b) * (m + 2 * b) * 8 > SV_LDS_LIMIT)
        b /= 2;
      if (!one && !gram_nc && (size_t)(2 * b) * (m + 2 * b) * 8 > SV_LDS_LIMIT)
        fail(QTT_E_UNSUPPORTED, "svd_batch: matrix too tall");
      SvMat &d = B.d[i];
      d.A = a.p;
      d.m = m;
      d.n = n;
      d.ars = a.rs;
      d.acs = a.cs;
      d.b = b;
      d.nb = (n + b - 1) / b;
      d.single = (n <= 2 * b) ? 1 : 0;
      if (d.single) d.nb = 1;
      d.U = U[base + i].p;
      d.urs = U[base + i].rs;
      d.ucs = U[base + i].cs;
      d.S = S[base + i];
      d.Vout = V[base + i].p;
      d.accumulate = V[base + i].p ? 1 : 0;
      d.vrs = V[base + i].rs;
      d.vcs = V[base + i].cs;
      ws += (int64_t)m * n + (int64_t)n * n + 1;
      const int nc = d.single ? n : 2 * b;
      lds_round = std::max(lds_round, gram_nc ? svg_lds(gram_nc, m) : (size_t)nc * (m + nc) * 8);
      lds_fin = std::max(lds_fin, (size_t)(2 * n + 4) * 8);
    }
    double *Wb = c.buf("svd_work", ws);
    int *cnt_host = (int *)(c.pinned + 2048);
    int *cnt_dev = (int *)c.raw("svd_counts", SV_MAXB * sizeof(int));
    double *fro2_dev = c.buf("svd_fro2", SV_MAXB);
    int64_t o = 0;
    for (int i = 0; i < cnt; ++i) {
      SvMat &d = B.d[i];
      d.W = Wb + o;
      o += (int64_t)d.m * d.n;
      d.V = Wb + o;
      o += (int64_t)d.n * d.n + 1;
      d.count = cnt_dev + i;
      d.fro2 = fro2_dev + i;
    }
    hipLaunchKernelGGL(k_sv_init, dim3(cnt), dim3(SV_THREADS), 0, c.stream, B);
    HIPC(hipGetLastError());
    bool acc_any = false;  // some matrix accumulates V (the round kernels' V path)
    for (int i = 0; i < cnt; ++i) acc_any = acc_any || B.d[i].accumulate;
    // rounds per sweep: the largest block count decides
    int rounds = 1;
    for (int i = 0; i < cnt; ++i)
      if (!B.d[i].single) rounds = std::max(rounds, B.d[i].nb + (B.d[i].nb & 1) - 1);
    int sweeps_run = 0;
    bool converged = false;
    for (int sweep = 0; sweep < c.svd_max_sweeps; ++sweep) {
      ++sweeps_run;
      for (int r = 0; r < rounds; ++r) {
        // workgroups of this round per matrix
        SvBatch R = B;
        int wg = 0;
        int active = 0;
        for (int i = 0; i < cnt; ++i) {
          SvMat &d = R.d[i];
          d.first = wg;
          int pairs;
          if (d.single) pairs = (r == 0) ? 1 : 0;
          else pairs = (r < d.nb + (d.nb & 1) - 1) ? (d.nb + (d.nb & 1)) / 2 : 0;
          wg += pairs;
          active += pairs;
        }
        if (active == 0) continue;
        // matrices with no work this round keep first = wg (no workgroup maps to them)
        if (single_group)
          hipLaunchKernelGGL(k_sv_round<SV_THREADS>, dim3(wg), dim3(SV_THREADS), lds_round,
                             c.stream, R, r);
        else if (gram_nc == 32 && acc_any)
          hipLaunchKernelGGL((k_svg_round<32, true>), dim3(wg), dim3(SVG_THREADS), lds_round,
                             c.stream, R, r);
        else if (gram_nc == 32)
          hipLaunchKernelGGL((k_svg_round<32, false>), dim3(wg), dim3(SVG_THREADS), lds_round,
                             c.stream, R, r);
        else if (gram_nc == 16 && acc_any)
          hipLaunchKernelGGL((k_svg_round<16, true>), dim3(wg), dim3(SVG_THREADS), lds_round,
                             c.stream, R, r);
        else if (gram_nc == 16)
          hipLaunchKernelGGL((k_svg_round<16, false>), dim3(wg), dim3(SVG_THREADS), lds_round,
                             c.stream, R, r);
        else
          hipLaunchKernelGGL(k_sv_round<SVB_THREADS>, dim3(wg), dim3(SVB_THREADS), lds_round,
                             c.stream, R, r);
        HIPC(hipGetLastError());
      }
      HIPC(hipMemcpyAsync(cnt_host, cnt_dev, cnt * sizeof(int), hipMemcpyDeviceToHost, c.stream));
      c.sync();
      bool done = true;
      for (int i = 0; i < cnt; ++i) done = done && (cnt_host[i] == 0);
      if (done) {
        converged = true;
        break;
      }
      HIPC(hipMemsetAsync(cnt_dev, 0, cnt * sizeof(int), c.stream));
    }
    // rotations still pending at the cap: the factors are used as they are
    // and the call reports QTT_W_SVD_MAXIT
    if (!converged) c.warn = std::max(c.warn, (int)QTT_W_SVD_MAXIT);
    if (sv_verbose())
      std::fprintf(stderr, "[qtt] svd %dx%d (+%d) sweeps %d rounds/sweep %d gram %d\n", B.d[0].m,
                   B.d[0].n, cnt - 1, sweeps_run, rounds, gram_nc);
    hipLaunchKernelGGL(k_sv_finish, dim3(cnt), dim3(SV_THREADS), lds_fin, c.stream, B);
    HIPC(hipGetLastError());
  }
}

// matrices that are one block pair and those split into blocks take different
// round kernels: run them as two groups
void svd_jacobi(Ctx &c, int count, const ConstMatView *A, const MatView *U, double *const *S,
                const MatView *V) {
  const size_t lim = sv_lds_limit(c);
  std::vector<int> ids[2];
  for (int i = 0; i < count; ++i) {
    const int m = A[i].rows, n = A[i].cols;
    const bool one = n <= SV_SINGLE && (size_t)n * (m + n) * 8 <= lim;
    ids[one ? 0 : 1].push_back(i);
  }
  for (int g = 0; g < 2; ++g) {
    if (ids[g].empty()) continue;
    std::vector<ConstMatView> a;
    std::vector<MatView> u, v;
    std::vector<double *> s;
    for (int i : ids[g]) {
      a.push_back(A[i]);
      u.push_back(U[i]);
      v.push_back(V[i]);
      s.push_back(S[i]);
    }
    svd_jacobi_group(c, (int)a.size(), a.data(), u.data(), s.data(), v.data(), g == 0);
  }
}

}  // namespace

}  // namespace qtt
