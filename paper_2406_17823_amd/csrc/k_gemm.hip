// Strided, batched and grouped GEMM on CDNA4 matrix cores.
//
// Every tensor-network contraction of the library (environment updates,
// local right-hand sides, the penalty matvec, QR/SVD factor products) is
// expressed as C[b1,b2](m,n) = alpha sum_k A(m,k) B(k,n) + beta X with
// arbitrary element strides, so that no tensor is ever transposed in HBM.
// One launch carries up to GEMM_GROUP independent problems (the four penalty
// pair terms of a CG matvec go out as one launch per step).
//
// Tiling: a workgroup owns a BM x BN output tile, 128 x 128 (512 threads,
// 2 x 4 wave64s) when the launch has at least one such tile per compute
// unit, else 64 x 64 (256 threads, 2 x 2); each wave holds 16 x 16 MFMA
// blocks.  K is staged through LDS in slices of KD = 32 (128-tiles) or 16
// (64-tiles) rows with two LDS buffers: the next slice's global loads are
// issued into registers before the current slice's MFMAs, so one barrier per
// slice suffices, and the deeper slice gives the loads of the large tiles
// twice the MFMA time to arrive.  The
// loader picks the thread-to-element map from the operand's unit-stride
// dimension so that global loads stay coalesced.  float32 slices are laid
// out for vector fragment reads (each lane reads its operands of all the
// wave's MFMA blocks in one 8- or 16-byte LDS read) with row offsets that
// keep the reads and the transposed stores free of bank conflicts; the
// other types read one element per block from rows padded by one element.
// float64: v_mfma_f64_16x16x4_f64; float32: v_mfma_f32_16x16x4_f32 with
// float64 operands rounded to float32 on the way into LDS and float32
// accumulation over the tile's K range; bfloat16: v_mfma_f32_16x16x16_bf16;
// compensated split bfloat16 (each operand as hi + lo bfloat16, three MFMAs
// per block dropping lo*lo, float32 accumulation over the tile's K range).
// Split-K partial tiles are summed in float64.
// When the output tiles cannot fill the 256 compute units, K is split across
// workgroups; the partial tiles are summed in split order by a second kernel
// (deterministic).  That kernel also sums several problems into one output
// (the two pair terms j = 1, 2 of y_i) and adds a separate input X.
#include "qtt_internal.h"
#include "qtt_cg.h"

#include <cstdio>
#include <type_traits>

namespace qtt {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));

// compensated split bfloat16 operand: v ~ hi + lo, both bfloat16 (16
// significant bits in all); products take hi*hi + hi*lo + lo*hi
struct bf3 {
  __bf16 hi, lo;
};

template <typename T> struct GemmKind;
template <> struct GemmKind<double> { static constexpr int value = 0; };
template <> struct GemmKind<float> { static constexpr int value = 1; };
template <> struct GemmKind<__bf16> { static constexpr int value = 2; };
template <> struct GemmKind<bf3> { static constexpr int value = 3; };

// accumulator of a 16 x 16 MFMA block: float32 for the float32 and split
// bfloat16 MFMAs, float64 otherwise (plain bfloat16 products are summed in
// float32 per 16-deep step and in float64 across steps)
template <typename T> struct AccOf { typedef d4v type; };
template <> struct AccOf<float> { typedef f4v type; };
template <> struct AccOf<bf3> { typedef f4v type; };

namespace {

constexpr int KT = 16, PADM = 1;

struct Prob {
  int M, N, K, B1, B2, tm, tn, ksplit, kchunk, direct;
  int64_t block0;
  const double *A;
  int64_t sAm, sAk, sAb1, sAb2;
  const double *B;
  int64_t sBk, sBn, sBb1, sBb2;
  double *C;  // direct mode: C = alpha acc + beta C
  int64_t sCm, sCn, sCb1, sCb2;
  double alpha, beta;
  double *part;  // partial mode: part[ks][b][m][n]
  int c32;  // result stored as float32 (operand storage is a template argument)
  // A / B qualify for 16-byte vector loads along their unit-stride dimension:
  // that dimension's extent, the other strides and the base are multiples of
  // the vector (so a vector lies wholly inside or wholly outside the operand)
  int va, vb;
  const double *Bw, *Bs;  // CG operand: B read as B - alpha (Bw + beta Bs)
};

struct GemmK {
  int np;
  Prob p[GEMM_GROUP];
  const int *skip;
  double *flop_ctr;
  double flops;
  const CGState *cgst;  // alpha and beta of the CG operand
};

// one KT-deep slice of MFMAs for a wave's FM x FN blocks of 16 x 16
template <typename T, int FM, int FN, int LD>
struct Mfma;

template <int FM, int FN, int LD>
struct Mfma<double, FM, FN, LD> {
  __device__ static void step(const double (*As)[LD], const double (*Bs)[LD], int lane, int m0,
                              int n0, d4v (&acc)[FM][FN]) {
#pragma unroll
    for (int kq = 0; kq < KT / 4; ++kq) {
      const int kk = kq * 4 + (lane >> 4);
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[kk][m0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[kk][n0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
};

// float32 and split-bfloat16 operand slices (4-byte elements) in LDS are
// read as vector fragments: lane l supplies the V = FM (or FN) consecutive
// columns V (l % 16) .. V (l % 16) + V - 1 of a row, one per MFMA block
// (block i takes wave-tile row V r + i as its row r), in one 8- or 16-byte
// LDS read.  Row k starts at word (k / 2) PP + (k % 2) PO:
//   V = 4: PO = W + 4, PP = 2 PO (rows padded by 4 words): a 16-byte read of
//          16 lanes covers one row, and the transposed stores of a
//          k-contiguous operand (consecutive threads, consecutive rows) spread
//          over the banks;
//   V = 2: the 8-byte reads of 32 lanes take two rows, k and k + KS (KS = 1
//          for the float32 MFMA, whose lane groups step one row; 4 for the
//          bfloat16 MFMA, whose lane groups step four): PO = 32 and PP = 2
//          modulo 64 banks (KS = 1), or PO = 8 and PP = 16 (KS = 4), put the
//          two rows on the two bank halves, and the rows of a transposed store
//          on different banks (two to a bank at most).
// Other element types: rows of W + 1 elements (PO = W + 1, PP = 2 PO).
// The row part of an access is a per-lane row plus an even compile-time row
// step (or an even per-lane row plus a compile-time one), which adds a
// compile-time word offset.
template <int W, int V, bool FRAG, int KS = 1>
struct Lay {
  static constexpr int up(int x, int r) { return (x - r + 63) / 64 * 64 + r; }  // >= x, = r mod 64
  static constexpr int PO = !FRAG ? W + 1 : V == 4 ? W + 4 : up(W, KS == 1 ? 32 : 8);
  static constexpr int PP = !FRAG || V == 4 ? 2 * PO : up(PO + W, KS == 1 ? 2 : 16);
  static_assert(!FRAG || V == 2 || V == 4, "fragments of two or four elements");
  static_assert(KS == 1 || KS == 4, "row step of the MFMA lane groups");
  static_assert(PO >= W && PP >= PO + W, "rows do not overlap");
  __device__ __forceinline__ static int row(int k) { return (k >> 1) * PP + (k & 1) * PO; }
  static constexpr int words(int kd) { return (kd / 2) * PP; }
};

template <int V>
__device__ __forceinline__ void frag_load(const float *p, float (&v)[V]) {
  typedef float fv __attribute__((ext_vector_type(V)));
  const fv x = *reinterpret_cast<const fv *>(p);
#pragma unroll
  for (int e = 0; e < V; ++e) v[e] = x[e];
}

// float32: the accumulators stay float32 over the whole K range of the
// tile (float32 accumulation, as the mixed mode prescribes); split-K
// partials are summed in float64 by the reduction kernel.  As, Bs: the
// slice buffers; kb: the first slice row of this step
template <int FM, int FN, int BM, int BN>
struct MfmaF32 {
  typedef Lay<BM, FM, true> LA;
  typedef Lay<BN, FN, true> LB;
  __device__ static void step(const float *As, const float *Bs, int lane, int m0, int n0, int kb,
                              f4v (&acc)[FM][FN]) {
    // lane terms: row lane / 16 of each group of four, the lane's columns
    const float *ap = As + LA::row(lane >> 4) + m0 + FM * (lane & 15);
    const float *bp = Bs + LB::row(lane >> 4) + n0 + FN * (lane & 15);
#pragma unroll
    for (int kq = 0; kq < KT / 4; ++kq) {
      float a[FM], b[FN];
      frag_load<FM>(ap + ((kb + kq * 4) >> 1) * LA::PP, a);
      frag_load<FN>(bp + ((kb + kq * 4) >> 1) * LB::PP, b);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
};

// bfloat16 operands, float32 accumulation (v_mfma_f32_16x16x16_bf16): lane l
// holds A[l % 16][4 (l / 16) + 0..3] and B[4 (l / 16) + 0..3][l % 16]
template <int FM, int FN, int LD>
struct Mfma<__bf16, FM, FN, LD> {
  __device__ static void step(const __bf16 (*As)[LD], const __bf16 (*Bs)[LD], int lane, int m0,
                              int n0, d4v (&acc)[FM][FN]) {
    b4v a[FM], b[FN];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = 4 * (lane >> 4) + e;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i][e] = As[kk][m0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j][e] = Bs[kk][n0 + j * 16 + (lane & 15)];
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const f4v f = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], f4v{0.f, 0.f, 0.f, 0.f},
                                                                0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)f[r];
      }
  }
};

// compensated split bfloat16: three v_mfma_f32_16x16x16_bf16 per block
// (lo*hi, hi*lo, then hi*hi), accumulated in float32 over the whole K range
// of the tile like the float32 MFMAs
template <int FM, int FN, int LD>
struct Mfma<bf3, FM, FN, LD> {
  __device__ static void step(const bf3 (*As)[LD], const bf3 (*Bs)[LD], int lane, int m0, int n0,
                              f4v (&acc)[FM][FN]) {
    b4v ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = 4 * (lane >> 4) + e;
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const bf3 v = As[kk][m0 + i * 16 + (lane & 15)];
        ah[i][e] = v.hi;
        al[i][e] = v.lo;
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf3 v = Bs[kk][n0 + j * 16 + (lane & 15)];
        bh[j][e] = v.hi;
        bl[j][e] = v.lo;
      }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
};

// split bfloat16 from fragments: lane l takes rows 4 (l / 16) + e, e = 0..3,
// of the 16-row step, each as one fragment of V bf3 words
template <int FM, int FN, int BM, int BN>
struct MfmaBf3F {
  typedef Lay<BM, FM, true, 4> LA;
  typedef Lay<BN, FN, true, 4> LB;
  template <int V>
  __device__ static void frag(const bf3 *p, b4v (&h)[V], b4v (&l)[V], int e) {
    typedef unsigned uv __attribute__((ext_vector_type(V)));
    const uv x = *reinterpret_cast<const uv *>(p);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const bf3 v = __builtin_bit_cast(bf3, (unsigned)x[i]);
      h[i][e] = v.hi;
      l[i][e] = v.lo;
    }
  }
  __device__ static void step(const bf3 *As, const bf3 *Bs, int lane, int m0, int n0, int kb,
                              f4v (&acc)[FM][FN]) {
    // row kb + 4 q + e: (kb / 2 + 2 q) PP + row(e), kb + 4 q even
    const int q = lane >> 4;
    const bf3 *ap = As + (kb / 2 + 2 * q) * LA::PP + m0 + FM * (lane & 15);
    const bf3 *bp = Bs + (kb / 2 + 2 * q) * LB::PP + n0 + FN * (lane & 15);
    b4v ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      frag<FM>(ap + LA::row(e), ah, al, e);
      frag<FN>(bp + LB::row(e), bh, bl, e);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
};

template <typename T>
__device__ inline T to_op(double v) {
  return (T)v;
}
template <>
__device__ inline __bf16 to_op<__bf16>(double v) {
  return (__bf16)(float)v;
}
template <>
__device__ inline bf3 to_op<bf3>(double v) {
  bf3 r;
  r.hi = (__bf16)(float)v;
  r.lo = (__bf16)(float)(v - (double)(float)r.hi);
  return r;
}

// WGM x WGN waves per workgroup, each owning (BM / WGM) x (BN / WGN) outputs;
// K goes through LDS in slices of KD (16 or 32) rows, each consumed as
// KD / 16 MFMA steps of 16: the float32 / bfloat16 partial sums stay 16 deep
// and float64 MFMAs accumulate in k order, so KD changes no result bit
// SA, SB: storage types of A and B (float64, or float32 for the convection
// networks of the mixed mode, with T = float); the operand words go through
// registers in their storage type and are converted on the way into LDS.
// BCG: B is the next CG residual r - alpha (w + beta s), formed as it loads
// VEC: every problem's A and B qualify for 16-byte loads (Prob::va, vb): a
// thread loads whole vectors along each operand's unit-stride dimension
template <typename T, int BM, int BN, int WGM, int WGN, int KD, typename SA = double,
          typename SB = double, bool BCG = false, bool VEC = false>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gemm(GemmK g) {
  if (g.skip && *g.skip) return;
  double cg_a = 0.0, cg_b = 0.0;
  bool cg_first = false;
  if constexpr (BCG) {
    const double gm = g.cgst->gamma, dl = g.cgst->delta;
    cg_first = g.cgst->first != 0;
    cg_b = cg_first ? 0.0 : gm / g.cgst->gamma_prev;
    cg_a = cg_first ? gm / dl : gm / (dl - cg_b * gm / g.cgst->alpha_prev);
  }
  if (g.flop_ctr && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(g.flop_ctr, g.flops);
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;  // wave tile
  constexpr int FM = WTM / 16, FN = WTN / 16;    // 16 x 16 blocks per wave
  constexpr int AL = BM * KD / NTHR, BL = BN * KD / NTHR;  // global loads per thread
  static_assert(BM == BN, "square tiles: the MFMA step takes one LDS pitch");
  static_assert(KD % KT == 0, "slices of whole MFMA steps");
  static_assert(AL * NTHR == BM * KD && BL * NTHR == BN * KD, "tile / thread mismatch");
  // float32: the fragment layout above; other types: rows padded by one
  // element, read element-wise
  constexpr bool BF3 = std::is_same<T, bf3>::value;
  constexpr bool FRAG = std::is_same<T, float>::value || BF3;
  constexpr int VFA = BM / WGM / 16, VFB = BN / WGN / 16;  // fragment lengths
  constexpr int LDA = BM + PADM, LDB = BN + PADM;
  typedef Lay<BM, VFA, FRAG, BF3 ? 4 : 1> LA;
  typedef Lay<BN, VFB, FRAG, BF3 ? 4 : 1> LB;
  static_assert(FRAG || (LA::PO == LDA && LB::PO == LDB), "padded rows of the element-wise types");
  __shared__ __align__(16) T As[2][LA::words(KD)];
  __shared__ __align__(16) T Bs[2][LB::words(KD)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  int pi = 0;
#pragma unroll
  for (int i = 1; i < GEMM_GROUP; ++i)
    if (i < g.np && (int64_t)blockIdx.x >= g.p[i].block0) pi = i;
  const Prob &P = g.p[pi];

  int64_t bid = (int64_t)blockIdx.x - P.block0;
  // every problem starts at a multiple of 8 blocks; the padding blocks after
  // a problem's last tile have nothing to do
  const int64_t ptotal = (int64_t)P.tm * P.tn * P.ksplit * P.B1 * P.B2;
  if (bid >= ptotal) return;
  // workgroups are dealt round-robin to the 8 XCDs (each with its own L2),
  // so renumber each problem's blocks such that every XCD walks a contiguous
  // range of its tiles, N-tile fastest: the tiles sharing an A row panel then
  // run back to back on one XCD and read it from its L2
  const bool xcd = (P.tn > 1);
  if (xcd) {
    const int64_t l8 = ptotal & ~(int64_t)7;
    if (bid < l8) bid = (bid & 7) * (l8 >> 3) + (bid >> 3);
  }
  const int tiles = P.tm * P.tn;
  const int t = (int)(bid % tiles);
  int64_t bb = bid / tiles;
  const int ks = (int)(bb % P.ksplit);
  bb /= P.ksplit;
  const int b1 = (int)(bb % P.B1);
  const int b2 = (int)(bb / P.B1);
  const int kbeg = ks * P.kchunk;
  const int kend = min(P.K, kbeg + P.kchunk);
  const int m0 = (xcd ? (t / P.tn) : (t % P.tm)) * BM;
  const int n0 = (xcd ? (t % P.tn) : (t / P.tm)) * BN;

  // element offsets into the operands' storage arrays
  const int64_t aoff = b1 * P.sAb1 + b2 * P.sAb2, boff = b1 * P.sBb1 + b2 * P.sBb2;
  const SA *Ap = reinterpret_cast<const SA *>(P.A);
  const SB *Bp = reinterpret_cast<const SB *>(P.B);
  const bool a_m_unit = (P.sAm == 1);
  const bool b_n_unit = (P.sBn == 1);

  typename AccOf<T>::type acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  // load slot i of a thread covers element (mm0 + dm i, kk0 + dk i) of the
  // slice: the thread's first element and a slot step that are fixed for
  // the whole K loop (consecutive threads along the operand's unit-stride
  // dimension).  With HOIST the per-slice address is base + i * step + k0 *
  // sk from per-thread bases kept in registers; the float32 128-tile, whose
  // two workgroups per compute unit need it under 128 registers, recomputes
  // the offsets instead.
  static_assert(NTHR % BM == 0 && NTHR % BN == 0 && NTHR % KD == 0, "slot map");
  constexpr bool HOIST = !(BM == 128 && GemmKind<T>::value == 1);
  const int a_mm0 = a_m_unit ? tid % BM : tid / KD, a_kk0 = a_m_unit ? tid / BM : tid % KD;
  const int a_dm = a_m_unit ? 0 : NTHR / KD, a_dk = a_m_unit ? NTHR / BM : 0;
  const int b_nn0 = b_n_unit ? tid % BN : tid / KD, b_kk0 = b_n_unit ? tid / BN : tid % KD;
  const int b_dn = b_n_unit ? 0 : NTHR / KD, b_dk = b_n_unit ? NTHR / BN : 0;
  int64_t a_base = 0, a_step = 0, b_base = 0, b_step = 0;
  if constexpr (HOIST) {
    a_base = aoff + (int64_t)(m0 + a_mm0) * P.sAm + (int64_t)a_kk0 * P.sAk;
    a_step = (int64_t)a_dm * P.sAm + (int64_t)a_dk * P.sAk;
    b_base = boff + (int64_t)(n0 + b_nn0) * P.sBn + (int64_t)b_kk0 * P.sBk;
    b_step = (int64_t)b_dn * P.sBn + (int64_t)b_dk * P.sBk;
  }
  SA ra[AL];
  SB rb[BL];
  // vector maps: a thread loads VA (VB) consecutive elements along the
  // unit-stride dimension in AL / VA (BL / VB) slots stepping along the other
  // one; m (n) unit-stride: thread -> (vector column, k row), k unit-stride:
  // thread -> (vector along k, m column)
  constexpr int VA = 16 / sizeof(SA), VB = 16 / sizeof(SB);
  constexpr int AV = AL / VA, BV = BL / VB;
  static_assert(!VEC || (AV * VA == AL && BV * VB == BL), "vector slots");
  static_assert(!VEC || (NTHR % (BM / VA) == 0 && NTHR % (KD / VA) == 0 &&
                         NTHR % (BN / VB) == 0 && NTHR % (KD / VB) == 0),
                "vector slot map");
  typedef SA VecA __attribute__((ext_vector_type(VA)));
  typedef SB VecB __attribute__((ext_vector_type(VB)));
  const int va_u = a_m_unit ? (tid % (BM / VA)) * VA : (tid % (KD / VA)) * VA;
  const int va_o = a_m_unit ? tid / (BM / VA) : tid / (KD / VA);
  const int va_d = a_m_unit ? NTHR * VA / BM : NTHR * VA / KD;
  const int vb_u = b_n_unit ? (tid % (BN / VB)) * VB : (tid % (KD / VB)) * VB;
  const int vb_o = b_n_unit ? tid / (BN / VB) : tid / (KD / VB);
  const int vb_d = b_n_unit ? NTHR * VB / BN : NTHR * VB / KD;
  // vector loads: per-thread base pointers and uniform slot steps set up
  // once, the problem's fields in registers (not re-read from the kernel
  // arguments inside the K loop)
  const int PM = P.M, PN = P.N;
  const int64_t sAk = P.sAk, sBk = P.sBk;
  const SA *va_p = Ap + aoff + (int64_t)(m0 + (a_m_unit ? va_u : va_o)) * P.sAm +
                   (int64_t)(a_m_unit ? va_o : va_u) * sAk;
  const int64_t vb_e = boff + (int64_t)(n0 + (b_n_unit ? vb_u : vb_o)) * P.sBn +
                       (int64_t)(b_n_unit ? vb_o : vb_u) * sBk;  // element offset
  const SB *vb_p = Bp + vb_e;
  const double *cg_w = P.Bw + vb_e, *cg_s = P.Bs + vb_e;  // CG operand (BCG)
  const int64_t va_s = (int64_t)va_d * (a_m_unit ? sAk : P.sAm);
  const int64_t vb_s = (int64_t)vb_d * (b_n_unit ? sBk : P.sBn);
  auto gload = [&](int k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < AV; ++i) {
        const int gm = m0 + (a_m_unit ? va_u : va_o + va_d * i);
        const int gk = k0 + (a_m_unit ? va_o + va_d * i : va_u);
        VecA v = VecA(SA(0));
        if (gm < PM && gk < kend)
          v = *reinterpret_cast<const VecA *>(va_p + i * va_s + (int64_t)k0 * sAk);
#pragma unroll
        for (int e = 0; e < VA; ++e) ra[i * VA + e] = v[e];
      }
#pragma unroll
      for (int i = 0; i < BV; ++i) {
        const int gn = n0 + (b_n_unit ? vb_u : vb_o + vb_d * i);
        const int gk = k0 + (b_n_unit ? vb_o + vb_d * i : vb_u);
        VecB v = VecB(SB(0));
        if (gn < PN && gk < kend) {
          const int64_t o = i * vb_s + (int64_t)k0 * sBk;
          v = *reinterpret_cast<const VecB *>(vb_p + o);
          if constexpr (BCG) {
            // the CG operand: B - alpha (w + beta s), w and s laid out like B
            // (fused multiply-adds spelled out: the same roundings as the
            // element-wise form below)
            const VecB w = *reinterpret_cast<const VecB *>(cg_w + o);
            VecB sv = w;
            if (!cg_first) sv = *reinterpret_cast<const VecB *>(cg_s + o);
#pragma unroll
            for (int e = 0; e < VB; ++e)
              v[e] = __builtin_fma(-cg_a, cg_first ? w[e] : __builtin_fma(cg_b, sv[e], w[e]), v[e]);
          }
        }
#pragma unroll
        for (int e = 0; e < VB; ++e) rb[i * VB + e] = v[e];
      }
      return;
    }
    const int64_t ak = (int64_t)k0 * P.sAk, bk = (int64_t)k0 * P.sBk;
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int gm = m0 + a_mm0 + a_dm * i, gk = k0 + a_kk0 + a_dk * i;
      const int64_t off = HOIST ? a_base + i * a_step + ak : aoff + gm * P.sAm + gk * P.sAk;
      ra[i] = (gm < P.M && gk < kend) ? Ap[off] : SA(0);
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int gn = n0 + b_nn0 + b_dn * i, gk = k0 + b_kk0 + b_dk * i;
      const int64_t off = HOIST ? b_base + i * b_step + bk : boff + gk * P.sBk + gn * P.sBn;
      if constexpr (BCG) {
        // first step: s starts from w (its old contents are not read)
        rb[i] = 0.0;
        if (gn < P.N && gk < kend) {
          const double w = P.Bw[off];
          rb[i] = __builtin_fma(-cg_a, cg_first ? w : __builtin_fma(cg_b, P.Bs[off], w), Bp[off]);
        }
      } else {
        rb[i] = (gn < P.N && gk < kend) ? Bp[off] : SB(0);
      }
    }
  };
  // LDS stores of the loaded slice; each branch is uniform (the operand's
  // unit-stride dimension), and its offsets are a per-lane word offset plus a
  // compile-time one.  A loaded vector along a float32 row goes into LDS in
  // pieces of the fragment length at most (each piece contiguous and aligned
  // there)
  constexpr int PA = VA < VFA ? VA : VFA, PB = VB < VFB ? VB : VFB;
  auto sstore = [&](int buf) {
    T *as = As[buf], *bs = Bs[buf];
    if constexpr (VEC) {
      if (a_m_unit) {
        // thread: row va_o + va_d i (va_d even), columns va_u ..
        const int l0 = LA::row(va_o) + va_u;
#pragma unroll
        for (int i = 0; i < AV; ++i) {
          T *dst = as + l0 + (va_d * i / 2) * LA::PP;
          if constexpr (FRAG && PA > 1) {
            typedef unsigned VT __attribute__((ext_vector_type(PA)));
#pragma unroll
            for (int e0 = 0; e0 < VA; e0 += PA) {
              VT v;
#pragma unroll
              for (int e = 0; e < PA; ++e)
                v[e] = __builtin_bit_cast(unsigned, to_op<T>((double)ra[i * VA + e0 + e]));
              *reinterpret_cast<VT *>(dst + e0) = v;
            }
          } else {
#pragma unroll
            for (int e = 0; e < VA; ++e) dst[e] = to_op<T>((double)ra[i * VA + e]);
          }
        }
      } else {
        // thread: rows va_u + e (va_u even), column va_o + va_d i
        const int l0 = (va_u >> 1) * LA::PP + va_o;
#pragma unroll
        for (int i = 0; i < AV; ++i)
#pragma unroll
          for (int e = 0; e < VA; ++e)
            as[l0 + LA::row(e) + va_d * i] = to_op<T>((double)ra[i * VA + e]);
      }
      if (b_n_unit) {
        const int l0 = LB::row(vb_o) + vb_u;
#pragma unroll
        for (int i = 0; i < BV; ++i) {
          T *dst = bs + l0 + (vb_d * i / 2) * LB::PP;
          if constexpr (FRAG && PB > 1) {
            typedef unsigned VT __attribute__((ext_vector_type(PB)));
#pragma unroll
            for (int e0 = 0; e0 < VB; e0 += PB) {
              VT v;
#pragma unroll
              for (int e = 0; e < PB; ++e)
                v[e] = __builtin_bit_cast(unsigned, to_op<T>((double)rb[i * VB + e0 + e]));
              *reinterpret_cast<VT *>(dst + e0) = v;
            }
          } else {
#pragma unroll
            for (int e = 0; e < VB; ++e) dst[e] = to_op<T>((double)rb[i * VB + e]);
          }
        }
      } else {
        const int l0 = (vb_u >> 1) * LB::PP + vb_o;
#pragma unroll
        for (int i = 0; i < BV; ++i)
#pragma unroll
          for (int e = 0; e < VB; ++e)
            bs[l0 + LB::row(e) + vb_d * i] = to_op<T>((double)rb[i * VB + e]);
      }
      return;
    }
    if (a_m_unit) {
      // thread: row tid / BM + (NTHR / BM) i, column tid % BM
      constexpr int DR = NTHR / BM;
      static_assert(DR % 2 == 0, "even row steps");
      const int l0 = LA::row(tid / BM) + tid % BM;
#pragma unroll
      for (int i = 0; i < AL; ++i) as[l0 + (DR * i / 2) * LA::PP] = to_op<T>((double)ra[i]);
    } else {
      // thread: row tid % KD, column tid / KD + (NTHR / KD) i
      const int l0 = LA::row(tid % KD) + tid / KD;
#pragma unroll
      for (int i = 0; i < AL; ++i) as[l0 + (NTHR / KD) * i] = to_op<T>((double)ra[i]);
    }
    if (b_n_unit) {
      constexpr int DR = NTHR / BN;
      static_assert(DR % 2 == 0, "even row steps");
      const int l0 = LB::row(tid / BN) + tid % BN;
#pragma unroll
      for (int i = 0; i < BL; ++i) bs[l0 + (DR * i / 2) * LB::PP] = to_op<T>((double)rb[i]);
    } else {
      const int l0 = LB::row(tid % KD) + tid / KD;
#pragma unroll
      for (int i = 0; i < BL; ++i) bs[l0 + (NTHR / KD) * i] = to_op<T>((double)rb[i]);
    }
  };

  if (kbeg < kend) {
    gload(kbeg);
    sstore(0);
    __syncthreads();
  }
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += KD) {
    const bool more = k0 + KD < kend;
    if (more) gload(k0 + KD);
#pragma unroll
    for (int h = 0; h < KD / KT; ++h) {
      if constexpr (BF3)
        MfmaBf3F<FM, FN, BM, BN>::step(As[buf], Bs[buf], lane, wm * WTM, wn * WTN, h * KT, acc);
      else if constexpr (FRAG)
        MfmaF32<FM, FN, BM, BN>::step(As[buf], Bs[buf], lane, wm * WTM, wn * WTN, h * KT, acc);
      else
        Mfma<T, FM, FN, LDA>::step(reinterpret_cast<const T(*)[LDA]>(As[buf]) + h * KT,
                                   reinterpret_cast<const T(*)[LDB]>(Bs[buf]) + h * KT, lane,
                                   wm * WTM, wn * WTN, acc);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // D(16x16): lane l holds column l % 16 of the block.  float32 / bfloat16:
  // register r is block row 4*(l/16) + r; float64 16x16x4: register r is
  // block row 4*r + l/16.  Blocks of a float32 wave tile interleave (block i
  // row r is wave-tile row FM r + i, block j column c is wave-tile column
  // FN c + j, as the fragments were read); other types stack them (row
  // 16 i + r, column 16 j + c).  The element offset is the lane's row and
  // column terms; the store kind (partials, float32, float64, with beta) is
  // uniform per problem and chosen outside the element loops.
  const int rowb = m0 + wm * WTM, colb = n0 + wn * WTN;
  auto row_of = [&](int i, int r) {
    const int br = (GemmKind<T>::value == 0) ? (4 * r + (lane >> 4)) : ((lane >> 4) * 4 + r);
    return FRAG ? rowb + FM * br + i : rowb + 16 * i + br;
  };
  auto col_of = [&](int j) {
    return FRAG ? colb + FN * (lane & 15) + j : colb + 16 * j + (lane & 15);
  };
  auto store_all = [&](auto *Cp, int64_t base, int64_t sm, int64_t sn, double alpha, double beta) {
    typedef std::remove_cv_t<std::remove_reference_t<decltype(*Cp)>> E;
    if constexpr (FRAG) {
      // unit column stride with every row start a multiple of FN elements:
      // each lane's FN consecutive columns of a row go out as one vector
      if (sn == 1 && base % FN == 0 && sm % FN == 0 &&
          reinterpret_cast<uintptr_t>(Cp) % (FN * sizeof(E)) == 0) {
        typedef E VE __attribute__((ext_vector_type(FN)));
        const int gn0 = col_of(0);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gm = row_of(i, r);
            if (gm >= P.M) continue;
            E *cp = Cp + base + (int64_t)gm * sm + gn0;
            if (gn0 + FN <= P.N) {
              VE v;
              VE old = beta != 0.0 ? *reinterpret_cast<const VE *>(cp) : VE(E(0));
#pragma unroll
              for (int j = 0; j < FN; ++j) {
                double x = alpha * (double)acc[i][j][r];
                if (beta != 0.0) x += beta * (double)old[j];
                v[j] = (E)x;
              }
              *reinterpret_cast<VE *>(cp) = v;
            } else {
#pragma unroll
              for (int j = 0; j < FN; ++j)
                if (gn0 + j < P.N) {
                  double x = alpha * (double)acc[i][j][r];
                  if (beta != 0.0) x += beta * (double)cp[j];
                  cp[j] = (E)x;
                }
            }
          }
        return;
      }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int gn = col_of(j);
        const int64_t bj = base + (int64_t)gn * sn;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = row_of(i, r);
          if (gm < P.M && gn < P.N) {
            auto *cp = Cp + bj + (int64_t)gm * sm;
            double v = alpha * (double)acc[i][j][r];
            if (beta != 0.0) v += beta * (double)*cp;
            *cp = (decltype(+*cp))v;
          }
        }
      }
  };
  if (!P.direct) {
    const int64_t bidx = (int64_t)b2 * P.B1 + b1;
    store_all(P.part, ((int64_t)ks * P.B1 * P.B2 + bidx) * P.M * P.N, (int64_t)P.N, (int64_t)1,
              1.0, 0.0);
  } else if (P.c32) {
    store_all(reinterpret_cast<float *>(P.C), b1 * P.sCb1 + b2 * P.sCb2, P.sCm, P.sCn, P.alpha,
              P.beta);
  } else {
    store_all(P.C, b1 * P.sCb1 + b2 * P.sCb2, P.sCm, P.sCn, P.alpha, P.beta);
  }
}

struct RedSrc {
  const double *part;
  int ksplit;
  double alpha;  // used when the output's sources carry different alphas
};
struct RedOut {
  double *C;
  int64_t sCm, sCn, sCb1, sCb2;
  const double *X;  // beta term input (may be C)
  int64_t sXm, sXn, sXb1, sXb2;
  int M, N, B1, B2;
  double alpha, beta;
  int nsrc;
  int salpha;  // 1: out = sum_q alpha_q (sum over q's splits), else alpha (sum)
  RedSrc src[GEMM_GROUP];
  int64_t total;           // elements of this output
  unsigned blk0, nblk;     // its workgroups: blk0 .. blk0 + nblk - 1
  int c32, x32;  // C / X stored as float32
  const double *Y;  // dot partner laid out like C (float64), or null
  int64_t cgoff;    // fused CG step: position of C's element 0 in the vectors
};
struct RedK {
  int nout;
  RedOut o[GEMM_GROUP];
  const int *skip;
  int64_t total;
  // fused dot sum_outputs C . Y: per-block partials in dpart, the last block
  // to arrive (counter dctr, reset to 0 by it) sums them in block order
  double *dpart, *dout;
  unsigned *dctr;
  // fused CG step (cst non-null): the outputs update the CG vectors
  CGState *cst;
  double *cx, *cr, *cw, *cp, *cs, *cz, *cpart;
};

// s += p[0], p[tot], ..., p[(ks - 1) tot] in that order; the loads of a
// batch of eight are issued before their adds (independent addresses), so a
// thread waits for one memory latency per batch rather than per split
__device__ inline void red_add_splits(double &s, const double *p, int ks, int64_t tot) {
  int k = 0;
  for (; k + 8 <= ks; k += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(int64_t)(k + u) * tot];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += t[u];
  }
  if (k + 4 <= ks) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = p[(int64_t)(k + u) * tot];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += t[u];
    k += 4;
  }
  for (; k < ks; ++k) s += p[(int64_t)k * tot];
}

__device__ inline double red_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// one element of the fused CG step (unpreconditioned, single reduction):
// s = w + beta s, p = r + beta p (first step: w, r), x += alpha p,
// r -= alpha s, w = A r = v + beta_X r; with the partial sums of r.r and w.r
// (fused multiply-adds spelled out: the roundings do not hang on the
// compiler's contraction choices)
__device__ __forceinline__ void cg_elem(const RedK &R, int64_t j, double wi, double ri, double so,
                                        double po, double xo, double v, double bx, double a,
                                        double b, bool first, double &rr, double &wr) {
  const double si = first ? wi : __builtin_fma(b, so, wi);
  const double pi = first ? ri : __builtin_fma(b, po, ri);
  R.cs[j] = si;
  R.cp[j] = pi;
  R.cx[j] = __builtin_fma(a, pi, xo);
  const double rn = __builtin_fma(-a, si, ri);
  const double wn = __builtin_fma(bx, rn, v);
  R.cr[j] = rn;
  R.cw[j] = wn;
  rr = __builtin_fma(rn, rn, rr);
  wr = __builtin_fma(wn, rn, wr);
}

// out = alpha * (sum over sources, splits in order) + beta * X, or with
// per-source alphas sum_q alpha_q (sum over q's splits) + beta * X
__global__ __launch_bounds__(256) void k_splitk_reduce(RedK R) {
  if (R.skip && *R.skip) return;
  double dacc = 0.0;
  // fused CG step: alpha and beta of this iteration (see GemmCg)
  double cg_a = 0.0, cg_b = 0.0, cg_rr = 0.0, cg_wr = 0.0, cg_g = 0.0;
  bool cg_first = false;
  if (R.cst) {
    cg_g = R.cst->gamma;
    const double dl = R.cst->delta;
    cg_first = R.cst->first != 0;
    cg_b = cg_first ? 0.0 : cg_g / R.cst->gamma_prev;
    cg_a = cg_first ? cg_g / dl : cg_g / (dl - cg_b * cg_g / R.cst->alpha_prev);
  }
  // each workgroup serves one output (selected from the block index, so the
  // output's fields are uniform across it)
  int oi = 0;
#pragma unroll
  for (int k = 1; k < GEMM_GROUP; ++k)
    if (k < R.nout && blockIdx.x >= R.o[k].blk0) oi = k;
  const RedOut &O = R.o[oi];
  const int64_t per = (int64_t)O.M * O.N;
  const int64_t tot = O.total;
  for (int64_t idx = (int64_t)(blockIdx.x - O.blk0) * blockDim.x + threadIdx.x; idx < tot;
       idx += (int64_t)O.nblk * blockDim.x) {
    double v = 0.0;
    if (O.salpha) {
      for (int q = 0; q < O.nsrc; ++q) {
        double s = 0.0;
        red_add_splits(s, O.src[q].part + idx, O.src[q].ksplit, tot);
        v += O.src[q].alpha * s;
      }
    } else {
      double s = 0.0;
      for (int q = 0; q < O.nsrc; ++q) red_add_splits(s, O.src[q].part + idx, O.src[q].ksplit, tot);
      v = O.alpha * s;
    }
    const int64_t bidx = idx / per;
    const int64_t r = idx % per;
    const int gm = (int)(r / O.N), gn = (int)(r % O.N);
    const int b1 = (int)(bidx % O.B1), b2 = (int)(bidx / O.B1);
    if (O.beta != 0.0 && !R.cst) {
      const int64_t xo = b1 * O.sXb1 + b2 * O.sXb2 + gm * O.sXm + gn * O.sXn;
      v += O.beta * (O.x32 ? (double)reinterpret_cast<const float *>(O.X)[xo] : O.X[xo]);
    }
    const int64_t co = b1 * O.sCb1 + b2 * O.sCb2 + gm * O.sCm + gn * O.sCn;
    if (R.cst) {
      // first step: s and p start from w and r (old contents unread); the
      // beta term of the matvec takes the new residual
      const int64_t j = O.cgoff + co;
      const double wi = R.cw[j], ri = R.cr[j];
      cg_elem(R, j, wi, ri, cg_first ? 0.0 : R.cs[j], cg_first ? 0.0 : R.cp[j], R.cx[j], v,
              O.beta, cg_a, cg_b, cg_first, cg_rr, cg_wr);
      continue;
    }
    if (O.c32) reinterpret_cast<float *>(O.C)[co] = (float)v;
    else O.C[co] = v;
    if (O.Y) dacc += v * O.Y[co];
  }
  if (R.cst) {
    __shared__ double shc[2][4];
    __shared__ bool lastc;
    cg_rr = red_wave_sum(cg_rr);
    cg_wr = red_wave_sum(cg_wr);
    if ((threadIdx.x & 63) == 0) {
      shc[0][threadIdx.x >> 6] = cg_rr;
      shc[1][threadIdx.x >> 6] = cg_wr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      R.cpart[2 * blockIdx.x] = (shc[0][0] + shc[0][1]) + (shc[0][2] + shc[0][3]);
      R.cpart[2 * blockIdx.x + 1] = (shc[1][0] + shc[1][1]) + (shc[1][2] + shc[1][3]);
      __threadfence();
      lastc = (atomicAdd(&R.cst->counter, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!lastc) return;
    __threadfence();
    const volatile double *vp = R.cpart;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += 256) {
      a += vp[2 * i];
      b += vp[2 * i + 1];
    }
    a = red_wave_sum(a);
    b = red_wave_sum(b);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      shc[0][threadIdx.x >> 6] = a;
      shc[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double rr = (shc[0][0] + shc[0][1]) + (shc[0][2] + shc[0][3]);
      const double wr = (shc[1][0] + shc[1][1]) + (shc[1][2] + shc[1][3]);
      CGState *st = R.cst;
      st->iters += 1;
      st->gamma_prev = cg_g;
      st->alpha_prev = cg_a;
      st->gamma = rr;
      st->delta = wr;
      st->first = 0;
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
    return;
  }
  if (!R.dout) return;
  __shared__ double sh[4];
  __shared__ bool last;
  dacc = red_wave_sum(dacc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dacc;
  __syncthreads();
  if (threadIdx.x == 0) {
    R.dpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __threadfence();
    last = (atomicAdd(R.dctr, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double *vp = R.dpart;
  double a = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += 256) a += vp[i];
  a = red_wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    *R.dout = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    *R.dctr = 0;
  }
}

void check_operands(Ctx &c, const Gemm &q) {
  int64_t lo = 0, hi = 0;
  span(lo, hi, q.M, q.sAm);
  span(lo, hi, q.K, q.sAk);
  span(lo, hi, q.B1, q.sAb1);
  span(lo, hi, q.B2, q.sAb2);
  if (q.K > 0) c.check_range(q.A, lo, hi, q.a32 ? sizeof(float) : sizeof(double), "gemm A");
  lo = hi = 0;
  span(lo, hi, q.K, q.sBk);
  span(lo, hi, q.N, q.sBn);
  span(lo, hi, q.B1, q.sBb1);
  span(lo, hi, q.B2, q.sBb2);
  if (q.K > 0) c.check_range(q.B, lo, hi, q.b32 ? sizeof(float) : sizeof(double), "gemm B");
  lo = hi = 0;
  span(lo, hi, q.M, q.sCm);
  span(lo, hi, q.N, q.sCn);
  span(lo, hi, q.B1, q.sCb1);
  span(lo, hi, q.B2, q.sCb2);
  c.check_range(q.C, lo, hi, q.c32 ? sizeof(float) : sizeof(double), "gemm C");
}

// launch of one tile configuration with the operands' storage types (float32
// storage only with float32 MFMAs; every problem of a launch shares them)
template <typename T, int BM, int WGM, int WGN, int KD, typename SA = double,
          typename SB = double>
void launch_k(bool vec, const dim3 &grid, hipStream_t st, const GemmK &g) {
  const dim3 blk(64 * WGM * WGN);
  if (vec)
    hipLaunchKernelGGL((k_gemm<T, BM, BM, WGM, WGN, KD, SA, SB, false, true>), grid, blk, 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm<T, BM, BM, WGM, WGN, KD, SA, SB, false, false>), grid, blk, 0, st,
                       g);
}

template <typename T>
void launch_tile(int MT, int sa, int sb, int64_t blocks, hipStream_t st, const GemmK &g) {
  const dim3 grid((unsigned)blocks);
  if (g.cgst) {
    if (!std::is_same<T, double>::value || MT != 64 || sa || sb)
      fail(QTT_E_ARG, "gemm: the CG operand needs float64 64-tiles");
    bool vec = true;
    for (int i = 0; i < g.np; ++i) vec = vec && g.p[i].va && g.p[i].vb;
    if (vec)
      hipLaunchKernelGGL((k_gemm<double, 64, 64, 2, 2, 16, double, double, true, true>), grid,
                         dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_gemm<double, 64, 64, 2, 2, 16, double, double, true, false>), grid,
                         dim3(256), 0, st, g);
    return;
  }
  // vector loads when every problem of the launch qualifies
  bool vec = true;
  for (int i = 0; i < g.np; ++i) vec = vec && g.p[i].va && g.p[i].vb;
  if constexpr (std::is_same<T, float>::value) {
    if (MT == 128) {
      if (sa && sb) launch_k<T, 128, 2, 4, 32, float, float>(vec, grid, st, g);
      else if (sa) launch_k<T, 128, 2, 4, 32, float, double>(vec, grid, st, g);
      else if (sb) launch_k<T, 128, 2, 4, 32, double, float>(vec, grid, st, g);
      else launch_k<T, 128, 2, 4, 32>(vec, grid, st, g);
    } else {
      if (sa && sb) launch_k<T, 64, 2, 2, 16, float, float>(vec, grid, st, g);
      else if (sa) launch_k<T, 64, 2, 2, 16, float, double>(vec, grid, st, g);
      else if (sb) launch_k<T, 64, 2, 2, 16, double, float>(vec, grid, st, g);
      else launch_k<T, 64, 2, 2, 16>(vec, grid, st, g);
    }
  } else if constexpr (std::is_same<T, bf3>::value) {
    // split bfloat16: float32 or float64 operand storage (float32 for the
    // convection networks, whose environments and chains are stored in float32)
    // 128 x 128 tiles on 2 x 2 waves (64 x 64 per wave): each operand value
    // read from LDS feeds four blocks, which keeps the three-MFMA step from
    // being bound by LDS reads
    if (MT == 128) {
      if (sa && sb) launch_k<T, 128, 2, 2, 32, float, float>(vec, grid, st, g);
      else if (sa) launch_k<T, 128, 2, 2, 32, float, double>(vec, grid, st, g);
      else if (sb) launch_k<T, 128, 2, 2, 32, double, float>(vec, grid, st, g);
      else launch_k<T, 128, 2, 2, 32>(vec, grid, st, g);
    } else {
      if (sa && sb) launch_k<T, 64, 2, 2, 16, float, float>(vec, grid, st, g);
      else if (sa) launch_k<T, 64, 2, 2, 16, float, double>(vec, grid, st, g);
      else if (sb) launch_k<T, 64, 2, 2, 16, double, float>(vec, grid, st, g);
      else launch_k<T, 64, 2, 2, 16>(vec, grid, st, g);
    }
  } else {
    if (sa || sb) fail(QTT_E_ARG, "gemm: float32 operand storage needs float32 or split bfloat16 MFMAs");
    if (MT == 128) launch_k<T, 128, 2, 4, 32>(vec, grid, st, g);
    else launch_k<T, 64, 2, 2, 16>(vec, grid, st, g);
  }
}

// Result-invariant tile autotuning.  For a launch without split-K, whose
// problems all write C = alpha A B (beta = 0, no summed or extra inputs),
// running it twice is harmless and every tile size gives bitwise the same C;
// the first time such a shape appears (outside graph capture) the tile sizes
// run interleaved three times each, timed with events, and the one with the
// fastest run is remembered for the shape (enabled by QTT_AUTOTUNE=1).
template <typename T, typename Build>
int tuned_tile(Ctx &c, int np, const Gemm *q, int ngroups, const double *const *X,
               int heuristic, Build &build, GemmK &g, int64_t &blocks, int64_t &part_need) {
  if (!c.autotune || c.capturing || ngroups != np) return heuristic;
  for (int i = 0; i < np; ++i)
    if (q[i].beta != 0.0 || X[i] != nullptr) return heuristic;
  char key[256];
  int o = std::snprintf(key, sizeof key, "%d:%d", GemmKind<T>::value, np);
  for (int i = 0; i < np && o < (int)sizeof key - 48; ++i)
    o += std::snprintf(key + o, sizeof key - o, "|%d,%d,%d,%d,%d,%d%d", q[i].M, q[i].N, q[i].K,
                       q[i].B1, q[i].B2, q[i].sAm == 1, q[i].sBn == 1);
  auto it = c.gemm_tune.find(key);
  if (it != c.gemm_tune.end()) return it->second;
  // candidates interleaved, three rounds, fastest single run of each
  const int cand[2] = {64, 128};
  float best[2] = {3.0e38f, 3.0e38f};
  hipEvent_t e0 = c.take_event(), e1 = c.take_event();
  for (int rep = 0; rep < 3; ++rep)
    for (int ci = 0; ci < 2; ++ci) {
      const int MT = cand[ci];
      build(MT);
      if (g.np == 0 || part_need > 0) {
        c.kt.pool.push_back(e0);
        c.kt.pool.push_back(e1);
        return heuristic;
      }
      HIPC(hipEventRecord(e0, c.stream));
      launch_tile<T>(MT, q[0].a32, q[0].b32, blocks, c.stream, g);
      HIPC(hipGetLastError());
      HIPC(hipEventRecord(e1, c.stream));
      HIPC(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, e0, e1));
      best[ci] = std::min(best[ci], ms);
    }
  const int choice = best[1] < best[0] ? 128 : 64;
  c.kt.pool.push_back(e0);
  c.kt.pool.push_back(e1);
  c.gemm_tune[key] = choice;
  return choice;
}

// np problems; problem i belongs to output group group[i] (a group holds
// one or two problems that share C; X[group] is the beta input, nullptr = C).
template <typename T>
void launch_group(Ctx &c, int np, const Gemm *q, int ngroups, const int *group,
                  const double *const *X, const int *skip, const GemmDot *dot = nullptr,
                  const GemmCg *cg = nullptr) {
  GemmK g{};
  g.np = 0;
  g.skip = skip;
  g.flops = 0.0;
  const int kind = GemmKind<T>::value;
  int64_t blocks = 0;
  int nsrc[GEMM_GROUP] = {0};
  for (int i = 0; i < np; ++i) {
    if (group[i] < 0 || group[i] >= ngroups || ngroups > GEMM_GROUP)
      fail(QTT_E_ARG, "gemm group: bad output group");
    nsrc[group[i]] += 1;
  }
  for (int i = 1; i < np; ++i)
    if (q[i].a32 != q[0].a32 || q[i].b32 != q[0].b32)
      fail(QTT_E_ARG, "gemm group: operand storage types must agree");
  g.cgst = q[0].cgst;
  for (int i = 0; i < np; ++i) {
    if (q[i].cgst != g.cgst) fail(QTT_E_ARG, "gemm group: CG operands must agree");
    if (q[i].cgst && (!q[i].Bw || !q[i].Bs || q[i].b32))
      fail(QTT_E_ARG, "gemm: the CG operand needs float64 w and s");
  }
  int64_t part_need = 0;
  int64_t part_off[GEMM_GROUP] = {0};
  int keep[GEMM_GROUP];
  // split-K is decided on the 64 x 64 tiling alone, so the tile size never
  // changes the summation order: every tile choice gives identical results
  int64_t tiles64 = 0, tiles128 = 0;
  for (int i = 0; i < np; ++i) {
    tiles64 += (int64_t)((q[i].M + 63) / 64) * ((q[i].N + 63) / 64) * q[i].B1 * q[i].B2;
    tiles128 += (int64_t)((q[i].M + 127) / 128) * ((q[i].N + 127) / 128) * q[i].B1 * q[i].B2;
  }
  const bool may_split = tiles64 < 256;
  auto build = [&](int MT) {
    const int NT = MT;
    g.np = 0;
    g.flops = 0.0;
    blocks = 0;
    part_need = 0;
    for (int i = 0; i < np; ++i) {
      const Gemm &s = q[i];
      keep[i] = -1;
      if (s.M <= 0 || s.N <= 0 || s.B1 <= 0 || s.B2 <= 0) continue;
      Prob &P = g.p[g.np];
      keep[i] = g.np++;
      P.M = s.M;
      P.N = s.N;
      P.K = s.K;
      P.B1 = s.B1;
      P.B2 = s.B2;
      P.tm = (s.M + MT - 1) / MT;
      P.tn = (s.N + NT - 1) / NT;
      P.A = s.A;
      P.sAm = s.sAm;
      P.sAk = s.sAk;
      P.sAb1 = s.sAb1;
      P.sAb2 = s.sAb2;
      P.B = s.B;
      P.sBk = s.sBk;
      P.sBn = s.sBn;
      P.sBb1 = s.sBb1;
      P.sBb2 = s.sBb2;
      P.C = s.C;
      P.sCm = s.sCm;
      P.sCn = s.sCn;
      P.sCb1 = s.sCb1;
      P.sCb2 = s.sCb2;
      P.alpha = s.alpha;
      P.beta = s.beta;
      P.part = nullptr;
      P.c32 = s.c32 ? 1 : 0;
      {
        // elements of one 16-byte vector in A's and B's storage
        const int VA = s.a32 ? 4 : 2, VB = s.b32 ? 4 : 2;
        auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
        P.va = (al(s.A) && s.sAb1 % VA == 0 && s.sAb2 % VA == 0 &&
                ((s.sAm == 1 && s.sAk % VA == 0 && s.M % VA == 0) ||
                 (s.sAm != 1 && s.sAk == 1 && s.sAm % VA == 0 && s.K % VA == 0)))
                   ? 1 : 0;
        P.vb = ((!s.cgst || (al(s.Bw) && al(s.Bs))) && al(s.B) && s.sBb1 % VB == 0 &&
                s.sBb2 % VB == 0 &&
                ((s.sBn == 1 && s.sBk % VB == 0 && s.N % VB == 0) ||
                 (s.sBn != 1 && s.sBk == 1 && s.sBn % VB == 0 && s.K % VB == 0)))
                   ? 1 : 0;
      }
      P.Bw = s.Bw;
      P.Bs = s.Bs;
      g.flops += 2.0 * s.M * (double)s.N * s.K * s.B1 * s.B2;
      const int64_t out_tiles = (int64_t)P.tm * P.tn * P.B1 * P.B2;
      P.ksplit = 1;
      P.kchunk = std::max(s.K, 1);
      // split K when the group's output tiles cannot fill the compute units
      if (may_split && s.K >= 4 * KT) {
        const int64_t want = (512 + tiles64 - 1) / tiles64;
        const int64_t maxs = s.K / (2 * KT);
        int ks = (int)std::max<int64_t>(1, std::min<int64_t>(want, maxs));
        if (ks > 1) {
          int chunk = (s.K + ks - 1) / ks;
          chunk = ((chunk + KT - 1) / KT) * KT;
          ks = (s.K + chunk - 1) / chunk;
          P.ksplit = ks;
          P.kchunk = chunk;
        }
      }
      P.direct = (P.ksplit == 1 && nsrc[group[i]] == 1 && X[group[i]] == nullptr) ? 1 : 0;
      part_off[g.np - 1] = part_need;
      if (!P.direct) part_need += (int64_t)P.ksplit * P.M * P.N * P.B1 * P.B2;
      // problems start on a multiple of 8 blocks (one per XCD, see k_gemm)
      blocks = (blocks + 7) & ~(int64_t)7;
      P.block0 = blocks;
      blocks += out_tiles * P.ksplit;
    }
  };
  for (int i = 0; i < np; ++i)
    if (q[i].M > 0 && q[i].N > 0 && q[i].B1 > 0 && q[i].B2 > 0) {
      check_operands(c, q[i]);
      if (q[i].cgst && q[i].K > 0) {
        int64_t lo = 0, hi = 0;
        span(lo, hi, q[i].K, q[i].sBk);
        span(lo, hi, q[i].N, q[i].sBn);
        span(lo, hi, q[i].B1, q[i].sBb1);
        span(lo, hi, q[i].B2, q[i].sBb2);
        c.check_range(q[i].Bw, lo, hi, sizeof(double), "gemm CG w");
        c.check_range(q[i].Bs, lo, hi, sizeof(double), "gemm CG s");
        c.check_range(q[i].cgst, 0, 0, sizeof(CGState), "gemm CG state");
      }
    }
  // tile size: 64 x 64 while split-K may be needed; otherwise the tuned
  // choice for this shape, or 128 x 128 when there is one such tile per CU
  int MT = (!may_split && tiles128 >= 256) ? 128 : 64;
  if (g.cgst) MT = 64;  // the CG operand exists for float64 64-tiles only
  else if (!may_split) MT = tuned_tile<T>(c, np, q, ngroups, X, MT, build, g, blocks, part_need);
  build(MT);
  if (g.np == 0) return;
  if (blocks > 0x7fffffffLL) fail(QTT_E_UNSUPPORTED, "gemm grid too large");
  if (part_need > ((int64_t)64 << 20)) fail(QTT_E_UNSUPPORTED, "gemm split-K buffer too large");
  if (part_need > 0) {
    static const char *const names[4] = {"gemm_splitk64", "gemm_splitk32", "gemm_splitk16",
                                         "gemm_splitk16x3"};
    double *part = c.buf(names[kind], part_need);
    for (int i = 0; i < g.np; ++i)
      if (!g.p[i].direct) g.p[i].part = part + part_off[i];
  }

  bool timed = false;
  std::pair<hipEvent_t, hipEvent_t> ev;
  const bool big = (MT == 128);
  const int tk = kind + (big ? 2 : 0);  // timer kind
  if (c.kt.on && kind < 2) g.flop_ctr = c.kt.flop_ctr + tk;
  if (c.capturing) {
    if (kind < 2) c.cap_launches[tk] += 1;
  } else if (c.kt.on && kind < 2) {
    timed = (c.kt.launches[tk] % c.kt.every) == 0;
    c.kt.launches[tk] += 1;
    if (timed) {
      if (c.kt.pending[tk].size() >= 16384) c.resolve_events();
      ev.first = c.take_event();
      ev.second = c.take_event();
      HIPC(hipEventRecord(ev.first, c.stream));
    }
  }
  std::pair<hipEvent_t, hipEvent_t> sev;
  const bool shape_rec = c.shape_stats && !c.capturing;
  if (shape_rec) {
    sev.first = c.take_event();
    sev.second = c.take_event();
    HIPC(hipEventRecord(sev.first, c.stream));
  }
  launch_tile<T>(MT, q[0].a32, q[0].b32, blocks, c.stream, g);
  HIPC(hipGetLastError());
  if (shape_rec) {
    HIPC(hipEventRecord(sev.second, c.stream));
    char key[200];
    const Prob &P = g.p[0];
    std::snprintf(key, sizeof key, "%s x%d M=%d N=%d K=%d B=%dx%d split=%d t%d %s%s%s%s",
                  kind == 0 ? "f64" : (kind == 1 ? "f32" : (kind == 2 ? "bf16" : "bf16x3")), g.np,
                  P.M, P.N, P.K, P.B1, P.B2, P.ksplit, MT,
                  P.sAm == 1 ? "Am" : "Ak", P.sBn == 1 ? "Bn" : "Bk", q[0].a32 ? " a32" : "",
                  q[0].b32 ? " b32" : "");
    c.shape_pending.push_back({key, sev});
    c.shape_flops_pending.push_back(g.flops);
    if (c.shape_pending.size() > 8192) c.resolve_shapes();
  }
  if (timed) {
    HIPC(hipEventRecord(ev.second, c.stream));
    c.kt.pending[tk].push_back(ev);
  }
  // reduction of split / summed outputs
  if (part_need > 0) {
    RedK R{};
    R.skip = skip;
    int64_t total = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
      RedOut O{};
      bool any = false;
      for (int i = 0; i < np; ++i) {
        if (group[i] != gi || keep[i] < 0) continue;
        const Prob &P = g.p[keep[i]];
        if (P.direct) continue;
        if (O.nsrc >= GEMM_GROUP) fail(QTT_E_ARG, "gemm group: too many problems per output");
        const Gemm &s = q[i];
        if (!any) {
          O.C = s.C;
          O.sCm = s.sCm;
          O.sCn = s.sCn;
          O.sCb1 = s.sCb1;
          O.sCb2 = s.sCb2;
          O.X = X[gi] ? X[gi] : s.C;
          O.sXm = s.sCm;
          O.sXn = s.sCn;
          O.sXb1 = s.sCb1;
          O.sXb2 = s.sCb2;
          O.M = s.M;
          O.N = s.N;
          O.B1 = s.B1;
          O.B2 = s.B2;
          O.alpha = s.alpha;
          O.beta = s.beta;
          // an explicit beta input is float64; C doubles as X in C's type
          O.c32 = s.c32 ? 1 : 0;
          O.x32 = X[gi] ? 0 : O.c32;
          any = true;
        } else if (s.M != O.M || s.N != O.N || s.B1 != O.B1 || s.B2 != O.B2 || s.C != O.C ||
                   s.beta != O.beta || s.c32 != (O.c32 != 0)) {
          fail(QTT_E_ARG, "gemm group: summed problems must share the output");
        } else if (s.alpha != O.alpha) {
          O.salpha = 1;
        }
        O.src[O.nsrc].part = P.part;
        O.src[O.nsrc].ksplit = P.ksplit;
        O.src[O.nsrc].alpha = s.alpha;
        O.nsrc += 1;
      }
      if (!any) continue;
      if (R.nout >= GEMM_GROUP) fail(QTT_E_ARG, "gemm group: too many reduced outputs");
      if (cg) {
        O.cgoff = cg->off[gi];
        if (O.c32 || O.B1 != 1 || O.B2 != 1 || O.sCn != 1 || O.sCm != O.N)
          fail(QTT_E_ARG, "gemm cg: packed float64 outputs only");
        if (O.cgoff < 0 || O.cgoff + (int64_t)O.M * O.N > cg->n)
          fail(QTT_E_ARG, "gemm cg: output outside the vectors");
      }
      if (dot) {
        O.Y = dot->Y[gi];
        int64_t lo = 0, hi = 0;
        span(lo, hi, O.M, O.sCm);
        span(lo, hi, O.N, O.sCn);
        span(lo, hi, O.B1, O.sCb1);
        span(lo, hi, O.B2, O.sCb2);
        if (O.Y) c.check_range(O.Y, lo, hi, sizeof(double), "gemm dot partner");
        if (O.c32) fail(QTT_E_ARG, "gemm dot: float64 outputs only");
      }
      if (X[gi]) {
        int64_t lo = 0, hi = 0;
        span(lo, hi, O.M, O.sXm);
        span(lo, hi, O.N, O.sXn);
        span(lo, hi, O.B1, O.sXb1);
        span(lo, hi, O.B2, O.sXb2);
        c.check_range(O.X, lo, hi, sizeof(double), "gemm X");
      }
      O.total = (int64_t)O.M * O.N * O.B1 * O.B2;
      total += O.total;
      R.o[R.nout++] = O;
    }
    R.total = total;
    if (total > 0) {
      // workgroups per output: one per 256 elements, scaled down to the cap
      // (at most 4096, or the partial slots of a fused dot / CG step)
      int64_t cap = 4096;
      if (cg) cap = std::min<int64_t>(cap, cg->nparts);
      if (dot) cap = std::min<int64_t>(cap, dot->nparts);
      int64_t want = 0;
      for (int o = 0; o < R.nout; ++o) want += (R.o[o].total + 255) / 256;
      unsigned rg = 0;
      for (int o = 0; o < R.nout; ++o) {
        int64_t nb = (R.o[o].total + 255) / 256;
        if (want > cap) nb = std::max<int64_t>(1, nb * (cap - R.nout) / want);
        R.o[o].blk0 = rg;
        R.o[o].nblk = (unsigned)nb;
        rg += (unsigned)nb;
      }
      if (rg > cap) fail(QTT_E_UNSUPPORTED, "gemm reduction: workgroup count");
      if (cg) {
        c.check_range(cg->part, 0, 2 * (int64_t)rg - 1, sizeof(double), "gemm cg partials");
        c.check_range(cg->st, 0, 0, sizeof(CGState), "gemm cg state");
        for (double *vv : {cg->x, cg->r, cg->w, cg->p, cg->s})
          c.check_range(vv, 0, cg->n - 1, sizeof(double), "gemm cg vector");
        R.cst = cg->st;
        R.cx = cg->x;
        R.cr = cg->r;
        R.cw = cg->w;
        R.cp = cg->p;
        R.cs = cg->s;
        R.cpart = cg->part;
      }
      if (dot) {
        c.check_range(dot->part, 0, rg - 1, sizeof(double), "gemm dot partials");
        R.dpart = dot->part;
        R.dout = dot->out;
        R.dctr = dot->ctr;
      }
      hipLaunchKernelGGL(k_splitk_reduce, dim3(rg), dim3(256), 0, c.stream, R);
      HIPC(hipGetLastError());
    }
  }
  if (dot || cg) {
    // every output must have gone through the reduction
    for (int i = 0; i < np; ++i)
      if (keep[i] >= 0 && g.p[keep[i]].direct)
        fail(QTT_E_ARG, "gemm dot/cg: outputs written directly by the GEMM");
    if (part_need == 0) fail(QTT_E_ARG, "gemm dot/cg: no reduced output");
  }
}

}  // namespace

void gemm(Ctx &c, const Gemm &g) {
  const int grp = 0;
  const double *X = nullptr;
  launch_group<double>(c, 1, &g, 1, &grp, &X, g.skip);
}

void gemm_f32(Ctx &c, const Gemm &g) {
  const int grp = 0;
  const double *X = nullptr;
  launch_group<float>(c, 1, &g, 1, &grp, &X, g.skip);
}

void gemm_bf16(Ctx &c, const Gemm &g) {
  const int grp = 0;
  const double *X = nullptr;
  launch_group<__bf16>(c, 1, &g, 1, &grp, &X, g.skip);
}

void gemm_bf16x3(Ctx &c, const Gemm &g) {
  const int grp = 0;
  const double *X = nullptr;
  launch_group<bf3>(c, 1, &g, 1, &grp, &X, g.skip);
}

void gemm_grouped(Ctx &c, int np, const Gemm *q, int ngroups, const int *group,
                  const double *const *X, const int *skip, int prec, const GemmDot *dot,
                  const GemmCg *cg) {
  if (np < 1 || np > GEMM_GROUP) fail(QTT_E_ARG, "gemm_grouped: 1..4 problems");
  if (dot && cg) fail(QTT_E_ARG, "gemm_grouped: dot and cg are exclusive");
  if (prec == QTT_PREC_F32) launch_group<float>(c, np, q, ngroups, group, X, skip, dot, cg);
  else if (prec == QTT_PREC_BF16X3) launch_group<bf3>(c, np, q, ngroups, group, X, skip, dot, cg);
  else launch_group<double>(c, np, q, ngroups, group, X, skip, dot, cg);
}

}  // namespace qtt
