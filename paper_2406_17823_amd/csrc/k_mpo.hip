// MPO layer of a network chain: one site's MPO core applied to an
// intermediate tensor,
//   T'[p][w_out][m'][q] = sum_{m, w_in} W[m][w_in][w_out][m'] T[p][m][w_in][q],
// where p runs over the bra and outer-layer bonds and q over the inner-layer
// and ket bonds.  The finite-difference cores are sparse (12 of 144 entries
// of the bond-3 derivative core, at most 144 of 1296 of a composed bond-9
// penalty core), so this is an HBM-streaming step: each thread owns V
// consecutive q of one output row (p, w_out m'), sums the few non-zeros of
// that output column (compressed columns built on the host once per MPO)
// with V-wide vector loads of the input rows, and stores V outputs; q is the
// fastest index so loads and stores are unit-stride across a wave.  The row
// index costs two integer divisions per V elements (the per-element form
// spent more time in index arithmetic than in memory traffic).
#include "qtt_internal.h"

namespace qtt {

namespace {

struct MJob {
  const void *T;
  void *Tout;
  const int *colptr, *rowidx;
  const double *val;
  int KI, KO;
  int64_t post, total;
  unsigned blk0, nblk;  // the job's workgroups: blk0 .. blk0 + nblk - 1
};
struct MJobs {
  int nj;
  MJob j[4];
};

// largest core mode of the staged column tables: 4 x a bond of 9 (the
// composed penalty cores)
constexpr int MPO_MAXK = 36;

template <typename TS, int V> struct VecOf;
template <> struct VecOf<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VecOf<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };

// up to four layers in one launch, V consecutive q per thread (post % V == 0,
// tensors aligned to V elements, pre * KO * post < 2^31); the same float64
// sums in the same order as the scalar form, so results are bitwise equal
template <typename TS, int V>
__global__ __launch_bounds__(256) void k_mpo_rows_grouped(MJobs J, const int *skip) {
  if (skip && *skip) return;
  typedef typename VecOf<TS, V>::type VT;
  int ji = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < J.nj && blockIdx.x >= J.j[i].blk0) ji = i;
  const MJob &M = J.j[ji];
  const unsigned qv = (unsigned)(M.post / V);
  const unsigned nvec = (unsigned)(M.total / V);
  const int KI = M.KI, KO = M.KO;
  const unsigned post = (unsigned)M.post;
  const TS *T = static_cast<const TS *>(M.T);
  TS *Tout = static_cast<TS *>(M.Tout);
  // the job's compressed columns staged in LDS (a core has at most 36 x 36
  // entries), so that a row's input loads wait on LDS reads only, not on
  // dependent global reads of the column tables; for large layers only (a
  // small layer's rows do not repay the staging and its barrier: measured
  // 36.4 -> 34.0 us on the float32 chain layers, 5.7 -> 6.1 us on the small
  // float64 ones)
  __shared__ int s_cp[MPO_MAXK + 1];
  __shared__ int s_ri[MPO_MAXK * MPO_MAXK];
  __shared__ double s_val[MPO_MAXK * MPO_MAXK];
  const int c0 = M.colptr[0], nz = M.colptr[KO] - c0;
  const bool staged = KO <= MPO_MAXK && nz <= MPO_MAXK * MPO_MAXK && nvec >= (1u << 20);
  if (staged) {  // uniform across the workgroup (the job's fields)
    for (int i = threadIdx.x; i <= KO; i += 256) s_cp[i] = M.colptr[i] - c0;
    for (int i = threadIdx.x; i < nz; i += 256) {
      s_ri[i] = M.rowidx[c0 + i];
      s_val[i] = M.val[c0 + i];
    }
    __syncthreads();
  }
  auto rows = [&](const int *cp, const int *ri, const double *va) {
    for (unsigned idx = (blockIdx.x - M.blk0) * 256u + threadIdx.x; idx < nvec;
         idx += M.nblk * 256u) {
      const unsigned row = idx / qv;
      const unsigned qi = idx - row * qv;
      const unsigned p = row / (unsigned)KO;
      const int o = (int)(row - p * (unsigned)KO);
      const TS *src = T + (size_t)p * KI * post + (size_t)qi * V;
      double s[V];
#pragma unroll
      for (int v = 0; v < V; ++v) s[v] = 0.0;
      const int end = cp[o + 1];
      for (int z = cp[o]; z < end; ++z) {
        const double w = va[z];
        const VT x = *reinterpret_cast<const VT *>(src + (size_t)ri[z] * post);
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] += w * (double)x[v];
      }
      VT y;
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = (TS)s[v];
      *reinterpret_cast<VT *>(Tout + (size_t)row * post + (size_t)qi * V) = y;
    }
  };
  if (staged) rows(s_cp, s_ri, s_val);
  else rows(M.colptr, M.rowidx, M.val);
}

// scalar form (rows not a multiple of the vector width, unaligned tensors or
// 64-bit indices): one output element per thread; up to four layers (one
// per job) in one launch, each workgroup serving one job (selected from the
// block index, so the job's fields are uniform).  TS: storage type of the
// tensors (float64, or float32 for the convection networks of the mixed
// mode); the sums run in float64
template <typename TS, typename IT>
__global__ __launch_bounds__(256) void k_mpo_csc_grouped(MJobs J, const int *skip) {
  if (skip && *skip) return;
  int ji = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < J.nj && blockIdx.x >= J.j[i].blk0) ji = i;
  const MJob &M = J.j[ji];
  const IT post = (IT)M.post, total = (IT)M.total;
  const int KI = M.KI, KO = M.KO;
  const TS *T = static_cast<const TS *>(M.T);
  TS *Tout = static_cast<TS *>(M.Tout);
  for (IT idx = (IT)(blockIdx.x - M.blk0) * 256 + threadIdx.x; idx < total;
       idx += (IT)M.nblk * 256) {
    const IT q = idx % post;
    const IT t = idx / post;
    const int o = (int)(t % (IT)KO);
    const IT p = t / (IT)KO;
    const TS *src = T + (int64_t)p * KI * post + q;
    double s = 0.0;
    const int end = M.colptr[o + 1];
    for (int z = M.colptr[o]; z < end; ++z) s += M.val[z] * (double)src[(int64_t)M.rowidx[z] * post];
    Tout[idx] = (TS)s;
  }
}

}  // namespace

void mpo_layer_grouped(Ctx &c, int nj, const MpoJob *jobs, const int *skip, bool f32) {
  if (nj < 1 || nj > 4) fail(QTT_E_ARG, "mpo_layer_grouped: 1..4 jobs");
  MJobs J{};
  int64_t blocks = 0, biggest = 0;
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  // vector width of the row form: every job's rows a multiple of it and its
  // tensors aligned to it
  const int V = f32 ? 4 : 2;
  bool vec = true;
  for (int i = 0; i < nj; ++i) {
    const MpoJob &s = jobs[i];
    if (s.pre <= 0 || s.post <= 0) continue;
    if (s.post % V || reinterpret_cast<uintptr_t>(s.T) % (V * es) ||
        reinterpret_cast<uintptr_t>(s.Tout) % (V * es))
      vec = false;
  }
  for (int i = 0; i < nj; ++i) {
    const MpoJob &s = jobs[i];
    if (s.pre <= 0 || s.post <= 0) continue;
    const int KI = 4 * s.mi, KO = 4 * s.mo;
    c.check_range(s.T, 0, s.pre * KI * s.post - 1, es, "mpo_layer in");
    c.check_range(s.Tout, 0, s.pre * KO * s.post - 1, es, "mpo_layer out");
    const MpoCsc &z = s.W->csc[s.rev ? 1 : 0];
    MJob &m = J.j[J.nj++];
    m.T = s.T;
    m.Tout = s.Tout;
    m.colptr = z.colptr + z.cp_off[s.site];
    m.rowidx = z.rowidx + z.nz_off[s.site];
    m.val = z.val + z.nz_off[s.site];
    m.KI = KI;
    m.KO = KO;
    m.post = s.post;
    m.total = s.pre * KO * s.post;
    m.blk0 = (unsigned)blocks;
    const int64_t per = vec ? m.total / V : m.total;
    m.nblk = (unsigned)std::min<int64_t>((per + 255) / 256, 32768);
    blocks += m.nblk;
    biggest = std::max(biggest, m.total + (int64_t)m.nblk * 256 * (vec ? V : 1));
  }
  if (blocks <= 0) return;
  const bool small = biggest < ((int64_t)1 << 31);
  if (vec && small) {
    if (f32)
      hipLaunchKernelGGL((k_mpo_rows_grouped<float, 4>), dim3((unsigned)blocks), dim3(256), 0,
                         c.stream, J, skip);
    else
      hipLaunchKernelGGL((k_mpo_rows_grouped<double, 2>), dim3((unsigned)blocks), dim3(256), 0,
                         c.stream, J, skip);
    HIPC(hipGetLastError());
    return;
  }
  if (f32 && small)
    hipLaunchKernelGGL((k_mpo_csc_grouped<float, unsigned>), dim3((unsigned)blocks), dim3(256), 0,
                       c.stream, J, skip);
  else if (f32)
    hipLaunchKernelGGL((k_mpo_csc_grouped<float, int64_t>), dim3((unsigned)blocks), dim3(256), 0,
                       c.stream, J, skip);
  else if (small)
    hipLaunchKernelGGL((k_mpo_csc_grouped<double, unsigned>), dim3((unsigned)blocks), dim3(256),
                       0, c.stream, J, skip);
  else
    hipLaunchKernelGGL((k_mpo_csc_grouped<double, int64_t>), dim3((unsigned)blocks), dim3(256),
                       0, c.stream, J, skip);
  HIPC(hipGetLastError());
}

void mpo_layer(Ctx &c, const double *T, double *Tout, const Mpo &W, int site, bool rev,
               int64_t pre, int mi, int mo, int64_t post, const int *skip, bool f32) {
  if (pre <= 0 || post <= 0) return;
  const MpoJob j{T, Tout, &W, site, rev, pre, post, mi, mo};
  mpo_layer_grouped(c, 1, &j, skip, f32);
}

}  // namespace qtt
