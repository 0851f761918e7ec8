// MPO layer of a network chain: one site's MPO core applied to an
// intermediate tensor,
//   T'[p][w_out][m'][q] = sum_{m, w_in} W[m][w_in][w_out][m'] T[p][m][w_in][q],
// where p runs over the bra and outer-layer bonds and q over the inner-layer
// and ket bonds.  The finite-difference cores are sparse (12 of 144 entries
// of the bond-3 derivative core, at most 144 of 1296 of a composed bond-9
// penalty core), so this is an HBM-streaming step: one thread per output
// element, which sums the few non-zeros of its output column (compressed
// columns built on the host once per MPO); q is the fastest index so loads
// and stores are unit-stride across a wave.
#include "qtt_internal.h"

namespace qtt {

namespace {

// TS: storage type of the tensors (float64, or float32 for the convection
// networks of the mixed mode); the sums run in float64
template <typename TS, typename IT>
__global__ __launch_bounds__(256) void k_mpo_csc(const TS *T, TS *Tout, const int *colptr,
                                                 const int *rowidx, const double *val, int KI,
                                                 int KO, IT post, IT total, const int *skip) {
  if (skip && *skip) return;
  // IT: 32-bit index arithmetic whenever the tensor fits (the divisions per
  // element are the kernel's main ALU cost)
  for (IT idx = blockIdx.x * (IT)blockDim.x + threadIdx.x; idx < total;
       idx += (IT)gridDim.x * blockDim.x) {
    const IT q = idx % post;
    const IT t = idx / post;
    const int o = (int)(t % (IT)KO);
    const IT p = t / (IT)KO;
    const TS *src = T + (int64_t)p * KI * post + q;
    double s = 0.0;
    const int e = colptr[o + 1];
    for (int z = colptr[o]; z < e; ++z) s += val[z] * (double)src[(int64_t)rowidx[z] * post];
    Tout[idx] = (TS)s;
  }
}

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

// up to four layers (one per job) in one launch; each workgroup serves one
// job (selected from the block index, so the job's fields are uniform)
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
    m.nblk = (unsigned)std::min<int64_t>((m.total + 255) / 256, 32768);
    blocks += m.nblk;
    biggest = std::max(biggest, m.total + (int64_t)m.nblk * 256);
  }
  if (blocks <= 0) return;
  const bool small = biggest < ((int64_t)1 << 31);
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
  const int KI = 4 * mi, KO = 4 * mo;
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  c.check_range(T, 0, pre * KI * post - 1, es, "mpo_layer in");
  c.check_range(Tout, 0, pre * KO * post - 1, es, "mpo_layer out");
  const MpoCsc &z = W.csc[rev ? 1 : 0];
  const int *cp = z.colptr + z.cp_off[site];
  const int *ri = z.rowidx + z.nz_off[site];
  const double *vv = z.val + z.nz_off[site];
  const int64_t total = pre * KO * post;
  int64_t g = (total + 255) / 256;
  if (g > 131072) g = 131072;
  const bool small = total + (int64_t)g * 256 < ((int64_t)1 << 31);
  const float *Tf = reinterpret_cast<const float *>(T);
  float *Tof = reinterpret_cast<float *>(Tout);
  if (f32 && small)
    hipLaunchKernelGGL((k_mpo_csc<float, unsigned>), dim3((unsigned)g), dim3(256), 0, c.stream, Tf,
                       Tof, cp, ri, vv, KI, KO, (unsigned)post, (unsigned)total, skip);
  else if (f32)
    hipLaunchKernelGGL((k_mpo_csc<float, int64_t>), dim3((unsigned)g), dim3(256), 0, c.stream, Tf,
                       Tof, cp, ri, vv, KI, KO, post, total, skip);
  else if (small)
    hipLaunchKernelGGL((k_mpo_csc<double, unsigned>), dim3((unsigned)g), dim3(256), 0, c.stream, T,
                       Tout, cp, ri, vv, KI, KO, (unsigned)post, (unsigned)total, skip);
  else
    hipLaunchKernelGGL((k_mpo_csc<double, int64_t>), dim3((unsigned)g), dim3(256), 0, c.stream, T,
                       Tout, cp, ri, vv, KI, KO, post, total, skip);
  HIPC(hipGetLastError());
}

}  // namespace qtt
