// MPO layer of a network chain: one site's MPO core applied to an
// intermediate tensor,
//   T'[p][w_out][m'][q] = sum_{m, w_in} W[m][w_in][w_out][m'] T[p][m][w_in][q],
// where p runs over the bra and outer-layer bonds and q over the inner-layer
// and ket bonds.  The finite-difference cores are sparse (12 of 144 entries
// of the bond-3 derivative core are non-zero) and tiny, so this is a pure
// HBM-streaming step: each thread owns one q column, reads its 4*mi inputs
// once, writes its 4*mo outputs once, and takes the core from LDS.
#include "qtt_internal.h"

namespace qtt {

namespace {

template <int KI, int KO>
__global__ __launch_bounds__(256) void k_mpo_layer(const double *T, double *Tout, const double *W,
                                                   int64_t post, int nqc, const int *skip) {
  if (skip && *skip) return;
  __shared__ double w[KI * KO];
  for (int i = threadIdx.x; i < KI * KO; i += 256) w[i] = W[i];
  __syncthreads();
  const int64_t b = blockIdx.x;
  const int qc = (int)(b % nqc);
  const int64_t p = b / nqc;
  const int64_t q = (int64_t)qc * 256 + threadIdx.x;
  if (q >= post) return;
  const double *src = T + p * KI * post + q;
  double in[KI];
#pragma unroll
  for (int k = 0; k < KI; ++k) in[k] = src[k * post];
  double *dst = Tout + p * KO * post + q;
#pragma unroll
  for (int o = 0; o < KO; ++o) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
      const double wv = w[k * KO + o];
      if (wv != 0.0) s += wv * in[k];
    }
    dst[o * post] = s;
  }
}

template <int KI, int KO>
void launch_t(Ctx &c, const double *T, double *Tout, const double *W, int64_t pre, int64_t post,
              const int *skip) {
  const int nqc = (int)((post + 255) / 256);
  const int64_t blocks = pre * nqc;
  if (blocks > 0x7fffffffLL) fail(QTT_E_UNSUPPORTED, "mpo_layer grid too large");
  hipLaunchKernelGGL((k_mpo_layer<KI, KO>), dim3((unsigned)blocks), dim3(256), 0, c.stream, T,
                     Tout, W, post, nqc, skip);
  HIPC(hipGetLastError());
}

template <int KI>
void launch_ko(Ctx &c, int mo, const double *T, double *Tout, const double *W, int64_t pre,
               int64_t post, const int *skip) {
  switch (mo) {
    case 1: return launch_t<KI, 4>(c, T, Tout, W, pre, post, skip);
    case 3: return launch_t<KI, 12>(c, T, Tout, W, pre, post, skip);
    case 6: return launch_t<KI, 24>(c, T, Tout, W, pre, post, skip);
    case 9: return launch_t<KI, 36>(c, T, Tout, W, pre, post, skip);
    case 18: return launch_t<KI, 72>(c, T, Tout, W, pre, post, skip);
    default: fail(QTT_E_UNSUPPORTED, "mpo_layer: MPO bond must be 1, 3, 6, 9 or 18");
  }
}

}  // namespace

void mpo_layer(Ctx &c, const double *T, double *Tout, const double *W, int64_t pre, int mi, int mo,
               int64_t post, const int *skip) {
  if (pre <= 0 || post <= 0) return;
  c.check_range(T, 0, pre * mi * 4 * post - 1, 8, "mpo_layer in");
  c.check_range(Tout, 0, pre * mo * 4 * post - 1, 8, "mpo_layer out");
  c.check_range(W, 0, (int64_t)mi * 16 * mo - 1, 8, "mpo_layer core");
  switch (mi) {
    case 1: return launch_ko<4>(c, mo, T, Tout, W, pre, post, skip);
    case 3: return launch_ko<12>(c, mo, T, Tout, W, pre, post, skip);
    case 6: return launch_ko<24>(c, mo, T, Tout, W, pre, post, skip);
    case 9: return launch_ko<36>(c, mo, T, Tout, W, pre, post, skip);
    case 18: return launch_ko<72>(c, mo, T, Tout, W, pre, post, skip);
    default: fail(QTT_E_UNSUPPORTED, "mpo_layer: MPO bond must be 1, 3, 6, 9 or 18");
  }
}

}  // namespace qtt
