// qtt_inner_noalloc: the inner product <x|y> of two MPS without any device
// allocation, for callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The contraction is the same as qtt_inner's (the left environment of the
// two-layer network <x|y>, advanced one site at a time), with its two
// environment buffers and the per-site intermediate held in a file-scope
// device array of fixed size instead of context workspace.  Each device
// that runs this holds one copy of the array until the process ends; every
// call on a device shares that copy, so calls that overlap on one device
// (different streams, different host threads) race.
#include "qtt.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

// largest bond product x.bond[s] * y.bond[s'] a call may need (s' = s or s + 1)
constexpr int64_t NOALLOC_MAX_BOND_PRODUCT = 65536;
// E0, E1: one bond product each; T: four
constexpr int64_t NOALLOC_DOUBLES = 6 * NOALLOC_MAX_BOND_PRODUCT;  // 3 MiB

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_scratch[MAX_DEVICES] = {};

// device address of this device's copy of `scratch` (looked up once per
// device, with that device current); null on failure
double *scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = static_cast<double *>(p);
  }
  return g_scratch[dev];
}

__global__ void k_na_one(double *E) { E[0] = 1.0; }

// T[a][(w b')] = sum_b E[a][b] Y[b][(w b')]; one output per thread
__global__ void k_na_ket(const double *__restrict__ E, const double *__restrict__ Y,
                         double *__restrict__ T, int lx, int ly, int ry) {
  const int64_t cols = 4 * (int64_t)ry;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)lx * cols) return;
  const int64_t a = i / cols, wb = i - a * cols;
  const double *e = E + a * ly;
  double s = 0.0;
  for (int b = 0; b < ly; ++b) s = fma(e[b], Y[b * cols + wb], s);
  T[i] = s;
}

// E'[a'][b'] = sum_(a w) X[(a w)][a'] T[(a w)][b']; one output per thread
__global__ void k_na_bra(const double *__restrict__ X, const double *__restrict__ T,
                         double *__restrict__ E, int lx, int rx, int ry) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rx * ry) return;
  const int ap = (int)(i / ry), bp = (int)(i - (int64_t)ap * ry);
  const int K = 4 * lx;
  double s = 0.0;
  for (int k = 0; k < K; ++k) s = fma(X[(int64_t)k * rx + ap], T[(int64_t)k * ry + bp], s);
  E[i] = s;
}

__global__ void k_na_out(const double *E, double *out) { out[0] = E[0]; }

int64_t mps_doubles(const qtt_mps &m) {
  int64_t s = 0;
  for (int k = 0; k < m.n; ++k) s += (int64_t)m.bond[k] * 4 * m.bond[k + 1];
  return s;
}

bool valid(const qtt_mps *m) {
  if (!m || !m->data || m->n < 1 || m->n > QTT_MAX_SITES) return false;
  if (m->bond[0] != 1 || m->bond[m->n] != 1) return false;
  for (int k = 1; k < m->n; ++k)
    if (m->bond[k] < 1) return false;
  return mps_doubles(*m) <= m->capacity;
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

extern "C" int qtt_inner_noalloc(void *hip_stream, const qtt_mps *x, const qtt_mps *y,
                                 double *out) {
  if (!valid(x) || !valid(y) || !out || x->n != y->n) return QTT_E_ARG;
  const int n = x->n;
  for (int s = 0; s < n; ++s) {
    const int64_t e = (int64_t)x->bond[s] * y->bond[s];
    const int64_t t = (int64_t)x->bond[s] * y->bond[s + 1];
    if (e > NOALLOC_MAX_BOND_PRODUCT || t > NOALLOC_MAX_BOND_PRODUCT) return QTT_E_CAPACITY;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return QTT_E_HIP;
  double *base = scratch_ptr(dev);
  if (!base) return QTT_E_HIP;
  double *E0 = base, *E1 = base + NOALLOC_MAX_BOND_PRODUCT;
  double *T = base + 2 * NOALLOC_MAX_BOND_PRODUCT;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  constexpr int TH = 256;
  k_na_one<<<1, 1, 0, st>>>(E0);
  const double *xc = x->data, *yc = y->data;
  for (int s = 0; s < n; ++s) {
    const int lx = x->bond[s], rx = x->bond[s + 1], ly = y->bond[s], ry = y->bond[s + 1];
    k_na_ket<<<blocks_for((int64_t)lx * 4 * ry, TH), TH, 0, st>>>(E0, yc, T, lx, ly, ry);
    k_na_bra<<<blocks_for((int64_t)rx * ry, TH), TH, 0, st>>>(xc, T, E1, lx, rx, ry);
    double *t = E0;
    E0 = E1;
    E1 = t;
    xc += (int64_t)lx * 4 * rx;
    yc += (int64_t)ly * 4 * ry;
  }
  k_na_out<<<1, 1, 0, st>>>(E0, out);
  return hipGetLastError() == hipSuccess ? QTT_OK : QTT_E_HIP;
}
