// Context, workspace buffers, and the host-side construction of the
// finite-difference MPOs (App. A carry logic, uploaded once per (n, dx)).
#include "qtt_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>

namespace qtt {

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the runtime's last-error state set
    fail(QTT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

double *Ctx::buf(const std::string &name, int64_t ndouble) {
  return (double *)raw(name, (size_t)std::max<int64_t>(ndouble, 1) * sizeof(double));
}

void *Ctx::raw(const std::string &name, size_t bytes) {
  DevBuf &b = bufs[name];
  if (b.bytes < bytes) {
    if (b.ptr) {
      sync();
      HIPC(hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    const size_t alloc = ((bytes + bytes / 4 + 4095) / 4096) * 4096;
    HIPC(hipMalloc(&b.ptr, alloc));
    b.bytes = alloc;
    ranges_dirty = true;
  }
  return b.ptr;
}

void Ctx::sync() { HIPC(hipStreamSynchronize(stream)); }

void Ctx::register_user(const void *p, size_t bytes) {
  if (p && bytes) {
    user_ranges.push_back({(uintptr_t)p, bytes});
    ranges_dirty = true;
  }
}

void Ctx::check_range(const void *p, int64_t lo, int64_t hi, size_t esize,
                      const char *what) const {
  if (hi < lo) return;
  const uintptr_t a = (uintptr_t)p + (intptr_t)(lo * (int64_t)esize);
  const uintptr_t b = (uintptr_t)p + (intptr_t)((hi + 1) * (int64_t)esize);
  if (ranges_dirty) {
    ranges.clear();
    for (auto &kv : bufs)
      if (kv.second.ptr)
        ranges.push_back({(uintptr_t)kv.second.ptr, (uintptr_t)kv.second.ptr + kv.second.bytes});
    for (auto &r : user_ranges) ranges.push_back({r.first, r.first + r.second});
    for (size_t i = 0; i < owned_sizes.size(); ++i)
      ranges.push_back({(uintptr_t)owned[i], (uintptr_t)owned[i] + owned_sizes[i]});
    std::sort(ranges.begin(), ranges.end());
    ranges_dirty = false;
  }
  // the allocation with the largest start at or below a (allocations do not
  // overlap; user ranges may, hence the full scan before failing)
  auto it = std::upper_bound(ranges.begin(), ranges.end(), a,
                             [](uintptr_t v, const std::pair<uintptr_t, uintptr_t> &r) {
                               return v < r.first;
                             });
  if (it != ranges.begin() && b <= std::prev(it)->second) return;
  for (auto &r : ranges)
    if (a >= r.first && b <= r.second) return;
  std::ostringstream s;
  s << what << ": access [" << lo << ", " << hi << "] outside every known allocation";
  fail(QTT_E_ARG, s.str());
}

double *Ctx::alloc_owned(int64_t ndouble) {
  void *p = nullptr;
  const size_t bytes = (size_t)std::max<int64_t>(ndouble, 1) * sizeof(double);
  HIPC(hipMalloc(&p, bytes));
  owned.push_back(p);
  owned_sizes.push_back(bytes);
  ranges_dirty = true;
  return (double *)p;
}

// timing-only events (read after a stream synchronisation): no system-scope
// fence, so recording one costs no cache write-back and the interval between
// two of them is the work between them, as a kernel trace reports it
hipEvent_t Ctx::take_event() {
  if (kt.pool.empty()) {
    hipEvent_t e;
    HIPC(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
  }
  hipEvent_t e = kt.pool.back();
  kt.pool.pop_back();
  return e;
}

void Ctx::resolve_events() {
  sync();
  for (int k = 0; k < KT_KINDS; ++k) {
    for (auto &pr : kt.pending[k]) {
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, pr.first, pr.second));
      kt.timed_ms[k] += ms;
      kt.timed[k] += 1;
      kt.pool.push_back(pr.first);
      kt.pool.push_back(pr.second);
    }
    kt.pending[k].clear();
  }
}

void Ctx::resolve_shapes() {
  sync();
  for (size_t i = 0; i < shape_pending.size(); ++i) {
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, shape_pending[i].second.first, shape_pending[i].second.second));
    ShapeRec &r = shapes[shape_pending[i].first];
    r.calls += 1;
    r.ms += ms;
    r.flops += shape_flops_pending[i];
    kt.pool.push_back(shape_pending[i].second.first);
    kt.pool.push_back(shape_pending[i].second.second);
  }
  shape_pending.clear();
  shape_flops_pending.clear();
}

std::unique_ptr<Ctx> make_worker(const Ctx &parent) {
  std::unique_ptr<Ctx> w(new Ctx());
  w->device = parent.device;
  HIPC(hipSetDevice(parent.device));
  HIPC(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
  w->own_stream = true;
  HIPC(hipHostMalloc((void **)&w->pinned, 4096 * sizeof(double), 0));
  // no stream capture in workers: an allocation or a synchronous copy made by
  // another worker while one captures would invalidate the capture (device-
  // wide synchronisation); eager CG chunks give the same results
  w->use_graphs = false;
  w->autotune = parent.autotune;
  w->svd_max_sweeps = parent.svd_max_sweeps;
  return w;
}

Ctx::~Ctx() {
  if (shape_stats) {
    try {
      resolve_shapes();
    } catch (...) {
    }
    std::vector<std::pair<double, std::string>> v;
    double tot = 0.0;
    for (auto &kv : shapes) {
      v.push_back({kv.second.ms, kv.first});
      tot += kv.second.ms;
    }
    std::sort(v.rbegin(), v.rend());
    std::fprintf(stderr, "[qtt] GEMM shapes by time (total %.1f ms)\n", tot);
    for (size_t i = 0; i < v.size() && i < 40; ++i) {
      const ShapeRec &r = shapes[v[i].second];
      std::fprintf(stderr, "[qtt] %9.2f ms %7lld calls %8.3f TF/s  %s\n", r.ms, (long long)r.calls,
                   r.flops / (r.ms * 1e-3) / 1e12, v[i].second.c_str());
    }
  }
  hipStreamSynchronize(stream);
  for (auto &kv : cg_graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  for (int k = 0; k < KT_KINDS; ++k)
    for (auto &pr : kt.pending[k]) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : kt.pool) hipEventDestroy(e);
  for (auto &kv : bufs)
    if (kv.second.ptr) hipFree(kv.second.ptr);
  for (void *p : owned) hipFree(p);
  if (pinned) hipHostFree(pinned);
  if (own_stream) hipStreamDestroy(stream);
}

Mps from_c(const qtt_mps &m) {
  Mps r;
  if (m.n < 1 || m.n > QTT_MAX_SITES) fail(QTT_E_ARG, "mps: n out of range");
  r.n = m.n;
  for (int k = 0; k <= m.n; ++k) {
    r.bond[k] = m.bond[k];
    if (m.bond[k] < 1) fail(QTT_E_SHAPE, "mps: bond < 1");
  }
  if (m.bond[0] != 1 || m.bond[m.n] != 1) fail(QTT_E_SHAPE, "mps: end bonds must be 1");
  r.data = m.data;
  r.capacity = m.capacity;
  if (r.size() > r.capacity) {
    std::ostringstream s;
    s << "mps: capacity " << r.capacity << " < size " << r.size();
    fail(QTT_E_CAPACITY, s.str());
  }
  if (!r.data) fail(QTT_E_ARG, "mps: null data");
  return r;
}

void to_c(const Mps &m, qtt_mps *out) {
  out->n = m.n;
  for (int k = 0; k <= QTT_MAX_SITES; ++k) out->bond[k] = (k <= m.n) ? m.bond[k] : 0;
}

// ---------------------------------------------------------------- MPO construction
// Central node C[a][w][w'][b] of the periodic first/second difference along
// one axis: the finer sites request op = b (0: keep, 1: +1, 2: -1) on this
// site's bit; a carry (wrap of the bit) is passed to the coarser site as a = op.
static void carry_core(int axis, double *C /* 3*4*4*3 */) {
  std::memset(C, 0, sizeof(double) * 144);
  const int shift = (axis == 1) ? 1 : 0;
  const int delta[3] = {0, 1, -1};
  for (int op = 0; op < 3; ++op)
    for (int w = 0; w < 4; ++w) {
      const int bit = (w >> shift) & 1;
      const int nb = bit + delta[op];
      const int carry = (nb >= 0 && nb <= 1) ? 0 : op;
      const int win = (w & ~(1 << shift)) | (((nb + 2) % 2) << shift);
      C[((carry * 4 + w) * 4 + win) * 3 + op] = 1.0;
    }
}

struct HostMpo {
  int n;
  std::vector<int> bond;
  std::vector<std::vector<double>> core;  // [a][w][w'][b]
};

static HostMpo derivative(int n, int axis, int order, double dx) {
  double C[144];
  carry_core(axis, C);
  double L[3] = {1.0, 1.0, 1.0};
  double R[3];
  if (order == 1) {
    R[0] = 0.0;
    R[1] = 1.0 / (2.0 * dx);
    R[2] = -1.0 / (2.0 * dx);
  } else {
    R[0] = -2.0 / (dx * dx);
    R[1] = 1.0 / (dx * dx);
    R[2] = 1.0 / (dx * dx);
  }
  HostMpo m;
  m.n = n;
  m.bond.assign(n + 1, 3);
  m.bond[0] = 1;
  m.bond[n] = 1;
  for (int k = 0; k < n; ++k) {
    const int al = m.bond[k], ar = m.bond[k + 1];
    std::vector<double> c((size_t)al * 16 * ar, 0.0);
    for (int a = 0; a < al; ++a)
      for (int w = 0; w < 4; ++w)
        for (int v = 0; v < 4; ++v)
          for (int b = 0; b < ar; ++b) {
            double s = 0.0;
            for (int aa = 0; aa < 3; ++aa) {
              if (al != 1 && aa != a) continue;
              const double la = (al == 1) ? L[aa] : 1.0;
              for (int bb = 0; bb < 3; ++bb) {
                if (ar != 1 && bb != b) continue;
                const double rb = (ar == 1) ? R[bb] : 1.0;
                s += la * C[((aa * 4 + w) * 4 + v) * 3 + bb] * rb;
              }
            }
            c[((a * 4 + w) * 4 + v) * ar + b] = s;
          }
    m.core.push_back(c);
  }
  return m;
}

static HostMpo sum(const HostMpo &A, const HostMpo &B) {
  HostMpo m;
  m.n = A.n;
  m.bond.resize(A.n + 1);
  for (int k = 0; k <= A.n; ++k) m.bond[k] = (k == 0 || k == A.n) ? 1 : A.bond[k] + B.bond[k];
  for (int k = 0; k < A.n; ++k) {
    const int al = m.bond[k], ar = m.bond[k + 1];
    std::vector<double> c((size_t)al * 16 * ar, 0.0);
    const int a1 = A.bond[k], b1 = A.bond[k + 1], a2 = B.bond[k], b2 = B.bond[k + 1];
    // A block at offset (0, 0); B block at offset (a1 or 0, b1 or 0)
    const int oa = (k == 0) ? 0 : a1, ob = (k == A.n - 1) ? 0 : b1;
    for (int a = 0; a < a1; ++a)
      for (int wv = 0; wv < 16; ++wv)
        for (int b = 0; b < b1; ++b) c[(a * 16 + wv) * ar + b] += A.core[k][(a * 16 + wv) * b1 + b];
    for (int a = 0; a < a2; ++a)
      for (int wv = 0; wv < 16; ++wv)
        for (int b = 0; b < b2; ++b)
          c[((oa + a) * 16 + wv) * ar + ob + b] += B.core[k][(a * 16 + wv) * b2 + b];
    m.core.push_back(c);
  }
  return m;
}

// W1 W2 (W2 applied first)
static HostMpo compose(const HostMpo &A, const HostMpo &B) {
  HostMpo m;
  m.n = A.n;
  m.bond.resize(A.n + 1);
  for (int k = 0; k <= A.n; ++k) m.bond[k] = A.bond[k] * B.bond[k];
  for (int k = 0; k < A.n; ++k) {
    const int a1 = A.bond[k], b1 = A.bond[k + 1], a2 = B.bond[k], b2 = B.bond[k + 1];
    std::vector<double> c((size_t)a1 * a2 * 16 * b1 * b2, 0.0);
    for (int x = 0; x < a1; ++x)
      for (int y = 0; y < a2; ++y)
        for (int w = 0; w < 4; ++w)
          for (int v = 0; v < 4; ++v)
            for (int p = 0; p < b1; ++p)
              for (int q = 0; q < b2; ++q) {
                double s = 0.0;
                for (int u = 0; u < 4; ++u)
                  s += A.core[k][((x * 4 + w) * 4 + u) * b1 + p] *
                       B.core[k][((y * 4 + u) * 4 + v) * b2 + q];
                c[((((int64_t)(x * a2 + y) * 4 + w) * 4 + v) * b1 + p) * b2 + q] = s;
              }
    m.core.push_back(c);
  }
  return m;
}

static HostMpo transpose(const HostMpo &A) {
  HostMpo m = A;
  for (int k = 0; k < A.n; ++k) {
    const int al = A.bond[k], ar = A.bond[k + 1];
    for (int a = 0; a < al; ++a)
      for (int w = 0; w < 4; ++w)
        for (int v = 0; v < 4; ++v)
          for (int b = 0; b < ar; ++b)
            m.core[k][((a * 4 + w) * 4 + v) * ar + b] = A.core[k][((a * 4 + v) * 4 + w) * ar + b];
  }
  return m;
}

void build_derivative_host(int n, int axis, int order, double dx, std::vector<double> &cores,
                           int *bond) {
  HostMpo m = derivative(n, axis, order, dx);
  cores.clear();
  for (int k = 0; k <= n; ++k) bond[k] = m.bond[k];
  for (auto &c : m.core) cores.insert(cores.end(), c.begin(), c.end());
}

static std::shared_ptr<Mpo> upload(Ctx &c, const HostMpo &h) {
  auto m = std::make_shared<Mpo>();
  m->n = h.n;
  for (int k = 0; k <= h.n; ++k) m->bond[k] = h.bond[k];
  const int64_t tot = m->off(h.n);
  std::vector<double> fwd, perm, rperm;
  fwd.reserve(tot);
  perm.reserve(tot);
  rperm.reserve(tot);
  for (int k = 0; k < h.n; ++k) {
    const int al = h.bond[k], ar = h.bond[k + 1];
    const std::vector<double> &C = h.core[k];
    fwd.insert(fwd.end(), C.begin(), C.end());
    std::vector<double> p(C.size()), rp(C.size());
    for (int a = 0; a < al; ++a)
      for (int w = 0; w < 4; ++w)
        for (int v = 0; v < 4; ++v)
          for (int b = 0; b < ar; ++b) {
            const double x = C[((a * 4 + w) * 4 + v) * ar + b];
            p[((a * 4 + v) * 4 + w) * ar + b] = x;   // [a][w'][w][b]
            rp[((b * 4 + v) * 4 + w) * al + a] = x;  // [b][w'][w][a]
          }
    perm.insert(perm.end(), p.begin(), p.end());
    rperm.insert(rperm.end(), rp.begin(), rp.end());
  }
  // compressed columns of the permuted cores for the streaming MPO kernel
  for (int which = 0; which < 2; ++which) {
    const std::vector<double> &src = which == 0 ? perm : rperm;
    std::vector<int> cp, ri;
    std::vector<double> vv;
    MpoCsc &z = m->csc[which];
    int64_t o = 0;
    for (int k = 0; k < h.n; ++k) {
      const int mi = which == 0 ? h.bond[k] : h.bond[k + 1];
      const int mo = which == 0 ? h.bond[k + 1] : h.bond[k];
      const int KI = 4 * mi, KO = 4 * mo;
      z.cp_off.push_back((int64_t)cp.size());
      z.nz_off.push_back((int64_t)ri.size());
      const int base = (int)ri.size();
      for (int oc = 0; oc < KO; ++oc) {
        cp.push_back((int)ri.size() - base);
        for (int kk = 0; kk < KI; ++kk) {
          const double x = src[o + (int64_t)kk * KO + oc];
          if (x != 0.0) {
            ri.push_back(kk);
            vv.push_back(x);
          }
        }
      }
      cp.push_back((int)ri.size() - base);
      o += (int64_t)KI * KO;
    }
    if (ri.empty()) {
      ri.push_back(0);
      vv.push_back(0.0);
    }
    z.colptr = (int *)c.alloc_owned(((int64_t)cp.size() + 1) / 2 + 1);
    z.rowidx = (int *)c.alloc_owned(((int64_t)ri.size() + 1) / 2 + 1);
    z.val = c.alloc_owned((int64_t)vv.size());
    HIPC(hipMemcpy(z.colptr, cp.data(), cp.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(z.rowidx, ri.data(), ri.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(z.val, vv.data(), vv.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  m->fwd = c.alloc_owned(tot);
  m->perm = c.alloc_owned(tot);
  m->rperm = c.alloc_owned(tot);
  HIPC(hipMemcpy(m->fwd, fwd.data(), tot * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(m->perm, perm.data(), tot * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(m->rperm, rperm.data(), tot * sizeof(double), hipMemcpyHostToDevice));
  return m;
}

// kinds: "D1", "D2", "D1T", "D2T", "P11", "P12", "P21", "P22" (D_i^T D_j), "LAP"
std::shared_ptr<Mpo> get_mpo(Ctx &c, int n, const std::string &kind, double dx, int lap_mode) {
  std::ostringstream key;
  key.precision(17);
  key << kind << ':' << n << ':' << dx << ':' << lap_mode;
  auto it = c.mpos.find(key.str());
  if (it != c.mpos.end()) return it->second;
  HostMpo h;
  if (kind == "D1") h = derivative(n, 1, 1, dx);
  else if (kind == "D2") h = derivative(n, 2, 1, dx);
  else if (kind == "D1T") h = transpose(derivative(n, 1, 1, dx));
  else if (kind == "D2T") h = transpose(derivative(n, 2, 1, dx));
  else if (kind.size() == 3 && kind[0] == 'P') {
    // penalty pair D_i^T D_j (i, j in {1, 2}) as one MPO of bond 9
    const int i = kind[1] - '0', j = kind[2] - '0';
    h = compose(transpose(derivative(n, i, 1, dx)), derivative(n, j, 1, dx));
  } else if (kind == "LAP") {
    if (lap_mode == 0)
      h = sum(derivative(n, 1, 2, dx), derivative(n, 2, 2, dx));
    else {
      HostMpo a = derivative(n, 1, 1, dx), b = derivative(n, 2, 1, dx);
      h = sum(compose(a, a), compose(b, b));
    }
  } else fail(QTT_E_ARG, "unknown mpo kind " + kind);
  auto m = upload(c, h);
  c.mpos[key.str()] = m;
  return m;
}

}  // namespace qtt
