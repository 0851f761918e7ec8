// extern "C" entry points declared in include/qtt.h.  Each converts the C
// descriptors, runs the device work on the context stream, and maps
// qtt::Error to the return code (message kept for qtt_last_error).
#include "qtt_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <thread>
#include <vector>

static_assert(qtt::PC_IN == QTT_PC_IN && qtt::PC_W == QTT_PC_WIDTH && qtt::PC_OUT == QTT_PC_OUT,
              "preconditioner sizes");

struct qtt_ctx {
  qtt::Ctx c;
};

namespace {

template <typename F>
int guard(qtt_ctx *ctx, F &&f) {
  if (!ctx) return QTT_E_ARG;
  ctx->c.err.clear();
  ctx->c.clear_user();
  ctx->c.warn = 0;
  try {
    HIPC(hipSetDevice(ctx->c.device));
    if (ctx->c.own_stream) HIPC(hipStreamSynchronize(nullptr));
    f();
    if (ctx->c.warn) ctx->c.err = "warning raised inside the call (see the return code)";
    return ctx->c.warn;
  } catch (qtt::Error &e) {
    ctx->c.err = e.msg;
    (void)hipGetLastError();
    if (e.code > 0) return std::max(e.code, ctx->c.warn);
    // leave the stream idle before reporting
    hipStreamSynchronize(ctx->c.stream);
    return e.code;
  } catch (std::exception &e) {
    ctx->c.err = e.what();
    return QTT_E_HIP;
  }
}

void reg(qtt::Ctx &c, const qtt_mps &m) { c.register_user(m.data, (size_t)m.capacity * 8); }

void check_finite(qtt::Ctx &c, const qtt::Mps &x, const char *what) {
  if (qtt::any_nonfinite(c, x.data, x.size())) qtt::fail(QTT_E_NAN, std::string(what) + ": NaN/Inf");
}

void check_params(const qtt_params *p) {
  if (!p) qtt::fail(QTT_E_ARG, "params: null");
  if (!(p->dx > 0.0) || !(p->re > 0.0) || !(p->mu >= 0.0) || p->chi < 1)
    qtt::fail(QTT_E_ARG, "params: dx, re must be > 0, mu >= 0, chi >= 1");
  if (!(p->cg_rtol >= 0.0) || p->cg_maxit < 1 || p->max_sweeps < 1)
    qtt::fail(QTT_E_ARG, "params: cg_rtol >= 0, cg_maxit >= 1, max_sweeps >= 1");
  if (p->lap_mode != 0 && p->lap_mode != 1) qtt::fail(QTT_E_ARG, "params: lap_mode");
  if (p->rhs_mode != 0 && p->rhs_mode != 1) qtt::fail(QTT_E_ARG, "params: rhs_mode");
  if (p->fit_sweeps < 0) qtt::fail(QTT_E_ARG, "params: fit_sweeps >= 0");
}

}  // namespace

extern "C" {

int qtt_ctx_create(qtt_ctx **out, int device, void *hip_stream) {
  if (!out) return QTT_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QTT_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return QTT_E_HIP;
  qtt_ctx *c = new qtt_ctx();
  c->c.device = device;
  c->c.stream = (hipStream_t)hip_stream;
  if (!c->c.stream) {
    // the legacy null stream cannot be captured into graphs: work goes to a
    // context-owned stream (default priority) that first waits for the null
    // stream at every call; every call ends with a stream synchronisation
    if (hipStreamCreateWithFlags(&c->c.stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      return QTT_E_HIP;
    }
    c->c.own_stream = true;
  }
  if (hipHostMalloc((void **)&c->c.pinned, 4096 * sizeof(double), 0) != hipSuccess) {
    (void)hipGetLastError();
    c->c.pinned = nullptr;
    delete c;
    return QTT_E_HIP;
  }
  const char *t = std::getenv("QTT_TIMING");
  c->c.timing = (t && t[0] == '1');
  const char *gr = std::getenv("QTT_GRAPHS");
  c->c.use_graphs = !(gr && gr[0] == '0');
  const char *at = std::getenv("QTT_AUTOTUNE");
  c->c.autotune = (at && at[0] == '1');
  const char *gs = std::getenv("QTT_GEMM_STATS");
  c->c.shape_stats = (gs && gs[0] == '1');
  const char *sv = std::getenv("QTT_SVD_MAX_SWEEPS");
  if (sv && std::atoi(sv) > 0) c->c.svd_max_sweeps = std::atoi(sv);
  *out = c;
  return QTT_OK;
}

void qtt_ctx_destroy(qtt_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->c.device);
  delete ctx;
}

const char *qtt_last_error(const qtt_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int64_t qtt_mps_size(int32_t n, const int32_t *bond) {
  if (n < 1 || n > QTT_MAX_SITES || !bond) return -1;
  int64_t s = 0;
  for (int k = 0; k < n; ++k) s += (int64_t)bond[k] * 4 * bond[k + 1];
  return s;
}

int qtt_mpo_derivative(qtt_ctx *ctx, int32_t n, int32_t axis, int32_t order, double dx,
                       qtt_mpo *out) {
  return guard(ctx, [&] {
    if (!out || n < 1 || n > QTT_MAX_SITES || (axis != 1 && axis != 2) ||
        (order != 1 && order != 2) || !(dx > 0.0))
      qtt::fail(QTT_E_ARG, "mpo_derivative: bad arguments");
    std::vector<double> cores;
    int bond[QTT_MAX_SITES + 1];
    qtt::build_derivative_host(n, axis, order, dx, cores, bond);
    if ((int64_t)cores.size() > out->capacity) {
      std::ostringstream s;
      s << "mpo_derivative: needs " << cores.size() << " doubles";
      qtt::fail(QTT_E_CAPACITY, s.str());
    }
    if (!out->data) qtt::fail(QTT_E_ARG, "mpo_derivative: null data");
    out->n = n;
    for (int k = 0; k <= QTT_MAX_SITES; ++k) out->bond[k] = (k <= n) ? bond[k] : 0;
    HIPC(hipMemcpyAsync(out->data, cores.data(), cores.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->c.stream));
    ctx->c.sync();
  });
}

int qtt_add(qtt_ctx *ctx, int32_t k, const double *coef, const qtt_mps *x, qtt_mps *y) {
  return guard(ctx, [&] {
    if (k < 1 || !coef || !x || !y) qtt::fail(QTT_E_ARG, "add: bad arguments");
    std::vector<qtt::Mps> xs;
    for (int j = 0; j < k; ++j) {
      reg(ctx->c, x[j]);
      xs.push_back(qtt::from_c(x[j]));
    }
    reg(ctx->c, *y);
    qtt::Mps out;
    out.data = y->data;
    out.capacity = y->capacity;
    if (!out.data) qtt::fail(QTT_E_ARG, "add: null output");
    qtt::mps_add(ctx->c, k, coef, xs.data(), out);
    ctx->c.sync();
    qtt::to_c(out, y);
  });
}

int qtt_truncate(qtt_ctx *ctx, qtt_mps *y, int32_t chi, double svd_rtol, double *discarded_sq) {
  return guard(ctx, [&] {
    if (!y || chi < 1 || !(svd_rtol >= 0.0)) qtt::fail(QTT_E_ARG, "truncate: bad arguments");
    reg(ctx->c, *y);
    qtt::Mps m = qtt::from_c(*y);
    double disc = 0.0;
    qtt::mps_truncate(ctx->c, {&m}, chi, svd_rtol, &disc);
    qtt::to_c(m, y);
    if (discarded_sq) *discarded_sq = disc;
  });
}

int qtt_apply_mpo(qtt_ctx *ctx, const qtt_mpo *W, const qtt_mps *x, int32_t chi, double svd_rtol,
                  qtt_mps *y, double *discarded_sq) {
  return guard(ctx, [&] {
    if (!W || !x || !y || chi < 0) qtt::fail(QTT_E_ARG, "apply_mpo: bad arguments");
    reg(ctx->c, *x);
    reg(ctx->c, *y);
    ctx->c.register_user(W->data, (size_t)W->capacity * 8);
    qtt::Mps xm = qtt::from_c(*x);
    if (W->n != xm.n || !W->data) qtt::fail(QTT_E_SHAPE, "apply_mpo: MPO does not match");
    qtt::Mpo w;
    w.n = W->n;
    for (int k = 0; k <= W->n; ++k) w.bond[k] = W->bond[k];
    if (w.bond[0] != 1 || w.bond[w.n] != 1) qtt::fail(QTT_E_SHAPE, "apply_mpo: MPO end bonds");
    if (w.off(w.n) > W->capacity) qtt::fail(QTT_E_CAPACITY, "apply_mpo: MPO capacity");
    w.fwd = W->data;
    qtt::Mps out;
    out.data = y->data;
    out.capacity = y->capacity;
    qtt::mps_apply_mpo(ctx->c, w, xm, out);
    double disc = 0.0;
    if (chi > 0) qtt::mps_truncate(ctx->c, {&out}, chi, svd_rtol, &disc);
    ctx->c.sync();
    qtt::to_c(out, y);
    if (discarded_sq) *discarded_sq = disc;
  });
}

int qtt_hadamard(qtt_ctx *ctx, const qtt_mps *a, const qtt_mps *b, int32_t chi, double svd_rtol,
                 qtt_mps *y, double *discarded_sq) {
  return guard(ctx, [&] {
    if (!a || !b || !y || chi < 0) qtt::fail(QTT_E_ARG, "hadamard: bad arguments");
    reg(ctx->c, *a);
    reg(ctx->c, *b);
    reg(ctx->c, *y);
    qtt::Mps am = qtt::from_c(*a), bm = qtt::from_c(*b);
    qtt::Mps out;
    out.data = y->data;
    out.capacity = y->capacity;
    qtt::mps_hadamard(ctx->c, am, bm, out);
    double disc = 0.0;
    if (chi > 0) qtt::mps_truncate(ctx->c, {&out}, chi, svd_rtol, &disc);
    ctx->c.sync();
    qtt::to_c(out, y);
    if (discarded_sq) *discarded_sq = disc;
  });
}

int qtt_inner(qtt_ctx *ctx, const qtt_mps *x, const qtt_mps *y, double *out) {
  return guard(ctx, [&] {
    if (!x || !y || !out) qtt::fail(QTT_E_ARG, "inner: bad arguments");
    reg(ctx->c, *x);
    reg(ctx->c, *y);
    *out = qtt::mps_inner(ctx->c, qtt::from_c(*x), qtt::from_c(*y));
  });
}

int qtt_to_dense(qtt_ctx *ctx, const qtt_mps *x, double *grid) {
  return guard(ctx, [&] {
    if (!x || !grid) qtt::fail(QTT_E_ARG, "to_dense: bad arguments");
    reg(ctx->c, *x);
    if (x->n < 1 || x->n > 13) qtt::fail(QTT_E_UNSUPPORTED, "to_dense: n must be 1..13");
    ctx->c.register_user(grid, ((size_t)1 << (2 * x->n)) * 8);
    qtt::mps_to_dense(ctx->c, qtt::from_c(*x), grid);
    ctx->c.sync();
  });
}

int qtt_from_dense(qtt_ctx *ctx, const double *grid, int32_t n, int32_t chi, double svd_rtol,
                   qtt_mps *out) {
  return guard(ctx, [&] {
    if (!grid || !out || chi < 1 || !(svd_rtol >= 0.0)) qtt::fail(QTT_E_ARG, "from_dense: bad arguments");
    if (n < 1 || n > 13) qtt::fail(QTT_E_UNSUPPORTED, "from_dense: n must be 1..13");
    ctx->c.register_user(grid, ((size_t)1 << (2 * n)) * 8);
    reg(ctx->c, *out);
    qtt::Mps m;
    m.data = out->data;
    m.capacity = out->capacity;
    if (!m.data) qtt::fail(QTT_E_ARG, "from_dense: null output");
    qtt::mps_from_dense(ctx->c, grid, n, chi, svd_rtol, m);
    qtt::to_c(m, out);
  });
}

int qtt_schmidt_counts(qtt_ctx *ctx, const double *grid, int32_t n, double eps, int32_t chi_cap,
                       int32_t *counts) {
  return guard(ctx, [&] {
    if (!grid || !counts || chi_cap < 1 || !(eps >= 0.0))
      qtt::fail(QTT_E_ARG, "schmidt_counts: bad arguments");
    if (n < 2 || n > 13) qtt::fail(QTT_E_UNSUPPORTED, "schmidt_counts: n must be 2..13");
    ctx->c.register_user(grid, ((size_t)1 << (2 * n)) * 8);
    qtt::schmidt_counts(ctx->c, grid, n, eps, chi_cap, counts);
  });
}

int qtt_dns_rhs(qtt_ctx *ctx, const double *u1, const double *u2, double *f1, double *f2,
                int32_t n, double re) {
  return guard(ctx, [&] {
    if (!u1 || !u2 || !f1 || !f2 || !(re > 0.0)) qtt::fail(QTT_E_ARG, "dns_rhs: bad arguments");
    if (n < 3 || n > 11) qtt::fail(QTT_E_UNSUPPORTED, "dns_rhs: n must be 3..11");
    const size_t bytes = ((size_t)1 << (2 * n)) * 8;
    for (const double *p : {u1, u2, (const double *)f1, (const double *)f2})
      ctx->c.register_user(p, bytes);
    qtt::dns_rhs(ctx->c, u1, u2, f1, f2, n, re);
    ctx->c.sync();
  });
}

int qtt_dns_project(qtt_ctx *ctx, double *u1, double *u2, int32_t n) {
  return guard(ctx, [&] {
    if (!u1 || !u2) qtt::fail(QTT_E_ARG, "dns_project: bad arguments");
    if (n < 3 || n > 11) qtt::fail(QTT_E_UNSUPPORTED, "dns_project: n must be 3..11");
    const size_t bytes = ((size_t)1 << (2 * n)) * 8;
    ctx->c.register_user(u1, bytes);
    ctx->c.register_user(u2, bytes);
    qtt::dns_project(ctx->c, u1, u2, n);
    ctx->c.sync();
  });
}

int qtt_dns_step(qtt_ctx *ctx, double *u1, double *u2, int32_t n, double re, double dt,
                 int32_t order, int32_t steps) {
  return guard(ctx, [&] {
    if (!u1 || !u2 || !(re > 0.0) || !std::isfinite(dt) || steps < 0 ||
        (order != 1 && order != 4))
      qtt::fail(QTT_E_ARG, "dns_step: bad arguments");
    if (n < 3 || n > 11) qtt::fail(QTT_E_UNSUPPORTED, "dns_step: n must be 3..11");
    const size_t bytes = ((size_t)1 << (2 * n)) * 8;
    ctx->c.register_user(u1, bytes);
    ctx->c.register_user(u2, bytes);
    qtt::dns_step(ctx->c, u1, u2, n, re, dt, order, steps);
    ctx->c.sync();
  });
}

int qtt_fidelity(qtt_ctx *ctx, const double *a, const double *b, int64_t len, double *F) {
  return guard(ctx, [&] {
    if (!a || !b || !F || len < 1) qtt::fail(QTT_E_ARG, "fidelity: bad arguments");
    ctx->c.register_user(a, (size_t)len * 8);
    ctx->c.register_user(b, (size_t)len * 8);
    double *d = ctx->c.buf("fidelity_dots", 3);
    qtt::fidelity(ctx->c, a, b, len, d);
    double h[3];
    HIPC(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->c.stream));
    ctx->c.sync();
    *F = (h[1] > 0.0 && h[2] > 0.0) ? (h[0] * h[0]) / (h[1] * h[2]) : 0.0;
  });
}

int32_t qtt_tke_shells(int32_t n) {
  if (n < 3 || n > 11) return 0;
  return qtt::tke_shells(n);
}

int qtt_tke_spectrum(qtt_ctx *ctx, const double *u1, const double *u2, const double *mean1,
                     const double *mean2, int32_t n, double *E, int32_t nshell) {
  return guard(ctx, [&] {
    if (!u1 || !u2 || !E || (!mean1) != (!mean2)) qtt::fail(QTT_E_ARG, "tke_spectrum: bad arguments");
    if (n < 3 || n > 11) qtt::fail(QTT_E_UNSUPPORTED, "tke_spectrum: n must be 3..11");
    if (nshell != qtt::tke_shells(n)) qtt::fail(QTT_E_ARG, "tke_spectrum: nshell must be qtt_tke_shells(n)");
    const size_t bytes = ((size_t)1 << (2 * n)) * 8;
    ctx->c.register_user(u1, bytes);
    ctx->c.register_user(u2, bytes);
    if (mean1) {
      ctx->c.register_user(mean1, bytes);
      ctx->c.register_user(mean2, bytes);
    }
    double *d = ctx->c.buf("tke_out", nshell);
    qtt::dns_tke(ctx->c, u1, u2, mean1, mean2, n, d);
    HIPC(hipMemcpyAsync(E, d, (size_t)nshell * 8, hipMemcpyDeviceToHost, ctx->c.stream));
    ctx->c.sync();
  });
}

int qtt_project(qtt_ctx *ctx, const qtt_mps *a, const qtt_mps *b, double h, const qtt_params *p,
                qtt_mps *v, qtt_stats *stats) {
  return guard(ctx, [&] {
    check_params(p);
    if (!a || !b || !v) qtt::fail(QTT_E_ARG, "project: bad arguments");
    for (int i = 0; i < 2; ++i) {
      reg(ctx->c, a[i]);
      reg(ctx->c, b[i]);
      reg(ctx->c, v[i]);
    }
    qtt::Mps am[2] = {qtt::from_c(a[0]), qtt::from_c(a[1])};
    qtt::Mps bm[2] = {qtt::from_c(b[0]), qtt::from_c(b[1])};
    qtt::Mps vm[2] = {qtt::from_c(v[0]), qtt::from_c(v[1])};
    for (int i = 0; i < 2; ++i) {
      check_finite(ctx->c, am[i], "project: a");
      check_finite(ctx->c, bm[i], "project: b");
      check_finite(ctx->c, vm[i], "project: guess");
    }
    if (stats) std::memset(stats, 0, sizeof(qtt_stats));
    int warn = 0;
    try {
      qtt::project(ctx->c, am, bm, h, *p, vm, stats, 0);
    } catch (qtt::Error &e) {
      if (e.code <= 0) throw;
      warn = e.code;
    }
    qtt::to_c(vm[0], &v[0]);
    qtt::to_c(vm[1], &v[1]);
    if (warn) throw qtt::Error{warn, "project: warning"};
  });
}

int qtt_rk4_step(qtt_ctx *ctx, qtt_mps *u, const qtt_params *p, qtt_stats *stats) {
  return guard(ctx, [&] {
    check_params(p);
    if (!u) qtt::fail(QTT_E_ARG, "rk4_step: bad arguments");
    reg(ctx->c, u[0]);
    reg(ctx->c, u[1]);
    qtt::Mps um[2] = {qtt::from_c(u[0]), qtt::from_c(u[1])};
    for (int i = 0; i < 2; ++i) check_finite(ctx->c, um[i], "rk4_step: state");
    if (stats) std::memset(stats, 0, sizeof(qtt_stats));
    int warn = 0;
    try {
      qtt::rk4_step(ctx->c, um, *p, stats);
    } catch (qtt::Error &e) {
      if (e.code <= 0) throw;
      warn = e.code;
    }
    qtt::to_c(um[0], &u[0]);
    qtt::to_c(um[1], &u[1]);
    if (warn) throw qtt::Error{warn, "rk4_step: warning"};
  });
}

int qtt_rk_step(qtt_ctx *ctx, qtt_mps *u, const qtt_params *p, int32_t order, qtt_stats *stats) {
  return guard(ctx, [&] {
    check_params(p);
    if (!u || (order != 1 && order != 2 && order != 4))
      qtt::fail(QTT_E_ARG, "rk_step: bad arguments (order 1, 2 or 4)");
    reg(ctx->c, u[0]);
    reg(ctx->c, u[1]);
    qtt::Mps um[2] = {qtt::from_c(u[0]), qtt::from_c(u[1])};
    for (int i = 0; i < 2; ++i) check_finite(ctx->c, um[i], "rk_step: state");
    if (stats) std::memset(stats, 0, sizeof(qtt_stats));
    int warn = 0;
    try {
      qtt::rk_step(ctx->c, um, *p, order, stats);
    } catch (qtt::Error &e) {
      if (e.code <= 0) throw;
      warn = e.code;
    }
    qtt::to_c(um[0], &u[0]);
    qtt::to_c(um[1], &u[1]);
    if (warn) throw qtt::Error{warn, "rk_step: warning"};
  });
}

int qtt_rk4_step_batched(qtt_ctx *ctx, int32_t nflows, qtt_mps *u, const qtt_params *p,
                         qtt_stats *stats, int32_t workers) {
  return guard(ctx, [&] {
    if (nflows < 0 || (nflows > 0 && (!u || !p)) || workers < 0)
      qtt::fail(QTT_E_ARG, "rk4_step_batched: bad arguments");
    if (nflows == 0) return;
    for (int f = 0; f < nflows; ++f) check_params(&p[f]);
    qtt::Ctx &c = ctx->c;
    const int W = std::max(1, std::min({workers == 0 ? 4 : (int)workers, (int)nflows, 8}));
    while ((int)c.workers.size() < W) c.workers.push_back(qtt::make_worker(c));
    // the workers' streams start after the work already on the caller's stream
    hipEvent_t ev;
    HIPC(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPC(hipEventRecord(ev, c.stream));
    for (int w = 0; w < W; ++w) HIPC(hipStreamWaitEvent(c.workers[w]->stream, ev, 0));
    std::vector<int> codes(nflows, 0);
    std::vector<std::string> msgs(nflows);
    std::vector<std::thread> th;
    for (int w = 0; w < W; ++w)
      th.emplace_back([&, w] {
        (void)hipSetDevice(c.device);
        qtt::Ctx &wc = *c.workers[w];
        for (int f = w; f < nflows; f += W) {
          wc.err.clear();
          wc.clear_user();
          wc.warn = 0;
          try {
            reg(wc, u[2 * f]);
            reg(wc, u[2 * f + 1]);
            qtt::Mps um[2] = {qtt::from_c(u[2 * f]), qtt::from_c(u[2 * f + 1])};
            for (int i = 0; i < 2; ++i) check_finite(wc, um[i], "rk4_step_batched: state");
            qtt_stats *sf = stats ? &stats[f] : nullptr;
            if (sf) std::memset(sf, 0, sizeof(qtt_stats));
            try {
              qtt::rk4_step(wc, um, p[f], sf);
            } catch (qtt::Error &e) {
              if (e.code <= 0) throw;
              codes[f] = e.code;
            }
            qtt::to_c(um[0], &u[2 * f]);
            qtt::to_c(um[1], &u[2 * f + 1]);
            codes[f] = std::max(codes[f], wc.warn);
          } catch (qtt::Error &e) {
            codes[f] = e.code;
            msgs[f] = e.msg;
            (void)hipGetLastError();
            (void)hipStreamSynchronize(wc.stream);
          } catch (std::exception &e) {
            codes[f] = QTT_E_HIP;
            msgs[f] = e.what();
          }
        }
      });
    for (auto &t : th) t.join();
    (void)hipEventDestroy(ev);
    int err = 0, warn = 0;
    std::string msg;
    for (int f = 0; f < nflows; ++f) {
      if (codes[f] < 0 && (err == 0 || codes[f] < err)) {
        err = codes[f];
        msg = "rk4_step_batched: flow " + std::to_string(f) + ": " + msgs[f];
      } else if (codes[f] > 0) {
        warn = std::max(warn, codes[f]);
      }
    }
    if (err < 0) qtt::fail(err, msg);
    if (warn) throw qtt::Error{warn, "rk4_step_batched: warning"};
  });
}

int qtt_kernel_timing(qtt_ctx *ctx, int32_t enable, int32_t sample_every) {
  return guard(ctx, [&] {
    qtt::Ctx &c = ctx->c;
    c.resolve_events();
    for (int k = 0; k < qtt::KT_KINDS; ++k) {
      c.kt.launches[k] = 0;
      c.kt.timed[k] = 0;
      c.kt.timed_ms[k] = 0.0;
    }
    c.kt.every = sample_every < 1 ? 1 : sample_every;
    c.kt.on = enable != 0;
    if (c.kt.on) {
      c.kt.flop_ctr = (double *)c.raw("kt_flops", qtt::KT_KINDS * sizeof(double));
      HIPC(hipMemsetAsync(c.kt.flop_ctr, 0, qtt::KT_KINDS * sizeof(double), c.stream));
      c.sync();
    }
  });
}

int qtt_kernel_stats_read(qtt_ctx *ctx, int32_t kernel, qtt_kernel_stats *out) {
  return guard(ctx, [&] {
    if (!out || kernel < 0 || kernel >= qtt::KT_KINDS)
      qtt::fail(QTT_E_ARG, "kernel_stats_read: bad arguments");
    qtt::Ctx &c = ctx->c;
    c.resolve_events();
    double fl[qtt::KT_KINDS] = {0.0, 0.0, 0.0, 0.0};
    if (c.kt.flop_ctr)
      HIPC(hipMemcpy(fl, c.kt.flop_ctr, qtt::KT_KINDS * sizeof(double), hipMemcpyDeviceToHost));
    out->launches = c.kt.launches[kernel];
    out->timed = c.kt.timed[kernel];
    out->flops = fl[kernel];
    out->timed_ms = c.kt.timed_ms[kernel];
  });
}

int qtt_precond_config(qtt_ctx *ctx, int32_t train_per_solve, double lr, uint64_t seed,
                       int32_t reset) {
  return guard(ctx, [&] {
    if (train_per_solve < 0 || !(lr > 0.0)) qtt::fail(QTT_E_ARG, "precond_config: bad arguments");
    qtt::Ctx &c = ctx->c;
    if (reset || !c.pc.ready) qtt::pc_reset(c, seed);
    c.pc.train_per_solve = train_per_solve;
    c.pc.lr = lr;
  });
}

int qtt_precond_info(qtt_ctx *ctx, int64_t *nparam, int64_t *steps, double *first_loss,
                     double *last_loss) {
  return guard(ctx, [&] {
    const qtt::PrecondNet &net = ctx->c.pc;
    if (nparam) *nparam = net.param_count();
    if (steps) *steps = net.steps;
    if (first_loss) *first_loss = net.first_loss;
    if (last_loss) *last_loss = net.last_loss;
  });
}

int qtt_precond_weights(qtt_ctx *ctx, int32_t set, double *w, int64_t n) {
  return guard(ctx, [&] {
    qtt::Ctx &c = ctx->c;
    qtt::pc_init(c);
    if (!w || n != c.pc.nparam) qtt::fail(QTT_E_ARG, "precond_weights: n must equal nparam");
    c.sync();
    if (set) {
      HIPC(hipMemcpy(c.pc.w, w, n * sizeof(double), hipMemcpyHostToDevice));
    } else {
      HIPC(hipMemcpy(w, c.pc.w, n * sizeof(double), hipMemcpyDeviceToHost));
    }
  });
}

// file form of the weights: 8-byte tag, four int64 (nparam, QTT_PC_IN,
// QTT_PC_WIDTH, QTT_PC_OUT), then nparam float64, host byte order
static const char PC_TAG[8] = {'Q', 'T', 'T', 'P', 'C', 'N', 'E', 'T'};

int qtt_precond_save(qtt_ctx *ctx, const char *path) {
  return guard(ctx, [&] {
    qtt::Ctx &c = ctx->c;
    qtt::pc_init(c);
    if (!path) qtt::fail(QTT_E_ARG, "precond_save: null path");
    std::vector<double> w(c.pc.nparam);
    c.sync();
    HIPC(hipMemcpy(w.data(), c.pc.w, w.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::FILE *f = std::fopen(path, "wb");
    if (!f) qtt::fail(QTT_E_ARG, std::string("precond_save: cannot open ") + path);
    const int64_t hdr[4] = {(int64_t)w.size(), QTT_PC_IN, QTT_PC_WIDTH, QTT_PC_OUT};
    bool ok = std::fwrite(PC_TAG, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(w.data(), sizeof(double), w.size(), f) == w.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) qtt::fail(QTT_E_ARG, std::string("precond_save: write failed: ") + path);
  });
}

int qtt_precond_load(qtt_ctx *ctx, const char *path) {
  return guard(ctx, [&] {
    qtt::Ctx &c = ctx->c;
    qtt::pc_init(c);
    if (!path) qtt::fail(QTT_E_ARG, "precond_load: null path");
    std::FILE *f = std::fopen(path, "rb");
    if (!f) qtt::fail(QTT_E_ARG, std::string("precond_load: cannot open ") + path);
    char tag[8];
    int64_t hdr[4];
    std::vector<double> w(c.pc.nparam);
    const bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, PC_TAG, 8) == 0 &&
                    std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == (int64_t)w.size() &&
                    hdr[1] == QTT_PC_IN && hdr[2] == QTT_PC_WIDTH && hdr[3] == QTT_PC_OUT &&
                    std::fread(w.data(), sizeof(double), w.size(), f) == w.size() &&
                    std::fgetc(f) == EOF;
    std::fclose(f);
    if (!ok) qtt::fail(QTT_E_ARG, std::string("precond_load: not a weights file of this network: ") + path);
    c.sync();
    HIPC(hipMemcpy(c.pc.w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
  });
}

int qtt_precond_grad(qtt_ctx *ctx, const double *X, int64_t npos, const double *dY, double *Y,
                     double *grad) {
  return guard(ctx, [&] {
    qtt::Ctx &c = ctx->c;
    qtt::pc_init(c);
    if (!X || !dY || !Y || !grad || npos < 1 || npos > (int64_t)1 << 24)
      qtt::fail(QTT_E_ARG, "precond_grad: bad arguments");
    c.register_user(X, (size_t)npos * qtt::PC_IN * 8);
    c.register_user(dY, (size_t)npos * qtt::PC_OUT * 8);
    c.register_user(Y, (size_t)npos * qtt::PC_OUT * 8);
    c.register_user(grad, (size_t)c.pc.nparam * 8);
    qtt::pc_net_grad(c, X, npos, dY, Y, grad);
    c.sync();
  });
}

}  // extern "C"
