// One-site variational sweep (App. B) and the RK4 step as four Euler
// minimisations (App. B, Table RK4, Eqs. U1-U4), orchestrated on the host,
// every contraction on the device.
//
// Tensor networks.  With v_i in mixed-canonical form around site d, the local
// system is  C_i + mu h^2 sum_j P_i^T D_i^T D_j P_j C_j = P_i^T a_i - h P_i^T B_i(b)
// (Eqs. first/second).  Each term is a network <v_i| W_1 .. W_p |ket>:
//   overlap      <v_i| a_i>                              (p = 0)
//   convection   <v_i| b_j (.) D_j |b_i>, <v_i| D_j b_j (.) |b_i>   (p = 2)
//   diffusion    <v_i| (D_1^2 + D_2^2) |b_i>             (p = 1)
//   penalty      <v_i| D_i^T D_j |v_j>                   (p = 1, the pair
//                composed into one MPO of bond 9; ket = trial)
// The environment of a network at bond b has layout
// [bra bond][layer bonds...][ket bond]; left environments (bonds <= d) and
// right environments (bonds > d) share one array per network because the two
// never hold the same bond at the same time.
//
// A "chain" contracts an environment with the ket core and then the layer
// cores of one site (ket first), leaving the bra index open:
//   T[bra][omega][layer bonds'][ket bond'].
// The local right-hand side is T contracted with the opposite environment;
// after the centre shift the new environment is the new bra core contracted
// with the same T, so each site costs one chain per network.  Moving right
// uses the cores as stored; moving left uses site-reversed copies
// ([r][w][l]), so one chain routine serves both directions.
#include "qtt_internal.h"
#include "qtt_cg.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <sstream>

namespace qtt {

namespace {

enum { LAYER_MPO = 0, LAYER_HAD = 1 };
// CG iterations are enqueued in a first chunk sized from the iteration count
// of the previous solve at the same site and direction, then in replayed
// graphs of GRAPH_CHUNK iterations until the device flag says done; the first
// chunk is one eager iteration and then replays of the same graph once its
// configuration has recurred (else eager launches); iterations enqueued past
// convergence return at once but still cost a launch each, so both chunks
// are kept short
constexpr int GRAPH_CHUNK = 4;

struct Layer {
  int kind = LAYER_MPO;
  const Mpo *mpo = nullptr;
  const Mps *had = nullptr;
  const double *had_rev = nullptr;
  int bond(int b) const { return kind == LAYER_MPO ? mpo->bond[b] : had->bond[b]; }
  const double *core(int d, bool rev) const {
    if (kind == LAYER_MPO) return (rev ? mpo->rperm : mpo->perm) + mpo->off(d);
    return (rev ? had_rev : had->data) + had->off(d);
  }
};

struct Net {
  int bra = 0;
  int nl = 0;
  Layer lay[2];
  bool trial_ket = false;
  int ket_comp = 0;
  const Mps *ket = nullptr;
  const double *ket_rev = nullptr;
  double coef = 1.0;
  int prec = QTT_PREC_F64;  // contraction precision of this network
  double *env = nullptr;
  std::vector<int64_t> eoff;
  double *T = nullptr;
  double *tmpn = nullptr;  // the other half of T's ping-pong pair (grouped chains)
  // float32-MFMA and split-bfloat16 networks keep their environments and
  // chain intermediates in float32 storage (half the bytes of the largest
  // tensors of the step); env and T then point at float arrays and eoff
  // counts float elements
  bool f32s() const { return prec == QTT_PREC_F32 || prec == QTT_PREC_BF16X3; }
  double *envp(int b) const {
    return f32s() ? reinterpret_cast<double *>(reinterpret_cast<float *>(env) + eoff[b])
                  : env + eoff[b];
  }
};

struct Sweep {
  Ctx &c;
  const qtt_params &p;
  int n;
  Mps *v;                 // the two trial MPS
  double *vrev[2];        // site-reversed copies of v
  std::vector<Net> rhs;   // right-hand-side networks
  std::vector<Net> pen;   // penalty networks, index 2*i + j
  double mu_h2;
  bool fit = false;       // fit of B(b): the local solution is the right-hand side
  CGState *st = nullptr;
  CGState *st_host = nullptr;
  double *part = nullptr;
  qtt_stats *stats = nullptr;
  int warn = 0;

  Sweep(Ctx &cc, const qtt_params &pp) : c(cc), p(pp) {}

  const Mps &ketmps(const Net &N) const { return N.trial_ket ? v[N.ket_comp] : *N.ket; }

  int64_t env_size(const Net &N, int b) const {
    int64_t s = (int64_t)v[N.bra].bond[b] * ketmps(N).bond[b];
    for (int l = 0; l < N.nl; ++l) s *= N.lay[l].bond(b);
    return s;
  }

  // largest intermediate of a chain through site d in either direction
  int64_t chain_max(const Net &N, int d) const {
    int64_t mx = 0;
    for (int dir = 0; dir < 2; ++dir) {
      const int bi = dir ? d + 1 : d, bo = dir ? d : d + 1;
      const int64_t a = v[N.bra].bond[bi];
      const int64_t g = ketmps(N).bond[bo];
      int64_t s = a * 4 * g;
      for (int l = 0; l < N.nl; ++l) s *= N.lay[l].bond(bi);
      mx = std::max(mx, s);
      for (int l = N.nl - 1; l >= 0; --l) {
        int64_t pre = a, post = g;
        for (int i = 0; i < l; ++i) pre *= N.lay[i].bond(bi);
        for (int i = l + 1; i < N.nl; ++i) post *= N.lay[i].bond(bo);
        mx = std::max(mx, pre * 4 * N.lay[l].bond(bo) * post);
      }
    }
    return mx;
  }

  // one step of a network chain: a GEMM or an MPO layer
  struct ChainStep {
    bool mpo = false;
    Gemm g;
    MpoJob j{};
  };

  // the steps of the chain through site d from the environment at the input
  // bond (steps[0] contracts the ket core, then the layers from the inner
  // one out); the result lands in T, with tmp as the other half of the
  // ping-pong pair.  Returns the number of steps (1 + N.nl).
  int chain_plan(const Net &N, int d, bool rev, const double *E, const double *ketcore,
                 double *T, double *tmp_buf, const int *skip, ChainStep *steps) {
    const int bi = rev ? d + 1 : d, bo = rev ? d : d + 1;
    const int a = v[N.bra].bond[bi];
    const Mps &kx = ketmps(N);
    const int g = kx.bond[bi], gp = kx.bond[bo];
    const int pl = N.nl;
    int mi[2] = {1, 1}, mo[2] = {1, 1};
    int64_t Pin = 1;
    for (int l = 0; l < pl; ++l) {
      mi[l] = N.lay[l].bond(bi);
      mo[l] = N.lay[l].bond(bo);
      Pin *= mi[l];
    }
    double *bufs[2] = {T, tmp_buf};
    int cur = (pl % 2 == 0) ? 0 : 1;
    int ns = 0;
    {
      ChainStep &st0 = steps[ns++];
      Gemm &q = st0.g;
      q.M = (int)(a * Pin);
      q.N = 4 * gp;
      q.K = g;
      q.A = E;
      q.sAm = g;
      q.sAk = 1;
      q.B = ketcore;
      q.sBk = 4 * gp;
      q.sBn = 1;
      q.C = bufs[cur];
      q.sCm = 4 * gp;
      q.sCn = 1;
      q.skip = skip;
      q.a32 = q.c32 = N.f32s();
    }
    for (int l = pl - 1; l >= 0; --l) {
      int64_t pre = a, post = gp;
      for (int i = 0; i < l; ++i) pre *= mi[i];
      for (int i = l + 1; i < pl; ++i) post *= mo[i];
      const double *src = bufs[cur];
      double *dst = bufs[1 - cur];
      ChainStep &st = steps[ns++];
      if (N.lay[l].kind == LAYER_MPO) {
        st.mpo = true;
        st.j = MpoJob{src, dst, N.lay[l].mpo, d, rev, pre, post, mi[l], mo[l]};
      } else {
        Gemm &q = st.g;
        q.skip = skip;
        q.B1 = (int)pre;
        q.B2 = 4;
        q.M = mo[l];
        q.N = (int)post;
        q.K = mi[l];
        q.A = N.lay[l].core(d, rev);
        q.sAm = 1;
        q.sAk = 4 * mo[l];
        q.sAb1 = 0;
        q.sAb2 = mo[l];
        q.B = src;
        q.sBk = 4 * post;
        q.sBn = 1;
        q.sBb1 = 4 * mi[l] * post;
        q.sBb2 = post;
        q.C = dst;
        q.sCm = post;
        q.sCn = 1;
        q.sCb1 = 4 * mo[l] * post;
        q.sCb2 = mo[l] * post;
        q.b32 = q.c32 = N.f32s();
      }
      cur = 1 - cur;
    }
    return ns;
  }

  // out_i += alpha * (T contracted with the opposite environment)
  Gemm open_gemm(const Net &N, int d, bool rev, const double *T, double *out, double alpha) {
    const int al = v[N.bra].bond[d], ar = v[N.bra].bond[d + 1];
    const int bo = rev ? d : d + 1;
    const int64_t rest = env_size(N, bo) / v[N.bra].bond[bo];
    Gemm q;
    q.alpha = alpha;
    q.beta = 1.0;
    q.a32 = q.b32 = N.f32s();  // T and the environment; out is float64
    if (!rev) {
      const double *R = N.envp(d + 1);
      q.M = 4 * al;
      q.N = ar;
      q.K = (int)rest;
      q.A = T;
      q.sAm = rest;
      q.sAk = 1;
      q.B = R;
      q.sBk = 1;
      q.sBn = rest;
      q.C = out;
      q.sCm = ar;
      q.sCn = 1;
    } else {
      const double *L = N.envp(d);
      q.B2 = 4;
      q.M = ar;
      q.N = al;
      q.K = (int)rest;
      q.A = T;
      q.sAm = 4 * rest;
      q.sAk = 1;
      q.sAb2 = rest;
      q.B = L;
      q.sBk = 1;
      q.sBn = rest;
      q.C = out;
      q.sCm = 1;
      q.sCn = 4 * ar;
      q.sCb2 = ar;
    }
    return q;
  }

  // environment at the output bond from T and the (new) bra core of site d
  Gemm env_gemm(const Net &N, int d, bool rev, const double *T) {
    const int al = v[N.bra].bond[d], ar = v[N.bra].bond[d + 1];
    const int bo = rev ? d : d + 1;
    const int64_t rest = env_size(N, bo) / v[N.bra].bond[bo];
    Gemm q;
    if (!rev) {
      q.M = ar;
      q.N = (int)rest;
      q.K = 4 * al;
      q.A = v[N.bra].core(d);
      q.sAm = 1;
      q.sAk = ar;
    } else {
      q.M = al;
      q.N = (int)rest;
      q.K = 4 * ar;
      q.A = vrev[N.bra] + v[N.bra].off(d);
      q.sAm = 1;
      q.sAk = al;
    }
    q.B = T;
    q.sBk = rest;
    q.sBn = 1;
    q.C = N.envp(bo);
    q.sCm = rest;
    q.sCn = 1;
    q.b32 = q.c32 = N.f32s();
    return q;
  }

  // ---- grouped network contractions: the networks of one group share a
  // contraction precision (float64, float32 or split bfloat16 MFMA) and each
  // step of their chains, their environment updates and their right-hand-
  // side terms go out as one grouped launch for the whole group (the GEMMs of
  // a step can have different shapes; MPO layers of a step share one launch)

  void launch_gemms(int cnt, Gemm *q, int prec, bool sum_outputs) {
    int grp[GEMM_GROUP];
    const double *C[GEMM_GROUP];
    const double *X[GEMM_GROUP] = {nullptr, nullptr, nullptr, nullptr};
    int ng = 0;
    for (int k = 0; k < cnt; ++k) {
      int gi = -1;
      if (sum_outputs)
        for (int u = 0; u < ng; ++u)
          if (C[u] == q[k].C) gi = u;
      if (gi < 0) {
        C[ng] = q[k].C;
        gi = ng++;
      }
      grp[k] = gi;
    }
    gemm_grouped(c, cnt, q, ng, grp, X, nullptr, prec);
  }

  // chains of the group's networks; E[k] is network k's input environment,
  // T[k] / tmp_k[k] its result and scratch
  void chain_group(int cnt, Net *const *Ns, int d, bool rev, const double *const *E,
                   double *const *T, double *const *tmp_k) {
    ChainStep steps[GEMM_GROUP][3];
    int ns[GEMM_GROUP], nmax = 0;
    for (int k = 0; k < cnt; ++k) {
      ns[k] = chain_plan(*Ns[k], d, rev, E[k], ket_core(*Ns[k], d, rev), T[k], tmp_k[k], nullptr,
                         steps[k]);
      nmax = std::max(nmax, ns[k]);
    }
    const bool f32 = Ns[0]->f32s();
    for (int t = 0; t < nmax; ++t) {
      Gemm q[GEMM_GROUP];
      MpoJob j[GEMM_GROUP];
      int nq = 0, nj = 0;
      for (int k = 0; k < cnt; ++k) {
        if (t >= ns[k]) continue;
        if (steps[k][t].mpo) j[nj++] = steps[k][t].j;
        else q[nq++] = steps[k][t].g;
      }
      if (nq) launch_gemms(nq, q, Ns[0]->prec, false);
      if (nj) mpo_layer_grouped(c, nj, j, nullptr, f32);
    }
  }

  void env_group(int cnt, Net *const *Ns, int d, bool rev, double *const *T) {
    Gemm q[GEMM_GROUP];
    for (int k = 0; k < cnt; ++k) q[k] = env_gemm(*Ns[k], d, rev, T[k]);
    launch_gemms(cnt, q, Ns[0]->prec, false);
  }

  // groups of up to GEMM_GROUP networks of one precision, in list order
  static std::vector<std::vector<Net *>> make_groups(const std::vector<Net *> &nets) {
    std::vector<std::vector<Net *>> out;
    std::vector<Net *> open[3];
    for (Net *N : nets) {
      auto &o = open[N->prec == QTT_PREC_F32 ? 1 : (N->prec == QTT_PREC_BF16X3 ? 2 : 0)];
      o.push_back(N);
      if ((int)o.size() == GEMM_GROUP) {
        out.push_back(o);
        o.clear();
      }
    }
    for (auto &o : open)
      if (!o.empty()) out.push_back(o);
    return out;
  }
  std::vector<std::vector<Net *>> rhs_groups, pen_groups;

  const double *ket_core(const Net &N, int d, bool rev) const {
    if (N.trial_ket) return rev ? vrev[N.ket_comp] + v[N.ket_comp].off(d) : v[N.ket_comp].core(d);
    return rev ? N.ket_rev + N.ket->off(d) : N.ket->core(d);
  }

  void reverse_core(const Mps &x, double *rev, int d) {
    const int l = x.bond[d], r = x.bond[d + 1];
    permute3(c, rev + x.off(d), x.core(d), r, 4, l, 1, r, 4 * (int64_t)r);
  }

  // environments and chain buffers live in context buffers that persist
  // across calls (no allocation once the largest shapes have been seen)
  void alloc(std::vector<Net *> all) {
    int idx = 0;
    for (Net *N : all) {
      N->eoff.assign(n + 2, 0);
      int64_t o = 0;
      // every environment starts on a 16-byte boundary (multiples of four
      // elements), so the GEMMs that read them can take 16-byte vector loads
      for (int b = 0; b <= n; ++b) {
        N->eoff[b] = o;
        o += (env_size(*N, b) + 3) & ~(int64_t)3;
      }
      // float32 storage: sizes in float elements, buffers in doubles
      const bool f = N->f32s();
      N->env = c.buf("sw_env" + std::to_string(idx), f ? (o + 1) / 2 : o);
      if (f) {
        fill_f32(c, reinterpret_cast<float *>(N->envp(0)), 1, 1.0f);
        fill_f32(c, reinterpret_cast<float *>(N->envp(n)), 1, 1.0f);
      } else {
        fill(c, N->envp(0), 1, 1.0);
        fill(c, N->envp(n), 1, 1.0);
      }
      int64_t own = 1;
      for (int d = 0; d < n; ++d) own = std::max(own, chain_max(*N, d));
      N->T = c.buf("sw_T" + std::to_string(idx), f ? (own + 1) / 2 : own);
      N->tmpn = c.buf("sw_Tb" + std::to_string(idx), f ? (own + 1) / 2 : own);
      ++idx;
    }
  }

  int64_t centre_size(int i, int d) const { return v[i].core_size(d); }

  // y = x + mu h^2 sum_j P_i^T D_i^T D_j P_j x_j: the four pair terms go out
  // as one grouped launch per step (ket contraction, MPO layer, contraction
  // with the right environment); the last also sums the two j terms of y_i
  // and adds x_i, so no copy kernel is needed.
  double *pT[4] = {nullptr, nullptr, nullptr, nullptr}, *pT2[4] = {nullptr, nullptr, nullptr, nullptr};

  void alloc_pen_tmp() {
    int64_t mx = 1;
    for (int d = 0; d < n; ++d)
      for (int k = 0; k < 4; ++k) {
        const Net &N = pen[k];
        const int i = k / 2, j = k % 2;
        const int64_t a = v[i].bond[d], gp = v[j].bond[d + 1];
        mx = std::max(mx, a * N.lay[0].bond(d) * 4 * gp);
        mx = std::max(mx, a * N.lay[0].bond(d + 1) * 4 * gp);
      }
    for (int k = 0; k < 4; ++k) {
      pT[k] = c.buf("sw_pT" + std::to_string(k), mx);
      pT2[k] = c.buf("sw_pT2_" + std::to_string(k), mx);
    }
  }

  // dot: the reduction of the last GEMM also forms delta = y . x into the CG
  // state (single-reduction CG)
  void matvec(int d, const double *x, double *y, const int *skip, bool dot = false,
              const GemmCg *cg = nullptr) {
    const int64_t s0 = centre_size(0, d);
    const double *xs[2] = {x, x + s0};
    double *ys[2] = {y, y + s0};
    Gemm kg[4], og[4];
    MpoJob mj[4];
    int kgrp[4] = {0, 1, 2, 3}, ogrp[4];
    const double *kX[4] = {nullptr, nullptr, nullptr, nullptr};
    const double *oX[2] = {xs[0], xs[1]};
    for (int k = 0; k < 4; ++k) {
      const int i = k / 2, j = k % 2;
      const Net &N = pen[k];
      const int a = v[i].bond[d], ar = v[i].bond[d + 1];
      const int g = v[j].bond[d], gp = v[j].bond[d + 1];
      const int mi = N.lay[0].bond(d), mo = N.lay[0].bond(d + 1);
      Gemm &q = kg[k];
      q.M = a * mi;
      q.N = 4 * gp;
      q.K = g;
      q.A = N.env + N.eoff[d];
      q.sAm = g;
      q.sAk = 1;
      q.B = xs[j];
      q.sBk = 4 * gp;
      q.sBn = 1;
      q.C = pT[k];
      q.sCm = 4 * gp;
      q.sCn = 1;
      if (cg) {
        // x is the CG residual r: the GEMM reads the next residual
        q.Bw = cg->w + (xs[j] - x);
        q.Bs = cg->s + (xs[j] - x);
        q.cgst = cg->st;
      }
      mj[k] = MpoJob{pT[k], pT2[k], N.lay[0].mpo, d, false, (int64_t)a, (int64_t)gp, mi, mo};
      const int64_t rest = (int64_t)mo * gp;
      Gemm &o = og[k];
      o.M = 4 * a;
      o.N = ar;
      o.K = (int)rest;
      o.A = pT2[k];
      o.sAm = rest;
      o.sAk = 1;
      o.B = N.env + N.eoff[d + 1];
      o.sBk = 1;
      o.sBn = rest;
      o.C = ys[i];
      o.sCm = ar;
      o.sCn = 1;
      o.alpha = mu_h2;
      o.beta = 1.0;
      ogrp[k] = i;
    }
    gemm_grouped(c, 4, kg, 4, kgrp, kX, skip, QTT_PREC_F64);
    mpo_layer_grouped(c, 4, mj, skip);
    if (dot) {
      GemmDot gd{};
      gd.Y[0] = xs[0];
      gd.Y[1] = xs[1];
      gd.out = &st->delta;
      gd.ctr = &st->counter;
      gd.part = dpart;
      gd.nparts = DPART;
      gemm_grouped(c, 4, og, 2, ogrp, oX, skip, QTT_PREC_F64, &gd);
    } else {
      gemm_grouped(c, 4, og, 2, ogrp, oX, skip, QTT_PREC_F64, nullptr, cg);
    }
  }
  static constexpr int DPART = 1024;
  double *dpart = nullptr;  // partials of the fused dot
  double *sv = nullptr;     // s = A p of the single-reduction CG

  void copy_skip(const double *x, double *y, int64_t n_, const int *skip);

  // cached graph of GRAPH_CHUNK CG iterations at site d; the key holds every
  // pointer and shape baked into the captured kernels
  CgGraph *graph_for(int d, bool rev, bool pre, const double *x, const double *r,
                     const double *pp, const double *q, const double *rhs) {
    std::vector<int64_t> key;
    auto add = [&](const void *ptr) { key.push_back((int64_t)(uintptr_t)ptr); };
    key.push_back(d);
    key.push_back(rev ? 1 : 0);
    int64_t mh;
    std::memcpy(&mh, &mu_h2, sizeof mh);
    key.push_back(mh);
    key.push_back(c.kt.on ? 1 : 0);
    key.push_back(pre ? 1 : 0);
    if (pre) {
      add(pcM);
      add(pcz);
      key.push_back(pc_np0);
    }
    for (int i = 0; i < 2; ++i) {
      key.push_back(v[i].bond[d]);
      key.push_back(v[i].bond[d + 1]);
    }
    add(x);
    add(r);
    add(pp);
    add(q);
    add(rhs);
    add(sv);
    add(dpart);
    add(st);
    add(part);
    add(c.kt.flop_ctr);
    for (const Net &N : pen) {
      add(N.env + N.eoff[d]);
      add(N.env + N.eoff[d + 1]);
      add(N.lay[0].mpo->csc[0].colptr);
      key.push_back(N.lay[0].bond(d));
      key.push_back(N.lay[0].bond(d + 1));
    }
    for (int k = 0; k < 4; ++k) {
      add(pT[k]);
      add(pT2[k]);
    }
    for (const char *nm : {"gemm_splitk64", "gemm_splitk32"}) {
      auto it = c.bufs.find(nm);
      add(it == c.bufs.end() ? nullptr : it->second.ptr);
    }
    const std::string k =
        std::to_string(d) + (rev ? "r" : "f") + (pre ? "p" : "c") + std::to_string(mh);
    CgGraph &g = c.cg_graphs[k];
    if (g.key == key) {
      g.hits += 1;
    } else {
      g.hits = 0;
      if (g.exec) HIPC(hipGraphExecDestroy(g.exec));
      g.exec = nullptr;
    }
    g.key = key;
    return &g;
  }

  // ---- preconditioner of the local system at site d (QTT_PC_*)
  double *pcM = nullptr, *pcz = nullptr;
  int64_t pc_np0 = 0;

  void apply_pc(const double *r, double *z, int d, const int *skip) {
    const int64_t s0 = centre_size(0, d);
    pc_apply(c, pcM, r, z, v[0].bond[d], v[0].bond[d + 1], skip);
    pc_apply(c, pcM + pc_np0 * 16, r + s0, z + s0, v[1].bond[d], v[1].bond[d + 1], skip);
  }

  // features of both components, then M from the block inverse (block
  // Jacobi) or from the network (learned; trained first when enabled)
  void pc_setup(int d) {
    const int64_t s0 = centre_size(0, d), ntot = s0 + centre_size(1, d);
    const int64_t np[2] = {(int64_t)v[0].bond[d] * v[0].bond[d + 1],
                           (int64_t)v[1].bond[d] * v[1].bond[d + 1]};
    const int64_t rows = np[0] + np[1];
    pc_np0 = np[0];
    double *X = c.buf("pc_X", rows * PC_IN), *B = c.buf("pc_B", rows * 16);
    pcM = c.buf("pc_M", rows * 16);
    pcz = c.buf("pc_z", ntot);
    for (int i = 0; i < 2; ++i) {
      const Net &N = pen[3 * i];  // pair (i, i)
      const int64_t r0 = i ? np[0] : 0;
      pc_features(c, N.env + N.eoff[d], N.env + N.eoff[d + 1], *N.lay[0].mpo, d, v[i].bond[d],
                  v[i].bond[d + 1], mu_h2, mu_h2 / (p.dx * p.dx), n, i, X + r0 * PC_IN,
                  B + r0 * 16);
    }
    if (p.precond == QTT_PC_BLOCK_JACOBI) {
      pc_block_inverse(c, B, pcM, rows);
      return;
    }
    PrecondNet &net = c.pc;
    if (net.train_per_solve > 0) {
      double *z = c.buf("pc_probe", ntot), *Az = c.buf("pc_Az", ntot);
      double *zz = c.buf("pc_zz", 1), *Mt = c.buf("pc_Mt", rows * 16);
      for (int t = 0; t < net.train_per_solve; ++t) {
        pc_probe(c, z, ntot, net.seed * 0x100000001B3ULL + net.probe_ctr);
        net.probe_ctr += 2 * (uint64_t)ntot;
        matvec(d, z, Az, nullptr);
        dot(c, z, z, ntot, zz);
        pc_forward(c, X, rows, Mt, true);
        fill(c, net.loss_dev, 1, 0.0);
        pc_loss_grad(c, Mt, 0, z, Az, v[0].bond[d], v[0].bond[d + 1], zz);
        pc_loss_grad(c, Mt, np[0], z + s0, Az + s0, v[1].bond[d], v[1].bond[d + 1], zz);
        pc_backward_adam(c, X, rows);
      }
      double *hl = c.pinned + 2048;
      HIPC(hipMemcpyAsync(hl, net.loss_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
      c.sync();
      if (net.first_loss < 0.0) net.first_loss = *hl;
      net.last_loss = *hl;
    }
    pc_forward(c, X, rows, pcM, false);
  }

  // CG / PCG iterations until the device flag says done, as replays of a
  // captured graph of GRAPH_CHUNK iterations, one graph per (site, direction,
  // mu h^2, preconditioning) and the buffers and shapes it was captured with
  void run_cg(int d, bool rev, bool pre, double *x, double *r, double *pp, double *q,
              const double *rhs, int64_t ntot) {
    auto enqueue_iters = [&](int k) {
      for (int i = 0; i < k; ++i) {
        if (pre) {
          matvec(d, pp, q, &st->done);
          cg_alpha(c, pp, q, ntot, st, part);
          cg_update(c, x, r, pp, q, ntot, st, part);
          apply_pc(r, pcz, d, &st->done);
          pcg_next(c, r, pcz, pp, ntot, st, part);
        } else {
          // single-reduction CG in one matvec per iteration (w = A r held in
          // q): its first GEMM reads the next residual, its reduction
          // updates the vectors and forms the two dot products
          GemmCg gc{};
          gc.st = st;
          gc.x = x;
          gc.r = r;
          gc.w = q;
          gc.p = pp;
          gc.s = sv;
          gc.n = ntot;
          gc.off[0] = 0;
          gc.off[1] = centre_size(0, d);
          gc.part = part;
          gc.nparts = 1024;
          matvec(d, r, q, &st->done, false, &gc);
        }
      }
    };
    const int hkey = (d * 2 + (rev ? 1 : 0)) * 2 + (pre ? 1 : 0);
    auto h = c.cg_hist.find(hkey);
    const int first_chunk = (h == c.cg_hist.end()) ? 8 : std::max(2, std::min(64, h->second + 1));
    auto capture = [&](CgGraph *g) {
      c.capturing = true;
      for (int k = 0; k < KT_KINDS; ++k) c.cap_launches[k] = 0;
      hipGraph_t graph = nullptr;
      HIPC(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
      try {
        enqueue_iters(GRAPH_CHUNK);
      } catch (...) {
        c.capturing = false;
        (void)hipStreamEndCapture(c.stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        throw;
      }
      c.capturing = false;
      HIPC(hipStreamEndCapture(c.stream, &graph));
      HIPC(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
      HIPC(hipGraphDestroy(graph));
      for (int k = 0; k < KT_KINDS; ++k) g->launches[k] = c.cap_launches[k];
    };
    auto replay = [&](CgGraph *g) {
      HIPC(hipGraphLaunch(g->exec, c.stream));
      if (stats) stats->graph_replays += 1;
      for (int k = 0; k < KT_KINDS; ++k) c.kt.launches[k] += c.kt.on ? g->launches[k] : 0;
    };
    // one eager iteration (it allocates what the iteration needs, so that
    // the graph key below sees the final buffers); the rest of the first
    // chunk as replays of the chunk graph when this configuration has been
    // seen before (iterations past convergence return at once), else eager
    enqueue_iters(1);
    {
      CgGraph *g = c.use_graphs ? graph_for(d, rev, pre, x, r, pp, q, rhs) : nullptr;
      if (g && (g->exec || g->hits >= 1)) {
        if (!g->exec) capture(g);
        for (int i = 0; i < (first_chunk - 1 + GRAPH_CHUNK - 1) / GRAPH_CHUNK; ++i) replay(g);
      } else {
        enqueue_iters(first_chunk - 1);
      }
    }
    HIPC(hipMemcpyAsync(st_host, st, sizeof(CGState), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    while (!st_host->done) {
      CgGraph *g = c.use_graphs ? graph_for(d, rev, pre, x, r, pp, q, rhs) : nullptr;
      if (g && !g->exec) capture(g);
      if (g) {
        replay(g);
      } else {
        enqueue_iters(GRAPH_CHUNK);
      }
      HIPC(hipMemcpyAsync(st_host, st, sizeof(CGState), hipMemcpyDeviceToHost, c.stream));
      c.sync();
    }
    c.cg_hist[hkey] = st_host->iters;
  }

  // r = rhs - A x on the device and the CG state reset (warm start from x)
  void cg_start(int d, bool pre, double *x, double *r, double *pp, double *q, const double *rhs,
                int64_t ntot) {
    cg_reset(c, st, p.cg_rtol, p.cg_maxit, pre ? 1 : 0);
    matvec(d, x, q, nullptr);
    cg_init(c, rhs, q, r, pp, x, ntot, st, part);
    if (pre) {
      apply_pc(r, pcz, d, &st->done);
      pcg_start(c, r, pcz, pp, ntot, st, part);
    } else {
      matvec(d, r, q, &st->done, true);  // w = A r, delta = w . r
    }
  }

  void local_solve(int d, bool rev) {
    const int64_t s0 = centre_size(0, d), s1 = centre_size(1, d), ntot = s0 + s1;
    double *rhs = c.buf("sw_rhs", ntot);
    double *x = c.buf("sw_x", ntot);
    double *r = c.buf("sw_r", ntot);
    double *pp = c.buf("sw_p", ntot);
    double *q = c.buf("sw_q", ntot);
    sv = c.buf("sw_s", ntot);
    dpart = c.buf("sw_dpart", DPART);
    fill(c, rhs, ntot, 0.0);
    double *rh[2] = {rhs, rhs + s0};
    auto t0 = std::chrono::steady_clock::now();
    for (auto &grp : rhs_groups) {
      const int cnt = (int)grp.size();
      const double *E[GEMM_GROUP];
      double *T[GEMM_GROUP], *tm[GEMM_GROUP];
      Gemm q[GEMM_GROUP];
      for (int k = 0; k < cnt; ++k) {
        E[k] = rev ? grp[k]->envp(d + 1) : grp[k]->envp(d);
        T[k] = grp[k]->T;
        tm[k] = grp[k]->tmpn;
      }
      chain_group(cnt, grp.data(), d, rev, E, T, tm);
      // the terms of one component are summed in the reduction of one launch
      for (int k = 0; k < cnt; ++k)
        q[k] = open_gemm(*grp[k], d, rev, grp[k]->T, rh[grp[k]->bra], grp[k]->coef);
      launch_gemms(cnt, q, grp[0]->prec, true);
    }
    if (fit) {
      // identity local matrix: the centres are the projected right-hand side
      double *const dst[2] = {v[0].core(d), v[1].core(d)};
      const double *const src[2] = {rhs, rhs + s0};
      const int64_t len[2] = {s0, s1};
      copy_pairs(c, 2, dst, src, len);
      if (stats && c.timing) {
        c.sync();
        stats->phase_ms[2] += ms_since(t0);
      }
      return;
    }
    auto load_guess = [&] {
      double *const dst[2] = {x, x + s0};
      const double *const src[2] = {v[0].core(d), v[1].core(d)};
      const int64_t len[2] = {s0, s1};
      copy_pairs(c, 2, dst, src, len);
    };
    load_guess();
    if (stats && c.timing) {
      c.sync();
      stats->phase_ms[2] += ms_since(t0);
    }
    t0 = std::chrono::steady_clock::now();
    // CG (Sec. II.C): device-resident scalars, host checks once per chunk
    const bool pre = p.precond != QTT_PC_NONE;
    if (pre) pc_setup(d);
    cg_start(d, pre, x, r, pp, q, rhs, ntot);
    run_cg(d, rev, pre, x, r, pp, q, rhs, ntot);
    int iters = st_host->iters;
    bool converged = st_host->converged;
    if (pre) {
      // float64 check: the true residual of the PCG result decides; plain CG
      // continues from it (from the guess after a non-finite result) when it
      // misses the tolerance
      if (!(st_host->rr_new == st_host->rr_new)) load_guess();
      cg_start(d, false, x, r, pp, q, rhs, ntot);
      HIPC(hipMemcpyAsync(st_host, st, sizeof(CGState), hipMemcpyDeviceToHost, c.stream));
      c.sync();
      if (!st_host->done) {
        run_cg(d, rev, false, x, r, pp, q, rhs, ntot);
        if (stats) stats->fallbacks += 1;
        warn = std::max(warn, (int)QTT_W_PRECOND_FALLBACK);
      }
      iters += st_host->iters;
      converged = st_host->converged;
    }
    if (stats) {
      stats->cg_iters_total += iters;
      stats->cg_iters_max = std::max(stats->cg_iters_max, iters);
      stats->cg_solves += 1;
      if (!converged) {
        stats->cg_maxit_hits += 1;
        warn = std::max(warn, (int)QTT_W_CG_MAXIT);
      }
      if (c.timing) stats->phase_ms[3] += ms_since(t0);
    } else if (!converged) {
      warn = std::max(warn, (int)QTT_W_CG_MAXIT);
    }
    {
      double *const dst[2] = {v[0].core(d), v[1].core(d)};
      const double *const src[2] = {x, x + s0};
      const int64_t len[2] = {s0, s1};
      copy_pairs(c, 2, dst, src, len);
    }
  }

  static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }

  std::vector<Net> &rhs_nets() { return rhs; }

  void shift(int d, bool right) {
    ConstMatView A[2];
    MatView Q[2], R[2];
    int64_t ro = 0, to = 0;
    int64_t rsz = 0, tsz = 0;
    for (int i = 0; i < 2; ++i) {
      const int l = v[i].bond[d], r = v[i].bond[d + 1];
      rsz += right ? (int64_t)r * r : (int64_t)l * l;
      tsz += right ? v[i].core_size(d + 1) : v[i].core_size(d - 1);
    }
    double *Rb = c.buf("sh_R", rsz);
    double *Tb = c.buf("sh_T", tsz);
    for (int i = 0; i < 2; ++i) {
      const int l = v[i].bond[d], r = v[i].bond[d + 1];
      if (right) {
        A[i] = ConstMatView{v[i].core(d), 4 * l, r, r, 1};
        Q[i] = MatView{v[i].core(d), 4 * l, r, r, 1};
        R[i] = MatView{Rb + ro, r, r, r, 1};
        ro += (int64_t)r * r;
      } else {
        A[i] = ConstMatView{v[i].core(d), 4 * r, l, 1, 4 * (int64_t)r};
        Q[i] = MatView{v[i].core(d), 4 * r, l, 1, 4 * (int64_t)r};
        R[i] = MatView{Rb + ro, l, l, l, 1};
        ro += (int64_t)l * l;
      }
    }
    qr_batch(c, 2, A, Q, R);
    // R (or L) into the neighbouring cores: both products in one launch
    ro = 0;
    Gemm g[2];
    double *dst[2];
    int64_t dsz[2], doff[2];
    for (int i = 0; i < 2; ++i) {
      const int l = v[i].bond[d], r = v[i].bond[d + 1];
      if (right) {
        const int r2 = v[i].bond[d + 2];
        g[i].M = r;
        g[i].N = 4 * r2;
        g[i].K = r;
        g[i].A = Rb + ro;
        g[i].sAm = r;
        g[i].sAk = 1;
        g[i].B = v[i].core(d + 1);
        g[i].sBk = 4 * r2;
        g[i].sBn = 1;
        g[i].C = Tb + to;
        g[i].sCm = 4 * r2;
        g[i].sCn = 1;
        dst[i] = v[i].core(d + 1);
        dsz[i] = v[i].core_size(d + 1);
        ro += (int64_t)r * r;
      } else {
        const int lp = v[i].bond[d - 1];
        g[i].M = 4 * lp;
        g[i].N = l;
        g[i].K = l;
        g[i].A = v[i].core(d - 1);
        g[i].sAm = l;
        g[i].sAk = 1;
        g[i].B = Rb + ro;
        g[i].sBk = 1;
        g[i].sBn = l;
        g[i].C = Tb + to;
        g[i].sCm = l;
        g[i].sCn = 1;
        dst[i] = v[i].core(d - 1);
        dsz[i] = v[i].core_size(d - 1);
        ro += (int64_t)l * l;
      }
      doff[i] = to;
      to += dsz[i];
    }
    {
      const int grp[2] = {0, 1};
      const double *X[2] = {nullptr, nullptr};
      gemm_grouped(c, 2, g, 2, grp, X, nullptr, QTT_PREC_F64);
    }
    {
      const double *const src[2] = {Tb + doff[0], Tb + doff[1]};
      copy_pairs(c, 2, dst, src, dsz);
    }
    if (!right)
      for (int i = 0; i < 2; ++i) reverse_core(v[i], vrev[i], d);
  }

  // environments at the new bond after a shift: the right-hand-side
  // networks reuse the chain results of the local step (their ket does not
  // change), the penalty networks contract the new trial cores
  void update_envs(int d, bool rev) {
    for (auto &grp : rhs_groups) {
      double *T[GEMM_GROUP];
      for (size_t k = 0; k < grp.size(); ++k) T[k] = grp[k]->T;
      env_group((int)grp.size(), grp.data(), d, rev, T);
    }
    for (auto &grp : pen_groups) envs_through(grp, d, rev);
  }

  // chain and environment update of every network of a group through site
  // d, from the environment at the input bond
  void envs_through(std::vector<Net *> &grp, int d, bool rev) {
    const int cnt = (int)grp.size();
    const double *E[GEMM_GROUP];
    double *T[GEMM_GROUP], *tm[GEMM_GROUP];
    for (int k = 0; k < cnt; ++k) {
      E[k] = rev ? grp[k]->envp(d + 1) : grp[k]->envp(d);
      T[k] = grp[k]->T;
      tm[k] = grp[k]->tmpn;
    }
    chain_group(cnt, grp.data(), d, rev, E, T, tm);
    env_group(cnt, grp.data(), d, rev, T);
  }

  double norm_sq_site0() {
    double *o = c.buf("sw_norm", 2);
    dot(c, v[0].core(0), v[0].core(0), v[0].core_size(0), o);
    dot(c, v[1].core(0), v[1].core(0), v[1].core_size(0), o + 1);
    double h[2];
    HIPC(hipMemcpyAsync(h, o, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    return h[0] + h[1];
  }
};

__global__ void k_copy_skip(const double *x, double *y, int64_t n, const int *skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

void Sweep::copy_skip(const double *x, double *y, int64_t n_, const int *skip) {
  c.check_range(x, 0, n_ - 1, 8, "copy_skip x");
  c.check_range(y, 0, n_ - 1, 8, "copy_skip y");
  unsigned g = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (n_ + 255) / 256));
  hipLaunchKernelGGL(k_copy_skip, dim3(g), dim3(256), 0, c.stream, x, y, n_, skip);
  HIPC(hipGetLastError());
}

void check_profile(const Mps &x, const char *what) {
  for (int k = 0; k < x.n; ++k)
    if (x.bond[k] > 4 * x.bond[k + 1] || x.bond[k + 1] > 4 * x.bond[k])
      fail(QTT_E_SHAPE, std::string(what) + ": bond profile must satisfy b[k] <= 4 b[k+1] and "
                                            "b[k+1] <= 4 b[k]");
}

}  // namespace

// one projection sweep.  Right-hand side: implicit (a and b: a_i - h B_i(b)
// through the 8 convection and 2 diffusion networks), explicit (a and w:
// a_i - h w_i through two layer-free networks), or fit (b only: B_i(b)
// alone and no penalty, so the local solution is the projected right-hand
// side, a least-squares fit of B(b) on the trial bonds)
static void project_impl(Ctx &c, const Mps *a, const Mps *b, const Mps *w, double h,
                         const qtt_params &p, Mps v[2], qtt_stats *st, int stage,
                         StageCache *cache, bool fit) {
  const int n = v[0].n;
  for (int i = 0; i < 2; ++i) {
    if ((a && a[i].n != n) || (b && b[i].n != n) || (w && w[i].n != n) || v[i].n != n)
      fail(QTT_E_SHAPE, "project: site counts differ");
    check_profile(v[i], "project: guess");
  }
  if (n < 2) fail(QTT_E_UNSUPPORTED, "project: n < 2");
  if (p.max_sweeps < 1 || p.cg_maxit < 1) fail(QTT_E_ARG, "project: max_sweeps/cg_maxit < 1");
  if (p.prec != QTT_PREC_F64 && p.prec != QTT_PREC_F32 && p.prec != QTT_PREC_BF16X3)
    fail(QTT_E_ARG, "project: prec");
  if (p.precond != QTT_PC_NONE && p.precond != QTT_PC_BLOCK_JACOBI &&
      p.precond != QTT_PC_LEARNED)
    fail(QTT_E_ARG, "project: precond");
  if (p.precond == QTT_PC_LEARNED) pc_init(c);

  auto t0 = std::chrono::steady_clock::now();
  Sweep S(c, p);
  S.n = n;
  S.v = v;
  S.stats = st;
  S.mu_h2 = p.mu * h * h;
  S.fit = fit;

  const bool reuse = cache && cache->valid;
  if (reuse) {
    // the canonical guess of the first stage (same a, same canonical form)
    for (int i = 0; i < 2; ++i) {
      for (int k = 0; k <= n; ++k) v[i].bond[k] = cache->bond[i][k];
      if (v[i].size() > v[i].capacity) fail(QTT_E_CAPACITY, "project: guess capacity");
      HIPC(hipMemcpyAsync(v[i].data, c.buf("rk4c_v" + std::to_string(i), v[i].size()),
                          v[i].size() * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
    }
  } else {
    mps_right_canonicalize(c, {&v[0], &v[1]});
  }

  // site-reversed copies of the fixed MPS and the trial MPS
  double *arev[2] = {nullptr, nullptr}, *brev[2] = {nullptr, nullptr};
  double *wrev[2] = {nullptr, nullptr};
  for (int i = 0; i < 2; ++i) {
    if (a) arev[i] = c.buf("sw_arev" + std::to_string(i), a[i].size());
    if (b) brev[i] = c.buf("sw_brev" + std::to_string(i), b[i].size());
    if (w) wrev[i] = c.buf("sw_wrev" + std::to_string(i), w[i].size());
    S.vrev[i] = c.buf("sw_vrev" + std::to_string(i), v[i].size());
    for (int d = 0; d < n; ++d) {
      if (a) S.reverse_core(a[i], arev[i], d);
      if (b) S.reverse_core(b[i], brev[i], d);
      if (w) S.reverse_core(w[i], wrev[i], d);
      S.reverse_core(v[i], S.vrev[i], d);
    }
  }
  auto D1 = get_mpo(c, n, "D1", p.dx, 0), D2 = get_mpo(c, n, "D2", p.dx, 0);
  auto LAP = get_mpo(c, n, "LAP", p.dx, p.lap_mode);
  const Mpo *D[2] = {D1.get(), D2.get()};
  const int conv_prec = p.prec;  // precision of the 8 convection networks

  // weight of B_i(b) in the right-hand side: -h, or 1 when fitting it
  const double g = fit ? 1.0 : -h;
  for (int i = 0; i < 2; ++i) {
    if (a) {
      Net ov;
      ov.bra = i;
      ov.nl = 0;
      ov.ket = &a[i];
      ov.ket_rev = arev[i];
      ov.coef = 1.0;
      S.rhs.push_back(ov);
    }
    if (w) {
      Net ow;
      ow.bra = i;
      ow.nl = 0;
      ow.ket = &w[i];
      ow.ket_rev = wrev[i];
      ow.coef = -h;
      S.rhs.push_back(ow);
      continue;
    }
    for (int j = 0; j < 2; ++j)
      for (int form = 0; form < 2; ++form) {
        // form 0: b_j (.) D_j b_i ; form 1: D_j (b_j (.) b_i) ; weight -h/2
        Net N;
        N.bra = i;
        N.nl = 2;
        Layer H;
        H.kind = LAYER_HAD;
        H.had = &b[j];
        H.had_rev = brev[j];
        Layer Dl;
        Dl.kind = LAYER_MPO;
        Dl.mpo = D[j];
        N.lay[0] = form == 0 ? H : Dl;
        N.lay[1] = form == 0 ? Dl : H;
        N.ket = &b[i];
        N.ket_rev = brev[i];
        N.coef = 0.5 * g;
        N.prec = conv_prec;
        S.rhs.push_back(N);
      }
    Net df;
    df.bra = i;
    df.nl = 1;
    df.lay[0].kind = LAYER_MPO;
    df.lay[0].mpo = LAP.get();
    df.ket = &b[i];
    df.ket_rev = brev[i];
    df.coef = -g / p.re;
    S.rhs.push_back(df);
  }
  std::shared_ptr<Mpo> PEN[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      PEN[i][j] = get_mpo(c, n, "P" + std::to_string(i + 1) + std::to_string(j + 1), p.dx, 0);
  for (int i = 0; i < 2 && !fit; ++i)
    for (int j = 0; j < 2; ++j) {
      // <v_i| D_i^T D_j |v_j> with the two MPOs composed into one of bond 9
      Net N;
      N.bra = i;
      N.nl = 1;
      N.lay[0].kind = LAYER_MPO;
      N.lay[0].mpo = PEN[i][j].get();
      N.trial_ket = true;
      N.ket_comp = j;
      N.coef = S.mu_h2;
      S.pen.push_back(N);
    }

  // device state: CG scalars, partial sums
  S.st = (CGState *)c.raw("sw_cgstate", sizeof(CGState));
  S.part = c.buf("sw_part", 2048);
  S.st_host = (CGState *)c.pinned;

  std::vector<Net *> all;
  for (Net &N : S.rhs) all.push_back(&N);
  for (Net &N : S.pen) all.push_back(&N);
  S.alloc(all);
  if (!fit) S.alloc_pen_tmp();
  {
    std::vector<Net *> r, q;
    for (Net &N : S.rhs) r.push_back(&N);
    for (Net &N : S.pen) q.push_back(&N);
    S.rhs_groups = Sweep::make_groups(r);
    S.pen_groups = Sweep::make_groups(q);
  }

  // right environments, sites n-1 .. 1; the overlap and penalty networks do
  // not involve b and are copied from the first stage when it is cached
  auto b_free = [](const Net &N) { return N.nl == 0 || N.trial_ket; };
  auto env_total = [&](const Net &N) { return N.eoff[n] + 1; };
  {
    std::vector<Net *> todo;
    for (Net *N : all)
      if (!(reuse && b_free(*N))) todo.push_back(N);
    auto groups = Sweep::make_groups(todo);
    for (int d = n - 1; d >= 1; --d)
      for (auto &grp : groups) S.envs_through(grp, d, true);
  }
  for (size_t idx = 0; idx < all.size(); ++idx) {
    if (!cache || !b_free(*all[idx])) continue;
    double *saved = c.buf("rk4c_env" + std::to_string(idx), env_total(*all[idx]));
    if (reuse)
      HIPC(hipMemcpyAsync(all[idx]->env, saved, env_total(*all[idx]) * sizeof(double),
                          hipMemcpyDeviceToDevice, c.stream));
    else
      HIPC(hipMemcpyAsync(saved, all[idx]->env, env_total(*all[idx]) * sizeof(double),
                          hipMemcpyDeviceToDevice, c.stream));
  }
  if (cache && !reuse) {
    for (int i = 0; i < 2; ++i) {
      for (int k = 0; k <= n; ++k) cache->bond[i][k] = v[i].bond[k];
      HIPC(hipMemcpyAsync(c.buf("rk4c_v" + std::to_string(i), v[i].size()), v[i].data,
                          v[i].size() * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
    }
    cache->valid = true;
  }
  if (st && c.timing) {
    c.sync();
    st->phase_ms[1] += Sweep::ms_since(t0);
  }

  double nrm_prev = S.norm_sq_site0();
  int sweeps = 0;
  bool converged = false;
  for (int s = 0; s < p.max_sweeps; ++s) {
    for (int d = 0; d < n - 1; ++d) {
      S.local_solve(d, false);
      auto t1 = std::chrono::steady_clock::now();
      S.shift(d, true);
      S.update_envs(d, false);
      if (st && c.timing) {
        c.sync();
        st->phase_ms[5] += Sweep::ms_since(t1);
      }
    }
    for (int d = n - 1; d >= 1; --d) {
      S.local_solve(d, true);
      auto t1 = std::chrono::steady_clock::now();
      S.shift(d, false);
      S.update_envs(d, true);
      if (st && c.timing) {
        c.sync();
        st->phase_ms[5] += Sweep::ms_since(t1);
      }
    }
    ++sweeps;
    const double nrm = S.norm_sq_site0();
    if (p.sweep_rtol > 0.0 && std::fabs(nrm - nrm_prev) <= p.sweep_rtol * nrm) {
      converged = true;
      break;
    }
    nrm_prev = nrm;
  }
  if (p.sweep_rtol > 0.0 && !converged) S.warn = std::max(S.warn, (int)QTT_W_SWEEP_MAXIT);
  if (st && stage >= 0 && stage < 4) st->sweeps[stage] += sweeps;
  c.sync();
  if (S.warn) throw Error{S.warn, "project: warning"};
}

void project(Ctx &c, const Mps a[2], const Mps b[2], double h, const qtt_params &p, Mps v[2],
             qtt_stats *st, int stage, StageCache *cache) {
  if (p.rhs_mode != 1) {
    project_impl(c, a, b, nullptr, h, p, v, st, stage, cache, false);
    return;
  }
  // explicit right-hand side: B(b) fitted on the bonds of b from the guess b
  // (fit_sweeps sweeps, else max_sweeps), then the minimisation with a - h w;
  // no stage cache
  // (the w network changes from stage to stage)
  Mps w[2];
  for (int i = 0; i < 2; ++i) {
    w[i] = b[i];
    w[i].data = c.buf("rkx_w" + std::to_string(i), b[i].size());
    w[i].capacity = b[i].size();
    mps_copy(c, b[i], w[i]);
  }
  qtt_params pf = p;
  if (p.fit_sweeps > 0) pf.max_sweeps = p.fit_sweeps;
  int warn = 0;
  try {
    project_impl(c, nullptr, b, nullptr, 0.0, pf, w, nullptr, stage, nullptr, true);
  } catch (Error &e) {
    if (e.code <= 0) throw;
    warn = e.code;
  }
  try {
    project_impl(c, a, nullptr, w, h, p, v, st, stage, nullptr, false);
  } catch (Error &e) {
    if (e.code <= 0) throw;
    warn = std::max(warn, e.code);
  }
  if (warn) throw Error{warn, "project: warning"};
}

// RK1 / RK2 schedules (App. B, Eqs. euler, midpoint_calc, full_calc): one
// minimisation with (a, b, h) = (u, u, dt), or the midpoint pair (u, u, dt/2)
// then (u, u_mid, dt); every minimisation starts from the guess u, so the
// second one reuses the first one's cached canonical guess and b-free
// environments.  The state keeps its bond profile (the trial MPS's).
static void rk_low_order(Ctx &c, Mps u[2], const qtt_params &p, int order, qtt_stats *st) {
  const int n = u[0].n;
  if (u[1].n != n) fail(QTT_E_SHAPE, "rk_step: site counts differ");
  for (int i = 0; i < 2; ++i) check_profile(u[i], "rk_step: state");
  Mps a[2], mid[2], v[2];
  for (int i = 0; i < 2; ++i) {
    const int64_t sz = u[i].size();
    a[i] = u[i];
    a[i].data = c.buf("rkl_a" + std::to_string(i), sz);
    a[i].capacity = sz;
    mps_copy(c, u[i], a[i]);
    mid[i] = u[i];
    mid[i].data = c.buf("rkl_m" + std::to_string(i), sz);
    mid[i].capacity = sz;
    v[i] = u[i];
    v[i].data = c.buf("rkl_v" + std::to_string(i), sz);
    v[i].capacity = sz;
  }
  int warn = 0;
  auto run = [&](auto &&f) {
    try {
      f();
    } catch (Error &e) {
      if (e.code > 0) warn = std::max(warn, e.code);
      else throw;
    }
  };
  StageCache cache;
  if (order == 1) {
    for (int i = 0; i < 2; ++i) mps_copy(c, a[i], v[i]);
    run([&] { project(c, a, a, p.dt, p, v, st, 0, &cache); });
  } else {
    for (int i = 0; i < 2; ++i) mps_copy(c, a[i], mid[i]);
    run([&] { project(c, a, a, 0.5 * p.dt, p, mid, st, 0, &cache); });
    for (int i = 0; i < 2; ++i) mps_copy(c, a[i], v[i]);
    run([&] { project(c, a, mid, p.dt, p, v, st, 1, &cache); });
  }
  for (int i = 0; i < 2; ++i) mps_copy(c, v[i], u[i]);
  c.sync();
  if (warn) throw Error{warn, "rk_step: warning"};
}

void rk_step(Ctx &c, Mps u[2], const qtt_params &p, int order, qtt_stats *st) {
  if (order == 4) rk4_step(c, u, p, st);
  else if (order == 1 || order == 2) rk_low_order(c, u, p, order, st);
  else fail(QTT_E_ARG, "rk_step: order must be 1, 2 or 4");
}

void rk4_step(Ctx &c, Mps u[2], const qtt_params &p, qtt_stats *st) {
  const int n = u[0].n;
  if (u[1].n != n) fail(QTT_E_SHAPE, "rk4: site counts differ");
  for (int i = 0; i < 2; ++i) {
    check_profile(u[i], "rk4: state");
    Mps cap;
    cap.n = n;
    cap.bond[0] = cap.bond[n] = 1;
    for (int k = 1; k < n; ++k)
      cap.bond[k] = std::min(p.chi, 1 << std::min(30, 2 * std::min(k, n - k)));
    if (u[i].capacity < cap.size()) {
      std::ostringstream s;
      s << "rk4: state capacity must hold " << cap.size() << " doubles";
      fail(QTT_E_CAPACITY, s.str());
    }
  }
  static const double hs[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  StageCache cache;
  static const double bc[3][2] = {{3.0, 0.25}, {1.5, 0.625}, {3.0, 0.25}};
  int warn = 0;
  Mps a[2], U[4][2], bb[2], sum[2];
  for (int i = 0; i < 2; ++i) {
    const int64_t sz = u[i].size();
    a[i] = u[i];
    a[i].data = c.buf("rk4_a" + std::to_string(i), sz);
    a[i].capacity = sz;
    scale_copy(c, a[i].data, u[i].data, sz, 1.0);
    scale_copy(c, a[i].data, u[i].data, u[i].core_size(0), 0.25);
    for (int k = 0; k < 4; ++k) {
      U[k][i] = u[i];
      U[k][i].data = c.buf("rk4_U" + std::to_string(k) + std::to_string(i), sz);
      U[k][i].capacity = sz;
    }
    // capacities of the 2-term and 4-term sums (bonds add)
    Mps two = u[i], four = u[i];
    for (int k = 1; k < n; ++k) {
      two.bond[k] = 2 * u[i].bond[k];
      four.bond[k] = 4 * u[i].bond[k];
    }
    bb[i].data = c.buf("rk4_b" + std::to_string(i), two.size());
    bb[i].capacity = two.size();
    sum[i].data = c.buf("rk4_sum" + std::to_string(i), four.size());
    sum[i].capacity = four.size();
  }
  auto run = [&](auto &&f) {
    try {
      f();
    } catch (Error &e) {
      if (e.code > 0) warn = std::max(warn, e.code);
      else throw;
    }
  };
  for (int k = 0; k < 4; ++k) {
    const Mps *b = u;
    if (k > 0) {
      auto t0 = std::chrono::steady_clock::now();
      for (int i = 0; i < 2; ++i) {
        const double coef[2] = {bc[k - 1][0], bc[k - 1][1]};
        Mps xs[2] = {U[k - 1][i], u[i]};
        mps_add(c, 2, coef, xs, bb[i]);
      }
      double disc[2];
      mps_truncate(c, {&bb[0], &bb[1]}, p.chi, p.svd_rtol, disc);
      if (st) {
        st->discarded_sq += disc[0] + disc[1];
        st->phase_ms[0] += std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - t0).count();
      }
      b = bb;
    }
    for (int i = 0; i < 2; ++i) mps_copy(c, a[i], U[k][i]);
    run([&] { project(c, a, b, hs[k] * p.dt, p, U[k], st, k, &cache); });
  }
  auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < 2; ++i) {
    const double coef[4] = {1.0, 1.0, 1.0, 1.0};
    Mps xs[4] = {U[0][i], U[1][i], U[2][i], U[3][i]};
    mps_add(c, 4, coef, xs, sum[i]);
  }
  double disc[2];
  mps_truncate(c, {&sum[0], &sum[1]}, p.chi, p.svd_rtol, disc);
  for (int i = 0; i < 2; ++i) mps_copy(c, sum[i], u[i]);
  c.sync();
  if (st) {
    st->discarded_sq += disc[0] + disc[1];
    st->phase_ms[0] +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (warn) throw Error{warn, "rk4: warning"};
}

}  // namespace qtt
