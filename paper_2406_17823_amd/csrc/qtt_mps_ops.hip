// MPS algebra on the device: sums, TT-rounding, MPO and Hadamard products,
// inner products, dense reconstruction and input compression.
#include "qtt_internal.h"

#include <algorithm>
#include <functional>
#include <cmath>
#include <sstream>

namespace qtt {

namespace {

bool overlaps(const double *a, int64_t na, const double *b, int64_t nb) {
  return a < b + nb && b < a + na;
}

int struct_bound(int n, int k) {
  // min(4^k, 4^(n-k)) capped to avoid overflow
  const int e = std::min(k, n - k);
  return e >= 15 ? (1 << 30) : (1 << (2 * e));
}

}  // namespace

void mps_copy(Ctx &c, const Mps &src, Mps &dst) {
  const int64_t sz = src.size();
  if (dst.capacity < sz) {
    std::ostringstream s;
    s << "copy: capacity " << dst.capacity << " < " << sz;
    fail(QTT_E_CAPACITY, s.str());
  }
  dst.n = src.n;
  for (int k = 0; k <= src.n; ++k) dst.bond[k] = src.bond[k];
  if (dst.data != src.data)
    HIPC(hipMemcpyAsync(dst.data, src.data, sz * sizeof(double), hipMemcpyDeviceToDevice,
                        c.stream));
}

// ---------------------------------------------------------------- add
void mps_add(Ctx &c, int k, const double *coef, const Mps *x, Mps &y) {
  if (k < 1) fail(QTT_E_ARG, "add: k < 1");
  const int n = x[0].n;
  for (int j = 1; j < k; ++j)
    if (x[j].n != n) fail(QTT_E_SHAPE, "add: site counts differ");
  Mps out;
  out.n = n;
  out.data = y.data;
  out.capacity = y.capacity;
  out.bond[0] = out.bond[n] = 1;
  for (int s = 1; s < n; ++s) {
    int b = 0;
    for (int j = 0; j < k; ++j) b += x[j].bond[s];
    out.bond[s] = b;
  }
  const int64_t need = out.size();
  if (need > y.capacity) {
    std::ostringstream s;
    s << "add: output needs " << need << " doubles";
    fail(QTT_E_CAPACITY, s.str());
  }
  for (int j = 0; j < k; ++j)
    if (overlaps(y.data, need, x[j].data, x[j].size()))
      fail(QTT_E_ARG, "add: output overlaps an input");
  fill(c, out.data, need, 0.0);
  if (n == 1) {
    for (int j = 0; j < k; ++j) axpy_into(c, out.data, x[j].data, 4, coef[j]);
  } else {
    for (int s = 0; s < n; ++s) {
      int ol = 0, orr = 0;
      for (int j = 0; j < k; ++j) {
        const int l = x[j].bond[s], r = x[j].bond[s + 1];
        const double a = (s == 0) ? coef[j] : 1.0;
        place_block(c, out.core(s), out.bond[s], out.bond[s + 1], x[j].core(s), l, r,
                    (s == 0) ? 0 : ol, (s == n - 1) ? 0 : orr, a);
        ol += l;
        orr += r;
      }
    }
  }
  y = out;
}

// ---------------------------------------------------------------- products
void mps_apply_mpo(Ctx &c, const Mpo &W, const Mps &x, Mps &y) {
  const int n = x.n;
  if (W.n != n) fail(QTT_E_SHAPE, "apply_mpo: site counts differ");
  Mps out;
  out.n = n;
  out.data = y.data;
  out.capacity = y.capacity;
  for (int s = 0; s <= n; ++s) out.bond[s] = W.bond[s] * x.bond[s];
  const int64_t need = out.size();
  if (need > y.capacity) {
    std::ostringstream s;
    s << "apply_mpo: output needs " << need << " doubles";
    fail(QTT_E_CAPACITY, s.str());
  }
  if (overlaps(y.data, need, x.data, x.size())) fail(QTT_E_ARG, "apply_mpo: output overlaps input");
  for (int s = 0; s < n; ++s)
    mpo_core(c, out.core(s), W.fwd + W.off(s), W.bond[s], W.bond[s + 1], x.core(s), x.bond[s],
             x.bond[s + 1]);
  y = out;
}

void mps_hadamard(Ctx &c, const Mps &a, const Mps &b, Mps &y) {
  const int n = a.n;
  if (b.n != n) fail(QTT_E_SHAPE, "hadamard: site counts differ");
  Mps out;
  out.n = n;
  out.data = y.data;
  out.capacity = y.capacity;
  for (int s = 0; s <= n; ++s) out.bond[s] = a.bond[s] * b.bond[s];
  const int64_t need = out.size();
  if (need > y.capacity) {
    std::ostringstream s;
    s << "hadamard: output needs " << need << " doubles";
    fail(QTT_E_CAPACITY, s.str());
  }
  if (overlaps(y.data, need, a.data, a.size()) || overlaps(y.data, need, b.data, b.size()))
    fail(QTT_E_ARG, "hadamard: output overlaps an input");
  for (int s = 0; s < n; ++s)
    hadamard_core(c, out.core(s), a.core(s), a.bond[s], a.bond[s + 1], b.core(s), b.bond[s],
                  b.bond[s + 1]);
  y = out;
}

// ---------------------------------------------------------------- inner product
double mps_inner(Ctx &c, const Mps &x, const Mps &y) {
  const int n = x.n;
  if (y.n != n) fail(QTT_E_SHAPE, "inner: site counts differ");
  int maxE = 1, maxT = 1;
  for (int s = 0; s <= n; ++s) maxE = std::max(maxE, x.bond[s] * y.bond[s]);
  for (int s = 0; s < n; ++s) maxT = std::max(maxT, x.bond[s] * 4 * y.bond[s + 1]);
  double *E0 = c.buf("inner_E0", maxE);
  double *E1 = c.buf("inner_E1", maxE);
  double *T = c.buf("inner_T", maxT);
  fill(c, E0, 1, 1.0);
  for (int s = 0; s < n; ++s) {
    const int lx = x.bond[s], rx = x.bond[s + 1], ly = y.bond[s], ry = y.bond[s + 1];
    Gemm g;  // T[a][(w b')] = sum_b E[a][b] y[b][(w b')]
    g.M = lx;
    g.N = 4 * ry;
    g.K = ly;
    g.A = E0;
    g.sAm = ly;
    g.sAk = 1;
    g.B = y.core(s);
    g.sBk = 4 * ry;
    g.sBn = 1;
    g.C = T;
    g.sCm = 4 * ry;
    g.sCn = 1;
    gemm(c, g);
    Gemm h;  // E'[a'][b'] = sum_(a w) x[(a w)][a'] T[(a w)][b']
    h.M = rx;
    h.N = ry;
    h.K = 4 * lx;
    h.A = x.core(s);
    h.sAm = 1;
    h.sAk = rx;
    h.B = T;
    h.sBk = ry;
    h.sBn = 1;
    h.C = E1;
    h.sCm = ry;
    h.sCn = 1;
    gemm(c, h);
    std::swap(E0, E1);
  }
  double r = 0.0;
  HIPC(hipMemcpyAsync(&r, E0, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  c.sync();
  return r;
}

// ---------------------------------------------------------------- dense reconstruction
void mps_to_dense(Ctx &c, const Mps &x, double *grid) {
  const int n = x.n;
  if (n > 13) fail(QTT_E_UNSUPPORTED, "to_dense: n > 13");
  int64_t maxv = 4;
  int64_t rows = 1;
  for (int s = 0; s < n; ++s) {
    maxv = std::max<int64_t>(maxv, rows * 4 * x.bond[s + 1]);
    rows *= 4;
  }
  double *v0 = c.buf("dense_v0", maxv);
  double *v1 = c.buf("dense_v1", maxv);
  HIPC(hipMemcpyAsync(v0, x.core(0), x.core_size(0) * sizeof(double), hipMemcpyDeviceToDevice,
                      c.stream));
  rows = 4;
  for (int s = 1; s < n; ++s) {
    const int l = x.bond[s], r = x.bond[s + 1];
    Gemm g;  // v'[rows][(w r)] = v[rows][l] core[l][(w r)]
    g.M = (int)rows;
    g.N = 4 * r;
    g.K = l;
    g.A = v0;
    g.sAm = l;
    g.sAk = 1;
    g.B = x.core(s);
    g.sBk = 4 * r;
    g.sBn = 1;
    g.C = v1;
    g.sCm = 4 * r;
    g.sCn = 1;
    gemm(c, g);
    std::swap(v0, v1);
    rows *= 4;
  }
  morton_gather(c, grid, v0, n);
}

// ---------------------------------------------------------------- canonical forms
void mps_right_canonicalize(Ctx &c, std::vector<Mps *> xs) {
  const int n = xs[0]->n;
  for (Mps *x : xs) {
    if (x->n != n) fail(QTT_E_SHAPE, "canonicalize: site counts differ");
    for (int k = 0; k < n; ++k)
      if (x->bond[k] > 4 * x->bond[k + 1] || x->bond[k + 1] > 4 * x->bond[k])
        fail(QTT_E_SHAPE, "canonicalize: bond profile not reducible in place");
  }
  const int cnt = (int)xs.size();
  for (int d = n - 1; d >= 1; --d) {
    std::vector<ConstMatView> A(cnt);
    std::vector<MatView> Q(cnt), R(cnt);
    int64_t rsz = 0, tsz = 0;
    for (int i = 0; i < cnt; ++i) {
      const Mps &x = *xs[i];
      rsz += (int64_t)x.bond[d] * x.bond[d];
      tsz += x.core_size(d - 1);
    }
    double *Rb = c.buf("canon_R", rsz);
    double *Tb = c.buf("canon_T", tsz);
    int64_t ro = 0;
    for (int i = 0; i < cnt; ++i) {
      const Mps &x = *xs[i];
      const int l = x.bond[d], r = x.bond[d + 1];
      // M^T (4r x l) with M = core (l x 4r)
      A[i] = ConstMatView{x.core(d), 4 * r, l, 1, 4 * (int64_t)r};
      Q[i] = MatView{x.core(d), 4 * r, l, 1, 4 * (int64_t)r};
      R[i] = MatView{Rb + ro, l, l, l, 1};
      ro += (int64_t)l * l;
    }
    qr_batch(c, cnt, A.data(), Q.data(), R.data());
    ro = 0;
    int64_t to = 0;
    for (int i = 0; i < cnt; ++i) {
      const Mps &x = *xs[i];
      const int l = x.bond[d], lp = x.bond[d - 1];
      Gemm g;  // core_{d-1}[(a w)][l] <- core_{d-1} R^T
      g.M = 4 * lp;
      g.N = l;
      g.K = l;
      g.A = x.core(d - 1);
      g.sAm = l;
      g.sAk = 1;
      g.B = Rb + ro;
      g.sBk = 1;
      g.sBn = l;
      g.C = Tb + to;
      g.sCm = l;
      g.sCn = 1;
      gemm(c, g);
      HIPC(hipMemcpyAsync(x.core(d - 1), Tb + to, x.core_size(d - 1) * sizeof(double),
                          hipMemcpyDeviceToDevice, c.stream));
      ro += (int64_t)l * l;
      to += x.core_size(d - 1);
    }
  }
}

// ---------------------------------------------------------------- TT-rounding
void mps_truncate(Ctx &c, std::vector<Mps *> ys, int chi, double rtol, double *disc) {
  const int cnt = (int)ys.size();
  const int n = ys[0]->n;
  for (Mps *y : ys)
    if (y->n != n) fail(QTT_E_SHAPE, "truncate: site counts differ");
  if (chi < 1) fail(QTT_E_ARG, "truncate: chi < 1");
  for (int i = 0; i < cnt; ++i) disc[i] = 0.0;
  if (n == 1) return;

  // slot buffers: each core keeps its original slot (sizes only shrink)
  std::vector<int64_t> base(cnt);
  int64_t tot = 0;
  for (int i = 0; i < cnt; ++i) {
    base[i] = tot;
    tot += ys[i]->size();
  }
  double *WA = c.buf("trunc_A", tot);
  double *WB = c.buf("trunc_B", tot);
  double *WC = c.buf("trunc_C", tot);
  std::vector<std::vector<int64_t>> slot(cnt, std::vector<int64_t>(n));
  std::vector<std::vector<int>> bd(cnt, std::vector<int>(n + 1));
  int64_t rmax = 0;
  for (int i = 0; i < cnt; ++i) {
    for (int k = 0; k < n; ++k) slot[i][k] = base[i] + ys[i]->off(k);
    for (int k = 0; k <= n; ++k) bd[i][k] = ys[i]->bond[k];
    HIPC(hipMemcpyAsync(WA + base[i], ys[i]->data, ys[i]->size() * sizeof(double),
                        hipMemcpyDeviceToDevice, c.stream));
    for (int k = 0; k < n; ++k) rmax += (int64_t)bd[i][k + 1] * bd[i][k + 1];
  }
  double *Rb = c.buf("trunc_R", rmax);

  // left-to-right QR sweep
  for (int k = 0; k < n - 1; ++k) {
    std::vector<ConstMatView> A(cnt);
    std::vector<MatView> Q(cnt), R(cnt);
    std::vector<int> rp(cnt);
    int64_t ro = 0;
    for (int i = 0; i < cnt; ++i) {
      const int l = bd[i][k], r = bd[i][k + 1];
      rp[i] = std::min(4 * l, r);
      double *src = (k == 0) ? WA + slot[i][0] : WB + slot[i][k];
      A[i] = ConstMatView{src, 4 * l, r, r, 1};
      Q[i] = MatView{WB + slot[i][k], 4 * l, rp[i], rp[i], 1};
      R[i] = MatView{Rb + ro, rp[i], r, r, 1};
      ro += (int64_t)rp[i] * r;
    }
    qr_batch(c, cnt, A.data(), Q.data(), R.data());
    ro = 0;
    for (int i = 0; i < cnt; ++i) {
      const int r = bd[i][k + 1], r2 = bd[i][k + 2];
      Gemm g;  // WB[k+1] = R (rp x r) * WA[k+1] (r x 4 r2)
      g.M = rp[i];
      g.N = 4 * r2;
      g.K = r;
      g.A = Rb + ro;
      g.sAm = r;
      g.sAk = 1;
      g.B = WA + slot[i][k + 1];
      g.sBk = 4 * r2;
      g.sBn = 1;
      g.C = WB + slot[i][k + 1];
      g.sCm = 4 * r2;
      g.sCn = 1;
      gemm(c, g);
      ro += (int64_t)rp[i] * r;
      bd[i][k + 1] = rp[i];
    }
  }

  // right-to-left SVD sweep with truncation
  int maxn = 1;
  for (int i = 0; i < cnt; ++i)
    for (int k = 1; k < n; ++k) maxn = std::max(maxn, std::min(bd[i][k], 4 * bd[i][k + 1]));
  double *Sdev = c.buf("trunc_S", (int64_t)cnt * maxn);
  std::vector<double> Shost((size_t)cnt * maxn);
  for (int k = n - 1; k >= 1; --k) {
    std::vector<ConstMatView> A(cnt);
    std::vector<MatView> U(cnt), V(cnt);
    std::vector<double *> S(cnt);
    std::vector<int> m(cnt), nn(cnt);
    std::vector<bool> tall(cnt);
    int64_t usz = 0, vsz = 0;
    for (int i = 0; i < cnt; ++i) {
      const int l = bd[i][k], r = bd[i][k + 1];
      tall[i] = (l >= 4 * r);
      m[i] = tall[i] ? l : 4 * r;
      nn[i] = tall[i] ? 4 * r : l;
      usz += (int64_t)m[i] * nn[i];
      vsz += (int64_t)nn[i] * nn[i];
    }
    double *Ub = c.buf("trunc_U", usz);
    double *Vb = c.buf("trunc_V", vsz);
    double *Gb = c.buf("trunc_G", usz);
    int64_t uo = 0, vo = 0;
    for (int i = 0; i < cnt; ++i) {
      const int l = bd[i][k], r = bd[i][k + 1];
      const double *src = (k == n - 1) ? WB + slot[i][k] : WA + slot[i][k];
      if (tall[i])
        A[i] = ConstMatView{src, l, 4 * r, 4 * (int64_t)r, 1};
      else
        A[i] = ConstMatView{src, 4 * r, l, 1, 4 * (int64_t)r};
      // tall: only S and V are needed (G = M V[:, :keep] below); wide: only
      // U and S (G = M U[:, :keep])
      U[i] = MatView{tall[i] ? nullptr : Ub + uo, m[i], nn[i], nn[i], 1};
      V[i] = MatView{tall[i] ? Vb + vo : nullptr, nn[i], nn[i], nn[i], 1};
      S[i] = Sdev + (int64_t)i * maxn;
      uo += (int64_t)m[i] * nn[i];
      vo += (int64_t)nn[i] * nn[i];
    }
    svd_batch(c, cnt, A.data(), U.data(), S.data(), V.data());
    HIPC(hipMemcpyAsync(Shost.data(), Sdev, sizeof(double) * cnt * maxn, hipMemcpyDeviceToHost,
                        c.stream));
    c.sync();
    uo = 0;
    vo = 0;
    for (int i = 0; i < cnt; ++i) {
      const int l = bd[i][k], r = bd[i][k + 1], lp = bd[i][k - 1];
      const double *s = Shost.data() + (size_t)i * maxn;
      const int ns = nn[i];
      int keep = std::min(std::min(chi, struct_bound(n, k)), ns);
      if (rtol > 0.0 && s[0] > 0.0) {
        int cntk = 0;
        for (int j = 0; j < ns; ++j) cntk += (s[j] > rtol * s[0]) ? 1 : 0;
        keep = std::min(keep, cntk);
      }
      if (s[0] == 0.0) keep = 1;
      keep = std::max(keep, 1);
      for (int j = keep; j < ns; ++j) disc[i] += s[j] * s[j];
      // right factor rows -> new core k (keep x 4r); left factor * S -> G (l x keep)
      if (tall[i]) {
        // M = U S V^T: core rows = V^T[:keep] ; G = U[:, :keep] S = M V[:, :keep]
        permute3(c, WC + slot[i][k], Vb + vo, keep, 1, 4 * r, 1, 0, ns);
        Gemm gm;
        gm.M = l;
        gm.N = keep;
        gm.K = 4 * r;
        gm.A = A[i].p;
        gm.sAm = A[i].rs;
        gm.sAk = A[i].cs;
        gm.B = Vb + vo;
        gm.sBk = ns;
        gm.sBn = 1;
        gm.C = Gb + uo;
        gm.sCm = keep;
        gm.sCn = 1;
        gemm(c, gm);
      } else {
        // M^T = U' S V'^T: core rows = U'^T[:keep] ; G = V'[:, :keep] S = M U'[:, :keep]
        permute3(c, WC + slot[i][k], Ub + uo, keep, 1, 4 * r, 1, 0, ns);
        Gemm gm;
        gm.M = l;
        gm.N = keep;
        gm.K = 4 * r;
        gm.A = A[i].p;
        gm.sAm = 4 * (int64_t)r;
        gm.sAk = 1;
        gm.B = Ub + uo;
        gm.sBk = ns;
        gm.sBn = 1;
        gm.C = Gb + uo;
        gm.sCm = keep;
        gm.sCn = 1;
        gemm(c, gm);
      }
      Gemm g;  // WA[k-1] = WB[k-1] (4 lp x l) * G (l x keep)
      g.M = 4 * lp;
      g.N = keep;
      g.K = l;
      g.A = WB + slot[i][k - 1];
      g.sAm = l;
      g.sAk = 1;
      g.B = Gb + uo;
      g.sBk = keep;
      g.sBn = 1;
      g.C = WA + slot[i][k - 1];
      g.sCm = keep;
      g.sCn = 1;
      gemm(c, g);
      bd[i][k] = keep;
      uo += (int64_t)m[i] * nn[i];
      vo += (int64_t)nn[i] * nn[i];
    }
  }
  // pack: core 0 from WA, cores 1.. from WC
  for (int i = 0; i < cnt; ++i) {
    Mps &y = *ys[i];
    for (int k = 0; k <= n; ++k) y.bond[k] = bd[i][k];
    for (int k = 0; k < n; ++k) {
      const double *src = (k == 0) ? WA + slot[i][0] : WC + slot[i][k];
      HIPC(hipMemcpyAsync(y.core(k), src, y.core_size(k) * sizeof(double),
                          hipMemcpyDeviceToDevice, c.stream));
    }
  }
  c.sync();
}

// ---------------------------------------------------------------- input compression
constexpr double FROM_DENSE_FLOOR = 1e-7;

void mps_from_dense(Ctx &c, const double *grid, int n, int chi, double rtol, Mps &out,
                    std::vector<std::vector<double>> *spectra) {
  if (n < 1 || n > 13) fail(QTT_E_ARG, "from_dense: n out of range");
  const int64_t N2 = (int64_t)1 << (2 * n);
  double *M0 = c.buf("fd_M0", N2);
  double *M1 = c.buf("fd_M1", N2);
  morton_scatter(c, M0, grid, n);
  Mps res;
  res.n = n;
  res.data = out.data;
  res.capacity = out.capacity;
  res.bond[0] = 1;
  int l = 1;
  int64_t cols = N2 / 4;
  int64_t off = 0;
  std::vector<double> Sh(4096);
  for (int k = 0; k < n - 1; ++k) {
    const int m = 4 * l;
    double *G = c.buf("fd_G", (int64_t)m * m);
    double *U = c.buf("fd_U", (int64_t)m * m);
    double *V = c.buf("fd_V", (int64_t)m * m);
    double *S = c.buf("fd_S", m);
    Gemm g;  // G = M M^T, M is (m x cols) row-major
    g.M = m;
    g.N = m;
    g.K = (int)std::min<int64_t>(cols, 0x7fffffff);
    g.A = M0;
    g.sAm = cols;
    g.sAk = 1;
    g.B = M0;
    g.sBk = 1;
    g.sBn = cols;
    g.C = G;
    g.sCm = m;
    g.sCn = 1;
    gemm(c, g);
    ConstMatView A{G, m, m, m, 1};
    MatView Uv{U, m, m, m, 1}, Vv{V, m, m, m, 1};
    double *Sp = S;
    svd_batch(c, 1, &A, &Uv, &Sp, &Vv);
    if (m > (int)Sh.size()) Sh.resize(m);
    HIPC(hipMemcpyAsync(Sh.data(), S, sizeof(double) * m, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    if (spectra) {
      std::vector<double> s2(m);
      for (int j = 0; j < m; ++j) s2[j] = std::max(Sh[j], 0.0);
      spectra->push_back(std::move(s2));
    }
    // eigenvalues of G are sigma^2; the Gram route resolves sigma only down
    // to ~1e-8 sigma_max, so the cutoff is at least FROM_DENSE_FLOOR
    int keep = std::min(std::min(chi, struct_bound(n, k + 1)), m);
    const double cut = std::max(rtol, FROM_DENSE_FLOOR);
    if (Sh[0] > 0.0) {
      int cntk = 0;
      for (int j = 0; j < m; ++j) cntk += (std::sqrt(std::max(Sh[j], 0.0)) > cut * std::sqrt(Sh[0])) ? 1 : 0;
      keep = std::min(keep, cntk);
    } else keep = 1;
    keep = std::max(keep, 1);
    res.bond[k + 1] = keep;
    const int64_t csz = (int64_t)l * 4 * keep;
    if (off + csz > out.capacity) fail(QTT_E_CAPACITY, "from_dense: output capacity");
    // core k = V[:, :keep] as (l*4) x keep
    permute3(c, res.data + off, V, m, 1, keep, m, 0, 1);
    off += csz;
    Gemm h;  // M' (keep x cols) = V[:, :keep]^T M
    h.M = keep;
    h.N = (int)cols;
    h.K = m;
    h.A = V;
    h.sAm = 1;
    h.sAk = m;
    h.B = M0;
    h.sBk = cols;
    h.sBn = 1;
    h.C = M1;
    h.sCm = cols;
    h.sCn = 1;
    gemm(c, h);
    std::swap(M0, M1);
    l = keep;
    cols /= 4;
  }
  res.bond[n] = 1;
  const int64_t csz = (int64_t)l * 4;
  if (off + csz > out.capacity) fail(QTT_E_CAPACITY, "from_dense: output capacity");
  HIPC(hipMemcpyAsync(res.data + off, M0, csz * sizeof(double), hipMemcpyDeviceToDevice,
                      c.stream));
  c.sync();
  out = res;
}

// Bond dimension chi_l(eps) of every bipartition (the paper's MPS compression
// efficiency analysis, Eq. epsilon): the least number of Schmidt values of
// bipartition l whose discarded tail keeps that bipartition's relative L2
// error within eps, from the squared singular values the sequential
// decomposition meets at each cut (truncated to cap between cuts, values below
// 1e-7 sigma_max dropped, as the input compression does)
void schmidt_counts(Ctx &c, const double *grid, int n, double eps, int cap, int32_t *counts) {
  if (n < 2 || n > 13) fail(QTT_E_ARG, "schmidt_counts: n must be 2..13");
  if (cap < 1 || !(eps >= 0.0)) fail(QTT_E_ARG, "schmidt_counts: cap >= 1, eps >= 0");
  Mps out;
  out.n = n;
  out.bond[0] = out.bond[n] = 1;
  for (int k = 1; k < n; ++k) out.bond[k] = std::min<int64_t>(cap, struct_bound(n, k));
  out.capacity = out.size();
  out.data = c.buf("sc_out", out.capacity);
  std::vector<std::vector<double>> spectra;
  mps_from_dense(c, grid, n, cap, 0.0, out, &spectra);
  if ((int)spectra.size() != n - 1) fail(QTT_E_UNSUPPORTED, "schmidt_counts: spectra");
  for (int k = 0; k < n - 1; ++k) {
    std::vector<double> s2 = spectra[k];
    std::sort(s2.begin(), s2.end(), std::greater<double>());
    double total = 0.0;
    for (double v : s2) total += v;
    if (total == 0.0) {
      counts[k] = 0;
      continue;
    }
    // least c with sum_{j >= c} s2_j <= eps^2 total, at least 1
    double tail = 0.0;
    int cnt = (int)s2.size();
    for (int j = (int)s2.size() - 1; j >= 0; --j) {
      tail += s2[j];
      if (tail > eps * eps * total) break;
      cnt = j;
    }
    counts[k] = std::max(1, cnt);
  }
}

}  // namespace qtt
