// Device-resident state of one CG / PCG solve and its kernel launchers.
#pragma once

#include "qtt_internal.h"

namespace qtt {

struct CGState {
  double rr, rr_new, rz, pq, alpha, beta, bnorm2, tol2, rtol;
  int done, iters, maxit, converged, zero_x;
  int precond;  // PCG: rz is r . z, maintained by pcg_start / pcg_next
  unsigned int counter;
  // single-reduction CG (Chronopoulos-Gear; its step runs inside the
  // matvec, GemmCg): gamma = r . r, delta = w . r with w = A r of the
  // current residual, gamma_prev and alpha_prev of the previous iteration
  double gamma, delta, gamma_prev, alpha_prev;
  int first;
};

// rtol, maxit, precond set, done and the arrival counter cleared, on the
// device (no host copy: the host does not wait for the stream)
void cg_reset(Ctx &c, CGState *st, double rtol, int maxit, int precond);
// partial-sum buffer: 2 * 512 doubles
void cg_init(Ctx &c, const double *rhs, const double *q, double *r, double *p, double *x,
             int64_t n, CGState *st, double *part);
void cg_alpha(Ctx &c, const double *p, const double *q, int64_t n, CGState *st, double *part);
void cg_update(Ctx &c, double *x, double *r, const double *p, const double *q, int64_t n,
               CGState *st, double *part);
void cg_pupdate(Ctx &c, const double *r, double *p, int64_t n, CGState *st);
void pcg_start(Ctx &c, const double *r, const double *z, double *p, int64_t n, CGState *st,
               double *part);
void pcg_next(Ctx &c, const double *r, const double *z, double *p, int64_t n, CGState *st,
              double *part);

}  // namespace qtt
