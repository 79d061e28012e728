/*
 * aio.c -- plain FP64 CPU oracle (see aio.h).
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  Built with -O2 -fno-fast-math
 * -ffp-contract=off so every operation is one IEEE double rounding.
 *
 * Parity status of each part (how it is pinned without a reference code):
 *   tableau          order conditions in exact rationals, FSAL row, stability
 *                    polynomial (tests/test_oracle_tableau.py)
 *   attempt/stepper  y' = lambda y against exp, observed orders 5 and 4
 *   initial step     closed form on y' = lambda y
 *   error norm,      properties on linear problems (error estimate equals the
 *   controller       difference of the two embedded solutions, t_end == tf,
 *                    step count ~ rtol^(-1/5), fevals identity); the control
 *                    constants themselves are ode45's documented rule and are
 *                    parity unpinned against MATLAB (none available)
 *   force            harmonic closed form, straight-line atom, Mathieu equation
 *                    by brute force, conservation laws, head-on elastic
 *                    collision, deflection-function quadrature
 *   observables      constructed trajectories (head-on bounce, flyby); the
 *                    lifetime and the position at the first bounce against
 *                    closed forms: a bound pair oscillating radially with the
 *                    trap off (period by quadrature) and a head-on collision
 *                    with a displaced ion (tests/test_oracle_observables.py)
 */
#include "aio.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <string.h>
#include <unistd.h>

int aio_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Dormand-Prince 5(4) pair (the pair ode45 uses; Sec. 1 and Fig. 2 caption,
   citing Dormand and Prince 1980).  Stage 7 is evaluated at the propagated
   fifth-order solution, so its row of a equals b (first same as last).      */

static const double C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};

static const double A[7][7] = {
    {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0.0, 0.0, 0.0, 0.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0.0, 0.0, 0.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0.0, 0.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0},
};

static const double B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                            -2187.0 / 6784.0, 11.0 / 84.0, 0.0};

static const double BHAT[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                               -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

/* E = b - bhat, written as the exact rationals. */
static const double E[7] = {71.0 / 57600.0, 0.0, -71.0 / 16695.0, 71.0 / 1920.0,
                            -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};

void aio_tableau(double *c, double *a, double *b, double *bhat, double *e) {
  for (int i = 0; i < 7; ++i) {
    c[i] = C[i];
    b[i] = B[i];
    bhat[i] = BHAT[i];
    e[i] = E[i];
    for (int j = 0; j < 7; ++j) a[7 * i + j] = A[i][j];
  }
}

/* ------------------------------------------------------------------------ */
/* Equations of motion (Sec. 2.1): y = (x_ion, v_ion, x_atom, v_atom),
   dV/dr = n Cn / r^(n+1) - m Cm / r^(m+1), and the Paul-trap term
   -(a_k + 2 q_k cos(Omega t)) Omega^2/4 x_k on the ion.                     */

void aio_force(const aio_system *s, double t, const double *y, double *f) {
  double r = sqrt((y[0] - y[6]) * (y[0] - y[6]) + (y[1] - y[7]) * (y[1] - y[7]) +
                  (y[2] - y[8]) * (y[2] - y[8]));
  double dVdr = s->n * s->Cn / pow(r, s->n + 1) - s->m * s->Cm / pow(r, s->m + 1);
  double cosrf = cos(s->omega_rf * t);
  double w2 = s->omega_rf * s->omega_rf / 4.0;

  f[0] = y[3];
  f[1] = y[4];
  f[2] = y[5];
  f[3] = -(1.0 / s->m_ion) * dVdr * (y[0] - y[6]) / r - (s->a[0] + 2.0 * s->q[0] * cosrf) * w2 * y[0];
  f[4] = -(1.0 / s->m_ion) * dVdr * (y[1] - y[7]) / r - (s->a[1] + 2.0 * s->q[1] * cosrf) * w2 * y[1];
  f[5] = -(1.0 / s->m_ion) * dVdr * (y[2] - y[8]) / r - (s->a[2] + 2.0 * s->q[2] * cosrf) * w2 * y[2];
  f[6] = y[9];
  f[7] = y[10];
  f[8] = y[11];
  f[9] = -(1.0 / s->m_atom) * dVdr * (y[6] - y[0]) / r;
  f[10] = -(1.0 / s->m_atom) * dVdr * (y[7] - y[1]) / r;
  f[11] = -(1.0 / s->m_atom) * dVdr * (y[8] - y[2]) / r;
}

/* Hamiltonian of Sec. 2.1. */
double aio_energy(const aio_system *s, double t, const double *y) {
  double va2 = y[9] * y[9] + y[10] * y[10] + y[11] * y[11];
  double vi2 = y[3] * y[3] + y[4] * y[4] + y[5] * y[5];
  double r = sqrt((y[0] - y[6]) * (y[0] - y[6]) + (y[1] - y[7]) * (y[1] - y[7]) +
                  (y[2] - y[8]) * (y[2] - y[8]));
  double h = 0.5 * s->m_atom * va2 + 0.5 * s->m_ion * vi2 - s->Cn / pow(r, s->n) +
             s->Cm / pow(r, s->m);
  double cosrf = cos(s->omega_rf * t);
  for (int k = 0; k < 3; ++k)
    h += (s->a[k] + 2.0 * s->q[k] * cosrf) * s->m_ion * s->omega_rf * s->omega_rf / 8.0 *
         y[k] * y[k];
  return h;
}

/* ------------------------------------------------------------------------ */
/* The ode45 algorithm (Fig. 2, grey box).                                   */

/* Distance from |t| to the next larger double (MATLAB's eps(t)). */
double aio_spacing(double t) {
  double at = fabs(t);
  return nextafter(at, INFINITY) - at;
}

/* Initial step from f(t0, y0): the step for which the leading error term
   would be 0.8 rtol^(1/5) in the weighted infinity norm, capped by hmax and
   the span, and at least 16 eps(t0).                                        */
double aio_initial_step(int dim, const double *y0, const double *f0, double t0, double tf,
                        double rtol, double threshold, double hmax) {
  double absh = fmin(hmax, fabs(tf - t0));
  double rh = 0.0;
  for (int i = 0; i < dim; ++i) {
    double v = fabs(f0[i]) / fmax(fabs(y0[i]), threshold);
    if (v > rh) rh = v;
  }
  rh = rh / (0.8 * pow(rtol, 0.2));
  if (absh * rh > 1.0) absh = 1.0 / rh;
  return fmax(absh, 16.0 * aio_spacing(t0));
}

/* err = |h| * || eps ./ max(|y|, |ynew|, threshold) ||_inf */
double aio_error_norm(int dim, double absh, const double *eps, const double *y,
                      const double *ynew, double threshold) {
  double m = 0.0;
  for (int i = 0; i < dim; ++i) {
    double scale = fmax(fmax(fabs(y[i]), fabs(ynew[i])), threshold);
    double v = fabs(eps[i]) / scale;
    if (v > m || v != v) m = v;
  }
  return absh * m;
}

/* Step after a rejected attempt: the first failure of a step predicts the
   step with error 0.8^5 rtol (but shrinks at most 10x); later failures of the
   same step halve it.                                                       */
double aio_step_after_failure(double absh, double err, double rtol, int first_failure,
                              double hmin) {
  if (first_failure) return fmax(hmin, absh * fmax(0.1, 0.8 * pow(rtol / err, 0.2)));
  return fmax(hmin, 0.5 * absh);
}

/* Step after an accepted attempt that had no failure: grow by 0.8
   (rtol/err)^(1/5), at most 5x.                                            */
double aio_step_after_success(double absh, double err, double rtol) {
  double temp = 1.25 * pow(err / rtol, 0.2);
  if (temp > 0.2) return absh / temp;
  return 5.0 * absh;
}

typedef aio_rhs_fn rhs_fn;
/* Called at t0 (step == 0) and after every accepted step; a nonzero return
   is the trajectory's exit status. */
typedef int (*accept_fn)(void *ctx, double t, const double *y, long long step);

/* One Dormand-Prince attempt of size h from (t, y) with k[0] = f(t, y):
   fills k[1..6], the new solution ynew (stage 7's input) and
   eps = sum_j E_j k_j.  tnew is the time of stage 7.                      */
static void dp_attempt(int dim, rhs_fn rhs, const void *ctx, double t, double h, double tnew,
                       const double *y, double k[7][AIO_MAXDIM], double *ynew, double *eps) {
  double ys[AIO_MAXDIM];
  for (int s = 1; s < 7; ++s) {
    for (int i = 0; i < dim; ++i) {
      double acc = 0.0;
      for (int j = 0; j < s; ++j) acc += A[s][j] * k[j][i];
      ys[i] = y[i] + h * acc;
    }
    double ts = (s == 6) ? tnew : t + C[s] * h;
    rhs(ctx, ts, ys, k[s]);
    if (s == 6)
      for (int i = 0; i < dim; ++i) ynew[i] = ys[i];
  }
  for (int i = 0; i < dim; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 7; ++j) acc += E[j] * k[j][i];
    eps[i] = acc;
  }
}

static int all_finite(int dim, const double *v) {
  for (int i = 0; i < dim; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* ode45 from t0 to tf > t0.  y_out receives the last accepted state. */
static int ode45(int dim, rhs_fn rhs, const void *rhs_ctx, accept_fn on_accept, void *acc_ctx,
                 double t0, double tf, const double *y0, double rtol, double atol,
                 double hmax_in, long long max_steps, double *y_out, aio_run *run,
                 double *t_hist, double *h_hist, long long hist_cap) {
  double k[7][AIO_MAXDIM];
  double y[AIO_MAXDIM], ynew[AIO_MAXDIM], eps[AIO_MAXDIM];
  int rtol_raised = 0;

  memset(run, 0, sizeof *run);
  memset(y, 0, sizeof y);
  if (rtol < 100.0 * DBL_EPSILON) {
    rtol = 100.0 * DBL_EPSILON;
    rtol_raised = 1;
  }
  double threshold = atol / rtol;
  double hmax = hmax_in > 0.0 ? hmax_in : 0.1 * fabs(tf - t0);

  double t = t0;
  for (int i = 0; i < dim; ++i) y[i] = y0[i];
  rhs(rhs_ctx, t, y, k[0]);
  long long nsteps = 0, nfailed = 0, nfevals = 1;
  int status = AIO_RUNNING;
  double absh = 0.0;

  if (!all_finite(dim, y) || !all_finite(dim, k[0])) {
    status = AIO_NONFINITE;
  } else {
    absh = aio_initial_step(dim, y, k[0], t0, tf, rtol, threshold, hmax);
    if (on_accept) status = on_accept(acc_ctx, t, y, 0);
  }

  while (status == AIO_RUNNING) {
    double hmin = 16.0 * aio_spacing(t);
    absh = fmin(hmax, fmax(hmin, absh));
    double h = absh;
    int done = 0;
    if (1.1 * absh >= tf - t) {
      h = tf - t;
      absh = h;
      done = 1;
    }

    int nofailed = 1;
    double err, tnew;
    for (;;) {
      tnew = done ? tf : t + h;
      dp_attempt(dim, rhs, rhs_ctx, t, h, tnew, y, k, ynew, eps);
      nfevals += 6;
      err = aio_error_norm(dim, absh, eps, y, ynew, threshold);
      if (!isfinite(err)) {
        status = AIO_NONFINITE;
        break;
      }
      if (err > rtol) {
        nfailed += 1;
        if (absh <= hmin) {
          status = AIO_HMIN;
          break;
        }
        absh = aio_step_after_failure(absh, err, rtol, nofailed, hmin);
        nofailed = 0;
        h = absh;
        done = 0;
        continue;
      }
      break;
    }
    if (status != AIO_RUNNING) break;

    /* accepted */
    nsteps += 1;
    if (t_hist && nsteps <= hist_cap) {
      t_hist[nsteps - 1] = tnew;
      h_hist[nsteps - 1] = h;
    }
    t = tnew;
    for (int i = 0; i < dim; ++i) {
      y[i] = ynew[i];
      k[0][i] = k[6][i];
    }
    if (nofailed) absh = aio_step_after_success(absh, err, rtol);

    int st = on_accept ? on_accept(acc_ctx, t, y, nsteps) : AIO_RUNNING;
    if (st != AIO_RUNNING)
      status = st;
    else if (done)
      status = AIO_TMAX;
    else if (nsteps >= max_steps)
      status = AIO_MAXSTEPS;
  }

  for (int i = 0; i < dim; ++i) y_out[i] = y[i];
  run->t_end = t;
  run->h_next = absh;
  run->nsteps = nsteps;
  run->nfailed = nfailed;
  run->nfevals = nfevals;
  run->status = status;
  run->rtol_raised = rtol_raised;
  return rtol_raised ? AIO_WRTOL : AIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Linear test problem y' = A y.                                            */

typedef struct {
  int dim;
  const double *A;
} linear_ctx;

static void linear_rhs(const void *vctx, double t, const double *y, double *f) {
  const linear_ctx *c = (const linear_ctx *)vctx;
  (void)t;
  for (int i = 0; i < c->dim; ++i) {
    double acc = 0.0;
    for (int j = 0; j < c->dim; ++j) acc += c->A[c->dim * i + j] * y[j];
    f[i] = acc;
  }
}

void aio_linear_attempt(int dim, const double *Amat, double t, double h, const double *y,
                        double *ynew, double *eps) {
  linear_ctx ctx = {dim, Amat};
  double k[7][AIO_MAXDIM];
  linear_rhs(&ctx, t, y, k[0]);
  dp_attempt(dim, linear_rhs, &ctx, t, h, t + h, y, k, ynew, eps);
}

int aio_linear_ode45(int dim, const double *Amat, double t0, double tf, const double *y0,
                     double rtol, double atol, double hmax, long long max_steps,
                     double *y_out, aio_run *run, double *t_hist, double *h_hist,
                     long long hist_cap) {
  if (dim < 1 || dim > AIO_MAXDIM || !(tf > t0) || !(rtol > 0.0) || !(atol > 0.0))
    return AIO_EINVAL;
  linear_ctx ctx = {dim, Amat};
  return ode45(dim, linear_rhs, &ctx, NULL, NULL, t0, tf, y0, rtol, atol, hmax, max_steps,
               y_out, run, t_hist, h_hist, hist_cap);
}

/* ------------------------------------------------------------------------ */
/* Any right-hand side given as a function pointer (used by the tests).     */

void aio_rhs_attempt(int dim, aio_rhs_fn rhs, const void *ctx, double t, double h,
                     const double *y, double *ynew, double *eps) {
  double k[7][AIO_MAXDIM];
  rhs(ctx, t, y, k[0]);
  dp_attempt(dim, rhs, ctx, t, h, t + h, y, k, ynew, eps);
}

int aio_rhs_ode45(int dim, aio_rhs_fn rhs, const void *ctx, double t0, double tf,
                  const double *y0, double rtol, double atol, double hmax, long long max_steps,
                  double *y_out, aio_run *run, double *t_hist, double *h_hist,
                  long long hist_cap) {
  if (dim < 1 || dim > AIO_MAXDIM || !(tf > t0) || !(rtol > 0.0) || !(atol > 0.0))
    return AIO_EINVAL;
  return ode45(dim, rhs, ctx, NULL, NULL, t0, tf, y0, rtol, atol, hmax, max_steps, y_out, run,
               t_hist, h_hist, hist_cap);
}

/* ------------------------------------------------------------------------ */
/* Atom-ion trajectories with on-the-fly observables (Sec. 3.3 and 4.1).    */

static void atomion_rhs(const void *ctx, double t, const double *y, double *f) {
  aio_force((const aio_system *)ctx, t, y, f);
}

typedef struct {
  const aio_system *s;
  double va0[3];
  double w_prev;
  int approached;
  long long bounces;
  double t_first, t_last, position;
  double rmin2;
} observer;

/* Closest approach: the atom-ion distance stops decreasing, i.e. the sign of
   w = (x_ion - x_atom) . (v_ion - v_atom) goes from negative to non-negative
   between accepted steps (or w >= 0 at t0).  A closest approach inside
   r_bounce is a bounce.  Exit once r > r_exit after a closest approach.   */
static int observe(void *vctx, double t, const double *y, long long step) {
  observer *o = (observer *)vctx;
  const aio_system *s = o->s;
  double dx = y[0] - y[6], dy = y[1] - y[7], dz = y[2] - y[8];
  double r2 = dx * dx + dy * dy + dz * dz;
  double w = dx * (y[3] - y[9]) + dy * (y[4] - y[10]) + dz * (y[5] - y[11]);

  if (step == 0) {
    o->va0[0] = y[9];
    o->va0[1] = y[10];
    o->va0[2] = y[11];
    o->approached = (w >= 0.0);
    o->w_prev = w;
    o->bounces = 0;
    o->t_first = o->t_last = o->position = 0.0;
    o->rmin2 = r2;
    return AIO_RUNNING;
  }
  if (o->w_prev < 0.0 && w >= 0.0) {
    o->approached = 1;
    if (r2 < s->r_bounce * s->r_bounce) {
      o->bounces += 1;
      if (o->bounces == 1) {
        o->t_first = t;
        o->position = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
      }
      o->t_last = t;
    }
  }
  o->w_prev = w;
  if (r2 < o->rmin2) o->rmin2 = r2;
  if (o->approached && s->r_exit > 0.0 && r2 > s->r_exit * s->r_exit) return AIO_ESCAPED;
  return AIO_RUNNING;
}

int aio_integrate_one(const aio_system *s, double t0, double tf, const double *y0,
                      double rtol, double atol, double *y_final, double *obs) {
  observer o;
  memset(&o, 0, sizeof o);
  o.s = s;
  o.va0[0] = y0[9];
  o.va0[1] = y0[10];
  o.va0[2] = y0[11];
  o.rmin2 = (y0[0] - y0[6]) * (y0[0] - y0[6]) + (y0[1] - y0[7]) * (y0[1] - y0[7]) +
            (y0[2] - y0[8]) * (y0[2] - y0[8]);
  aio_run run;
  int rc = ode45(AIO_NSTATE, atomion_rhs, s, observe, &o, t0, tf, y0, rtol, atol, s->hmax,
                 s->max_steps, y_final, &run, NULL, NULL, 0);
  const double *y = y_final;
  double dx = y[0] - y[6], dy = y[1] - y[7], dz = y[2] - y[8];
  double va[3] = {y[9], y[10], y[11]};
  double cx = o.va0[1] * va[2] - o.va0[2] * va[1];
  double cy = o.va0[2] * va[0] - o.va0[0] * va[2];
  double cz = o.va0[0] * va[1] - o.va0[1] * va[0];
  double dot = o.va0[0] * va[0] + o.va0[1] * va[1] + o.va0[2] * va[2];
  double dvx = va[0] - o.va0[0], dvy = va[1] - o.va0[1], dvz = va[2] - o.va0[2];

  obs[AIO_OBS_TEND] = run.t_end;
  obs[AIO_OBS_STATUS] = (double)run.status;
  obs[AIO_OBS_NSTEPS] = (double)run.nsteps;
  obs[AIO_OBS_NFAILED] = (double)run.nfailed;
  obs[AIO_OBS_BOUNCES] = (double)o.bounces;
  obs[AIO_OBS_LIFETIME] = o.bounces >= 2 ? o.t_last - o.t_first : 0.0;
  obs[AIO_OBS_ANGLE] = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
  obs[AIO_OBS_TRANSFER] = s->m_atom * sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
  obs[AIO_OBS_POSITION] = o.position;
  obs[AIO_OBS_DIST] = sqrt(dx * dx + dy * dy + dz * dz);
  obs[AIO_OBS_KE] = 0.5 * s->m_ion * (y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
  obs[AIO_OBS_RMIN] = sqrt(o.rmin2);
  obs[AIO_OBS_HNEXT] = run.h_next;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Ensembles: one trajectory at a time per thread, indices handed out by an
   atomic counter.                                                          */

typedef struct {
  const aio_system *s;
  const double *y0;
  long long n, ld;
  double t0, tmax, rtol, atol;
  double *y_final, *obs;
  atomic_llong next;
  atomic_int warn;
} ensemble_job;

static void *ensemble_worker(void *arg) {
  ensemble_job *job = (ensemble_job *)arg;
  double y0[AIO_NSTATE], yf[AIO_NSTATE], ob[AIO_NOBS];
  for (;;) {
    long long i = atomic_fetch_add(&job->next, 1);
    if (i >= job->n) break;
    for (int c = 0; c < AIO_NSTATE; ++c) y0[c] = job->y0[c * job->ld + i];
    int rc = aio_integrate_one(job->s, job->t0, job->tmax, y0, job->rtol, job->atol, yf, ob);
    if (rc == AIO_WRTOL) atomic_store(&job->warn, 1);
    for (int c = 0; c < AIO_NSTATE; ++c) job->y_final[c * job->ld + i] = yf[c];
    for (int c = 0; c < AIO_NOBS; ++c) job->obs[c * job->ld + i] = ob[c];
  }
  return NULL;
}

static int finite_system(const aio_system *s) {
  double v[] = {s->m_ion, s->m_atom, s->Cn, s->Cm, s->a[0], s->a[1], s->a[2], s->q[0],
                s->q[1], s->q[2], s->omega_rf, s->r_exit, s->r_bounce, s->hmax};
  for (unsigned i = 0; i < sizeof v / sizeof v[0]; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

int aio_integrate(const aio_system *s, const double *y0, long long n, long long ld,
                  double t0, double tmax, double rtol, double atol, double *y_final,
                  double *obs, int nthreads) {
  if (!s || n < 0 || ld < n) return AIO_EINVAL;
  if (n > 0 && (!y0 || !y_final || !obs)) return AIO_EINVAL;
  if (!finite_system(s) || !(s->m_ion > 0.0) || !(s->m_atom > 0.0) || s->n < 1 ||
      s->n >= s->m || s->hmax < 0.0 || s->r_exit < 0.0 || s->r_bounce < 0.0 ||
      s->max_steps < 1)
    return AIO_EINVAL;
  if (!isfinite(t0) || !isfinite(tmax) || !(tmax > t0) || !isfinite(rtol) || !(rtol > 0.0) ||
      !isfinite(atol) || !(atol > 0.0))
    return AIO_EINVAL;
  if (n == 0) return rtol < 100.0 * DBL_EPSILON ? AIO_WRTOL : AIO_OK;

  ensemble_job job;
  job.s = s;
  job.y0 = y0;
  job.n = n;
  job.ld = ld;
  job.t0 = t0;
  job.tmax = tmax;
  job.rtol = rtol;
  job.atol = atol;
  job.y_final = y_final;
  job.obs = obs;
  atomic_init(&job.next, 0);
  atomic_init(&job.warn, 0);

  if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nthreads < 1) nthreads = 1;
  if ((long long)nthreads > n) nthreads = (int)n;
  pthread_t tid[512];
  if (nthreads > 512) nthreads = 512;
  int started = 0;
  for (int i = 1; i < nthreads; ++i) {
    if (pthread_create(&tid[started], NULL, ensemble_worker, &job) != 0) break;
    ++started;
  }
  ensemble_worker(&job);
  for (int i = 0; i < started; ++i) pthread_join(tid[i], NULL);
  return atomic_load(&job.warn) ? AIO_WRTOL : AIO_OK;
}
