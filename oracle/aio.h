/*
 * aio.h -- plain FP64 CPU oracle for the ensemble atom + trapped-ion integration.
 *
 * TEST INFRASTRUCTURE.  This library is the reference the HIP path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never calls it.  It shares no source
 * with the HIP library.
 *
 * What it computes (arXiv 2509.12381):
 *   - the equations of motion y' = f(t, y) of an ion in a Paul trap and an atom
 *     interacting through V(r) = -Cn/r^n + Cm/r^m (Sec. 2.1, equation for f and
 *     the Hamiltonian);
 *   - the ode45 algorithm of Fig. 2 (Dormand-Prince 5(4) pair with ode45's
 *     initial step, error norm and step-size control), run per trajectory to its
 *     exit (Sec. 3.2: final conditions plus scalar observables, 10^6-step cap);
 *   - the observables of Sec. 4.1: scattering angle, bounces, complex lifetime,
 *     position at the first bounce, momentum transfer, final distance, number of
 *     steps and final ion kinetic energy.
 *
 * Arrays of states are twelve planes: element (i, c) at ptr[c * ld + i].
 */
#ifndef AIO_ORACLE_H
#define AIO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define AIO_NSTATE 12
#define AIO_NOBS 13
#define AIO_MAXDIM 12

/* observable planes */
enum {
  AIO_OBS_TEND = 0, AIO_OBS_STATUS, AIO_OBS_NSTEPS, AIO_OBS_NFAILED, AIO_OBS_BOUNCES,
  AIO_OBS_LIFETIME, AIO_OBS_ANGLE, AIO_OBS_TRANSFER, AIO_OBS_POSITION, AIO_OBS_DIST,
  AIO_OBS_KE, AIO_OBS_RMIN, AIO_OBS_HNEXT
};

/* per-trajectory end status */
enum { AIO_RUNNING = 0, AIO_ESCAPED = 1, AIO_TMAX = 2, AIO_MAXSTEPS = 3, AIO_HMIN = 4,
       AIO_NONFINITE = 5 };

/* return codes */
enum { AIO_OK = 0, AIO_EINVAL = -1, AIO_WRTOL = 1 };

typedef struct {
  double m_ion, m_atom;        /* masses, electron masses */
  int n, m;                    /* exponents of V(r) = -Cn/r^n + Cm/r^m */
  double Cn, Cm;
  double a[3], q[3];           /* trap parameters per axis, paper form */
  double omega_rf;             /* trap radio frequency, inverse atomic time */
  double r_exit;               /* exit radius after closest approach; 0 = off */
  double r_bounce;             /* bounce radius */
  long long max_steps;         /* cap on accepted steps */
  double hmax;                 /* step-size cap; 0 = 0.1 |tf - t0| */
} aio_system;

/* Summary of one ode45 run. */
typedef struct {
  double t_end, h_next;
  long long nsteps, nfailed, nfevals;
  int status;
  int rtol_raised;
} aio_run;

int aio_version(void);

/* The Dormand-Prince tableau as held by the oracle: c[7], a[7*7] row-major,
   b[7], bhat[7] and the error weights e[7] = b - bhat. */
void aio_tableau(double *c, double *a, double *b, double *bhat, double *e);

/* f(t, y) of Sec. 2.1 and the Hamiltonian H(t, y). */
void aio_force(const aio_system *s, double t, const double *y, double *f);
double aio_energy(const aio_system *s, double t, const double *y);

/* Pieces of the ode45 algorithm, exported so tests can check each one. */
double aio_spacing(double t);
double aio_initial_step(int dim, const double *y0, const double *f0, double t0, double tf,
                        double rtol, double threshold, double hmax);
double aio_error_norm(int dim, double absh, const double *eps, const double *y,
                      const double *ynew, double threshold);
double aio_step_after_failure(double absh, double err, double rtol, int first_failure,
                              double hmin);
double aio_step_after_success(double absh, double err, double rtol);

/* Any right-hand side f(ctx, t, y, out) of dimension dim <= AIO_MAXDIM. */
typedef void (*aio_rhs_fn)(const void *ctx, double t, const double *y, double *f);
void aio_rhs_attempt(int dim, aio_rhs_fn rhs, const void *ctx, double t, double h,
                     const double *y, double *ynew, double *eps);
int aio_rhs_ode45(int dim, aio_rhs_fn rhs, const void *ctx, double t0, double tf,
                  const double *y0, double rtol, double atol, double hmax, long long max_steps,
                  double *y_out, aio_run *run, double *t_hist, double *h_hist,
                  long long hist_cap);

/* Linear test problem y' = A y (A dim x dim, row-major, dim <= AIO_MAXDIM). */
void aio_linear_attempt(int dim, const double *A, double t, double h, const double *y,
                        double *ynew, double *eps);
int aio_linear_ode45(int dim, const double *A, double t0, double tf, const double *y0,
                     double rtol, double atol, double hmax, long long max_steps,
                     double *y_out, aio_run *run, double *t_hist, double *h_hist,
                     long long hist_cap);

/* One atom-ion trajectory from t0 towards tf: final state and observables. */
int aio_integrate_one(const aio_system *s, double t0, double tf, const double *y0,
                      double rtol, double atol, double *y_final, double *obs);

/* An ensemble of n trajectories on nthreads host threads (<= 0: all cores). */
int aio_integrate(const aio_system *s, const double *y0, long long n, long long ld,
                  double t0, double tmax, double rtol, double atol, double *y_final,
                  double *obs, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
