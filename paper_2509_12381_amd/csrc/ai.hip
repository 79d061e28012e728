// ai.hip -- HIP kernels and C ABI of libai.so (declared in include/ai.h).
//
// Built with -ffp-contract=off: every fused multiply-add is written out, so
// the per-lane sequence of roundings is fixed by this source and identical in
// every kernel that inlines it (plain, persistent, any schedule).
//
// Ensemble ode45 (Dormand-Prince 5(4)) integration of atom + trapped-ion
// trajectories, one trajectory per lane, FP64, for gfx950 (CDNA4, wave64).
//
// Mapping of the method onto the device:
//  * Each lane owns one trajectory.  Its state y, the first-same-as-last stage
//    k1 and the controller and observable scalars live in registers for the
//    whole integration; the only global traffic is the 12-plane load of y0 and
//    the 12 + 13-plane store of the results (structure-of-arrays planes, so a
//    wave's 64 lanes touch 64 consecutive doubles per plane).
//  * The control flow of ode45 (Fig. 2: attempt, error test, shrink and retry
//    or accept and grow) is flattened into one loop whose every iteration is
//    one attempt for every busy lane.  A lane that rejected retries in the next
//    iteration while its neighbours start their next step, so lanes of a wave
//    stay in step instead of waiting for the slowest lane's retries.
//  * Plain kernel: lane i of the grid integrates trajectory i.
//  * Persistent kernel: a grid that just fills the GPU; when lanes of a wave
//    have finished, the wave takes that many new trajectory indices from a
//    device counter with one atomic (ballot of the free lanes, popcount, lane
//    offsets by mbcnt) and the free lanes start them.  Per-trajectory
//    arithmetic is identical in both kernels, so results are bitwise equal.
//  * Nothing here is a dense contraction: the work is FP64 vector arithmetic
//    bound by the VALU, so no matrix cores are used.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ai.h"
#include "internal.h"
#include "schedule.h"

namespace {

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) pair (Dormand and Prince 1980; the pair ode45 uses,
// Sec. 1 and Fig. 2 caption).  Nodes c, weights b of the propagated
// fifth-order solution and error weights e = b - bhat.
constexpr double C2 = 1.0 / 5.0, C3 = 3.0 / 10.0, C4 = 4.0 / 5.0, C5 = 8.0 / 9.0;
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                 B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                 E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

// The force depends on positions and time only (Sec. 2.1), so the stage
// velocities of the 12-component system never need to be formed: with A the
// pair's stage matrix, the stage positions are
//   X_s = x + c_s h v + h^2 sum_l (A^2)_sl F_l,
// the new position x + h v + h^2 sum_l (bA)_l F_l (stage 7's position), the
// new velocity v + h sum_l b_l F_l, and the error vector's position part
// sum_j e_j V_j = h sum_l (eA)_l F_l (the e_j sum to zero).  These equal the
// 12-component stage formulas exactly in exact arithmetic; the entries
// below are the exact rationals of A^2, bA and eA.
constexpr double Q31 = 9.0 / 200.0;
constexpr double Q41 = -12.0 / 25.0, Q42 = 4.0 / 5.0;
constexpr double Q51 = -12248.0 / 6561.0, Q52 = 7208.0 / 2187.0, Q53 = -6784.0 / 6561.0;
constexpr double Q61 = -533.0 / 264.0, Q62 = 91.0 / 22.0, Q63 = -56.0 / 33.0, Q64 = 7.0 / 88.0;
constexpr double Q71 = 35.0 / 384.0, Q73 = 50.0 / 159.0, Q74 = 25.0 / 192.0,
                 Q75 = -243.0 / 6784.0;  // (bA)_2 = (bA)_6 = 0
constexpr double P1 = 611.0 / 230400.0, P3 = -514.0 / 83475.0, P4 = 391.0 / 38400.0,
                 P5 = -4617.0 / 1356800.0, P6 = -11.0 / 3360.0;  // (eA)_l, (eA)_2 = 0

constexpr int WAVE = 64;
constexpr int BLOCK = 64;  // one wave per workgroup: a finished wave frees its slot at once

// Leading positions of a scheduled plain launch integrated by four lanes each,
// by the AI_WIDE code of the kernel argument: 256 (16 waves) by default: past
// position 256 of the 2^20-trajectory thermal ensemble's order no trajectory
// needs more than 80% of the longest one's attempts, and 1024 lanes are a
// negligible share of the launch; none, 1024 or 4096 on request (the tuners
// try them).
__host__ __device__ constexpr long long wide_trajectories(int32_t kernel) {
  return ((kernel >> 16) & 3) == 1 ? 0 : ((kernel >> 16) & 3) == 2 ? 1024
         : ((kernel >> 16) & 3) == 3 ? 4096 : 256;
}

// Launch constants: the system constants folded into the forms the force and
// the controller use, computed once per call on the host, and the call's
// buffers.  The integration kernels take it as their only argument; the force
// constants are held in scalar registers, the loop's other constants in
// vector registers (Ctl below).
struct Launch {
  double mr;                 // m_atom / m_ion: F_ion = -mr F_atom - kappa(t) x_ion
  double nCa, mCa;           // n Cn / m_atom and m Cm / m_atom: F_atom = g_a d with, for n=4, m=8,
                             // g_a = ((dV/dr)/r) / m_atom = s^3 (nCa - mCa s^2), s = 1/r^2
  int pot_n, pot_m;          // the exponents n < m of V(r) = -Cn/r^n + Cm/r^m
  double ka[3], kq[3];       // kappa_k(t) = ka_k + kq_k cos(omega t) = (a_k + 2 q_k cos) omega^2/4
  double omega;
  double r_exit2, r_bounce2;
  double half_mi, m_atom;    // for the observables
  double t0, tf, hmax, rtol, inv_rtol, thr;
  double vbound;             // (RelTol/AbsTol)(1 + 2^-20): bound on a velocity ratio per |e|
  double hinit_den;          // 0.8 rtol^(1/5)
  long long n, ld;
  long long first_dynamic;   // persistent kernel: first index handed out by the queue
  long long wide;            // scheduled plain kernel: leading positions integrated by four
                             // lanes each (see integrate_wide)
  int wide_waves;            // the waves at the start of the grid that hold them
  int max_steps;
  int exit_on;               // r_exit > 0
  int refill_min;            // persistent kernel: idle lanes a wave gathers before drawing work
  double near2;              // single-precision stages: squared distance below which a wave
                             // integrates in double
  const double* y0;          // n x 12 initial states (planes of ld)
  double* yf;                // n x 12 final states (may alias y0)
  double* obs;               // n x AI_NOBS observables
  const unsigned* order;     // schedule: trajectory at each position (null: identity)
  const unsigned* key;       // schedule: predicted cost code at each position (null: none)
  unsigned long long* queue; // persistent kernel: dynamic positions handed out so far
};

// Per-lane integration state.  x and v hold (ion, atom) positions and
// velocities, F1 the accelerations at (t, x): the first stage of the next
// attempt (first same as last).  cph, sph track the trap phase omega t; each
// accepted step rotates them by omega (t_new - t) (the exact difference of the
// two doubles), so they follow the rounded time t as a direct evaluation
// would.  The step size h always equals absh here
// (integration runs forward), and the step floor 16 eps(t) is recomputed.
template <class R>
struct LaneT {
  double x[6], v[6];
  R F1[6];                   // in the stage precision R
  double t, absh;
  double cph, sph;           // cos and sin of omega t
  double w_prev, t_first, t_last, position, rmin2;
  long long nfailed;
  int nsteps, bounces, status;
  // flags as ints: a bool that lives across the loop is kept as a 64-bit lane
  // mask in scalar registers, an int in one vector register
  int done, nofailed, fresh, approached;
};
using Lane = LaneT<double>;
using Lane32 = LaneT<float>;

// The integration loop's constants other than the force constants, one copy
// per lane in vector registers.  A wave has about 100 scalar registers; the
// force constants, the tableau constants that FMAs take as scalar operands and
// these do not all fit, and spilled scalars are restored with a v_readlane
// (one VALU slot) at every use inside the loop.  The empty asm gives each
// value a vector-register definition, so it stays there.
struct Ctl {
  double tf, hmax, rtol, inv_rtol, thr, vbound, r_exit2, r_bounce2, omega;
  int max_steps, exit_on;
};

template <typename T>
__device__ __forceinline__ T in_vgpr(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The force constants for the loop.  The trap coefficients go to vector
// registers as well: fma(kq, cos, ka) with both in scalar registers needs a
// copy of one of them first (an instruction reads one scalar operand).
struct Force {
  double mr, nCa, mCa, ka[3], kq[3];
};

__device__ __forceinline__ Force lane_force(const Launch& P) {
  Force f;
  f.mr = P.mr;
  f.nCa = P.nCa;
  f.mCa = P.mCa;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f.ka[k] = in_vgpr(P.ka[k]);
    f.kq[k] = in_vgpr(P.kq[k]);
  }
  return f;
}

// The force constants of a potential with other exponents: g_a = (dV/dr)/r
// / m_atom = (n Cn r^-(n+2) - m Cm r^-(m+2)) / m_atom, powers of s = 1/r^2
// (times sqrt(s) = 1/r for an odd exponent).
struct ForceNM {
  double mr, nCa, mCa, ka[3], kq[3];
  int en, em;  // n + 2 and m + 2
};

__device__ __forceinline__ ForceNM lane_force_nm(const Launch& P) {
  ForceNM f;
  f.mr = P.mr;
  f.nCa = P.nCa;
  f.mCa = P.mCa;
  f.en = P.pot_n + 2;
  f.em = P.pot_m + 2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f.ka[k] = in_vgpr(P.ka[k]);
    f.kq[k] = in_vgpr(P.kq[k]);
  }
  return f;
}

__device__ __forceinline__ Force lane_force_of(const Launch& P, const Force*) { return lane_force(P); }
__device__ __forceinline__ ForceNM lane_force_of(const Launch& P, const ForceNM*) {
  return lane_force_nm(P);
}

// The force constants in single precision, for the single-precision-stage
// variant.
struct Force32 {
  float mr, nCa, mCa, ka[3], kq[3];
};

__device__ __forceinline__ Force32 lane_force32(const Launch& P) {
  Force32 f;
  f.mr = (float)P.mr;
  f.nCa = (float)P.nCa;
  f.mCa = (float)P.mCa;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f.ka[k] = in_vgpr((float)P.ka[k]);
    f.kq[k] = in_vgpr((float)P.kq[k]);
  }
  return f;
}

__device__ __forceinline__ Ctl lane_ctl(const Launch& P) {
  Ctl c;
  c.tf = in_vgpr(P.tf);
  c.hmax = in_vgpr(P.hmax);
  c.rtol = in_vgpr(P.rtol);
  c.inv_rtol = in_vgpr(P.inv_rtol);
  c.thr = in_vgpr(P.thr);
  c.vbound = in_vgpr(P.vbound);
  c.r_exit2 = in_vgpr(P.r_exit2);
  c.r_bounce2 = in_vgpr(P.r_bounce2);
  c.omega = in_vgpr(P.omega);
  c.max_steps = in_vgpr(P.max_steps);
  c.exit_on = in_vgpr(P.exit_on);
  return c;
}

// Distance from |t| to the next larger double (MATLAB's eps(t)); exact.
__device__ __forceinline__ double spacing(double t) {
  const double at = fabs(t);
  return __longlong_as_double(__double_as_longlong(at) + 1) - at;
}

// 1/a from the hardware estimate r (relative error e = 1 - a r below 2^-23,
// computed exactly enough by one FMA): 1/a = r / (1 - e) = r (1 + e + e^2)
// up to r e^3 (below 2^-69 relative), in three dependent FMAs.
__device__ __forceinline__ double recip(double a) {
  const double r = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// 1/a for the force: the hardware estimate r (|1 - a r| at most 2^-24.4 over
// 2^24 random doubles of exponents -60..60 on gfx950) and one Newton step,
// r (1 + e), which leaves a relative error of about e^2 <= 2^-48.7 (10 ulp):
// far below the solution's own tolerance, and one FMA shorter than recip().
__device__ __forceinline__ double recip_force(double a) {
  const double r = __builtin_amdgcn_rcp(a);
  return fma(r, fma(-a, r, 1.0), r);
}

// Taylor polynomials of cos and sin of a small angle u (|u| <= pi/4 on every
// call), truncated after u^16 and u^17 (remainders below 3e-18).
__device__ __forceinline__ double cos_poly(double u2) {
  double c = 1.0 / 20922789888000.0;                     // 1/16!
  c = fma(c, u2, -1.0 / 87178291200.0);                  // -1/14!
  c = fma(c, u2, 1.0 / 479001600.0);                     // 1/12!
  c = fma(c, u2, -1.0 / 3628800.0);                      // -1/10!
  c = fma(c, u2, 1.0 / 40320.0);                         // 1/8!
  c = fma(c, u2, -1.0 / 720.0);                          // -1/6!
  c = fma(c, u2, 1.0 / 24.0);                            // 1/4!
  c = fma(c, u2, -0.5);                                  // -1/2!
  return fma(c, u2, 1.0);
}
__device__ __forceinline__ double sin_poly(double u, double u2) {
  double s = 1.0 / 355687428096000.0;                    // 1/17!
  s = fma(s, u2, -1.0 / 1307674368000.0);                // -1/15!
  s = fma(s, u2, 1.0 / 6227020800.0);                    // 1/13!
  s = fma(s, u2, -1.0 / 39916800.0);                     // -1/11!
  s = fma(s, u2, 1.0 / 362880.0);                        // 1/9!
  s = fma(s, u2, -1.0 / 5040.0);                         // -1/7!
  s = fma(s, u2, 1.0 / 120.0);                           // 1/5!
  s = fma(s, u2, -1.0 / 6.0);                            // -1/3!
  return fma(s * u2, u, u);
}

// cos(x) and sin(x) for |x| < 2^31 pi/2 (checked on the host): Cody-Waite
// reduction x = n pi/2 + r with pi/2 split into two doubles (the first
// product is exact under the fused multiply-add, the split error is 1.5e-33
// per unit of n), then the polynomials above on |r| <= pi/4.
__device__ __forceinline__ void sincos_rf(double x, double& cx, double& sx) {
  constexpr double TWO_OVER_PI = 0.63661977236758134;  // 2/pi rounded
  constexpr double PIO2_HI = 1.5707963267948966;       // pi/2 rounded
  constexpr double PIO2_LO = 6.123233995736766e-17;    // pi/2 - PIO2_HI rounded
  const double n = rint(x * TWO_OVER_PI);
  double r = fma(-n, PIO2_HI, x);
  r = fma(-n, PIO2_LO, r);
  const int q = (int)n;
  const double r2 = r * r;
  const double c = cos_poly(r2), s = sin_poly(r, r2);
  // cos(q pi/2 + r) = cos r, -sin r, -cos r, sin r and
  // sin(q pi/2 + r) = sin r, cos r, -sin r, -cos r for q = 0, 1, 2, 3 (mod 4)
  const double cv = (q & 1) ? s : c, sv = (q & 1) ? c : s;
  cx = ((q + 1) & 2) ? -cv : cv;
  sx = (q & 2) ? -sv : sv;
}

__device__ __forceinline__ double cos_rf(double x) {
  double c, s;
  sincos_rf(x, c, s);
  return c;
}

// Largest step angle omega (t_new - t) for which the stage phases are
// rotations of the step's start phase built from the small angles below.
constexpr double SMALL_ANGLE = 0.5;

// A rotation by an angle: its cosine and sine.
struct Rot {
  double c, s;
};

// cos and sin of |u| <= SMALL_ANGLE / 9: Taylor series truncated after u^8
// and u^9 (remainders below 0.056^10/10! = 8e-20 and 0.056^11/11! = 4e-22).
__device__ __forceinline__ Rot rot_small(double u) {
  const double u2 = u * u;
  double c = 1.0 / 40320.0;                              // 1/8!
  c = fma(c, u2, -1.0 / 720.0);                          // -1/6!
  c = fma(c, u2, 1.0 / 24.0);                            // 1/4!
  c = fma(c, u2, -0.5);                                  // -1/2!
  double s = 1.0 / 362880.0;                             // 1/9!
  s = fma(s, u2, -1.0 / 5040.0);                         // -1/7!
  s = fma(s, u2, 1.0 / 120.0);                           // 1/5!
  s = fma(s, u2, -1.0 / 6.0);                            // -1/3!
  return {fma(c, u2, 1.0), fma(s * u2, u, u)};
}
// Sum of two angles, and twice an angle.
__device__ __forceinline__ Rot rot_add(Rot a, Rot b) {
  return {fma(a.c, b.c, -(a.s * b.s)), fma(a.s, b.c, a.c * b.s)};
}
__device__ __forceinline__ Rot rot_twice(Rot a) {
  const double s2 = a.s + a.s;
  return {fma(-s2, a.s, 1.0), s2 * a.c};
}

// max(|a|, |b|), max(a, b) and min(a, b) as single v_max_f64 / v_min_f64.
// fmax and fmin would first quiet a possible signalling NaN in each operand
// whose origin the compiler cannot see (one more instruction per operand);
// the operands here are finite or caught by the error norm's NaN test.
__device__ __forceinline__ double max_abs(double a, double b) {
  double r;
  asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// (err/rtol)^(-1/5) for the step-size controller.  Arguments are clamped to
// [1e-30, 1e30]: outside it the controller's own limits (growth at most 5x,
// shrink at least 0.1x) decide.  A single-precision estimate (relative error
// below 1e-6 over that range, ~6e-8 for ratios within 2^+-7) is refined by one
// Newton step of w <- w (6 - q w^5) / 5, which maps a relative error e to
// -3 e^2 (below 3e-12; the step size carries it, far below the ~1e-7 rounding
// noise of the error estimate it is computed from).  The step is written
// 1.2 w - 0.2 q w^6 so that it is four dependent operations deep.
__device__ __forceinline__ double inv_fifth_root(double q) {
  q = fmin(fmax(q, 1e-30), 1e30);
  const double w = (double)__builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf((float)q));
  const double w2 = w * w;
  const double w3 = w2 * w;
  return fma(-0.2 * q, w3 * w3, 1.2 * w);
}

// g_a = (dV/dr)/(r m_atom) of V(r) = -Cn/r^n + Cm/r^m (Sec. 2.1; general n, m
// in Sec. 4.1) from s = 1/r^2: for n = 4, m = 8, s^3 (4 C4 - 8 C8 s^2) / m_atom
// with the constants divided by m_atom on the host.
__device__ __forceinline__ double force_g(const Force& P, double s) {
  const double s2 = s * s;
  return (s2 * s) * fma(-P.mCa, s2, P.nCa);
}

// r^-k = s^(k/2) for an exponent k the same across the launch: binary powers
// of s, times 1/r for odd k.
__device__ __forceinline__ double inv_rpow(double s, double rinv, int k) {
  double p = (k & 1) ? rinv : 1.0, b = s;
  for (int e = k >> 1; e > 0; e >>= 1) {
    if (e & 1) p *= b;
    b *= b;
  }
  return p;
}

__device__ __forceinline__ double force_g(const ForceNM& P, double s) {
  const double rinv = ((P.en | P.em) & 1) ? sqrt(s) : 0.0;
  return fma(P.nCa, inv_rpow(s, rinv, P.en), -P.mCa * inv_rpow(s, rinv, P.em));
}

// Accelerations F(t, X) of Sec. 2.1 for V(r) = -C4/r^4 + C8/r^8:
// F_ion = -(g/m_ion) d - kappa(t) x_ion, F_atom = (g/m_atom) d with
// d = x_ion - x_atom and g = (dV/dr)/r, formed as F_atom = g_a d and F_ion =
// -(m_atom/m_ion) F_atom - kappa(t) x_ion (g_a = g/m_atom): the ion's
// interaction term is the atom's times the mass ratio, which saves a product
// per stage.  cosrf = cos(omega t).  Returns r^2 and d.
template <class C>
__device__ __forceinline__ double accel(const C& P, double cosrf, const double* X,
                                        double* F, double& dx, double& dy, double& dz) {
  dx = X[0] - X[3];
  dy = X[1] - X[4];
  dz = X[2] - X[5];
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double s = recip_force(r2);
  const double ga = force_g(P, s);
  F[3] = ga * dx;
  F[4] = ga * dy;
  F[5] = ga * dz;
  // -(mr F_atom + kappa x) written as (-mr) F_atom + kappa (-x): the same
  // value (the rounding is symmetric), with the negations as free operand
  // modifiers
  F[0] = fma(-P.mr, F[3], fma(P.kq[0], cosrf, P.ka[0]) * -X[0]);
  F[1] = fma(-P.mr, F[4], fma(P.kq[1], cosrf, P.ka[1]) * -X[1]);
  F[2] = fma(-P.mr, F[5], fma(P.kq[2], cosrf, P.ka[2]) * -X[2]);
  return r2;
}

// The y0 column of trajectory idx.
__device__ __forceinline__ void load_column(const Launch& P, long long idx, double* y) {
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = P.y0[c * P.ld + idx];
}

// 1/a in single precision: hardware estimate and one Newton step.
__device__ __forceinline__ float recipf(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return fmaf(r, fmaf(-a, r, 1.0f), r);
}

// The accelerations of accel() in single precision, from the separation
// d = x_ion - x_atom and the ion position xi, both formed by the caller from
// the double-precision state plus single-precision stage increments.
// Returns r^2.
__device__ __forceinline__ float accel32(const Force32& P, float cosrf, const float* d,
                                         const float* xi, float* F) {
  const float r2 = fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
  const float s = recipf(r2);
  const float s2 = s * s;
  const float ga = (s2 * s) * fmaf(-P.mCa, s2, P.nCa);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    F[3 + k] = ga * d[k];
    F[k] = -fmaf(P.mr, F[3 + k], fmaf(P.kq[k], cosrf, P.ka[k]) * xi[k]);
  }
  return r2;
}

// What starting a trajectory needs besides its initial state, the same for
// every trajectory of a call: t0, the trap phase at t0, the initial step's cap
// min(hmax, tf - t0) and floor 16 eps(t0), AbsTol/RelTol, 0.8 RelTol^(1/5).
struct StartConst {
  double t0, cph0, sph0, hcap, hmin0, thr, inv_hinit;  // inv_hinit = 1 / (0.8 rtol^(1/5))
};

__device__ __forceinline__ StartConst start_const(const Launch& P) {
  StartConst S;
  S.t0 = P.t0;
  sincos_rf(P.omega * P.t0, S.cph0, S.sph0);
  S.hcap = fmin(P.hmax, P.tf - P.t0);
  S.hmin0 = 16.0 * spacing(P.t0);
  S.thr = P.thr;
  S.inv_hinit = 1.0 / P.hinit_den;
  return S;
}

// Start of a trajectory from its initial state y: f(t0, y0), ode45's initial
// step and the observables' initial values.
template <class F>
__device__ __forceinline__ void start(const F& Fc, const StartConst& S, const double* y,
                                      Lane& L) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.x[k] = y[k];
    L.v[k] = y[3 + k];
    L.x[3 + k] = y[6 + k];
    L.v[3 + k] = y[9 + k];
  }
  double dx, dy, dz;
  L.cph = S.cph0;
  L.sph = S.sph0;
  const double r2 = accel(Fc, L.cph, L.x, L.F1, dx, dy, dz);
  L.t = S.t0;
  L.nsteps = L.bounces = 0;
  L.nfailed = 0;
  L.fresh = true;
  L.done = false;
  L.nofailed = true;

  // initial step: the weighted first-order increment h f(t0, y0) equals
  // 0.8 rtol^(1/5); position derivatives are the velocities.  The largest
  // |f_c| / max(|y_c|, thr) is found by cross-multiplication along two chains
  // (the six position and the six velocity components) merged at the end,
  // which keeps both the registers and the dependency chain short, then one
  // reciprocal.
  bool finite = true;
  double num[2] = {0.0, 0.0}, den[2] = {1.0, 1.0};
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const int g = c < 6 ? 0 : 1;
    const double f = c < 6 ? L.v[c] : L.F1[c - 6];
    const double y = c < 6 ? L.x[c] : L.v[c - 6];
    finite = finite && isfinite(f) && isfinite(y);
    const double dc = max_abs(y, S.thr);
    if (fabs(f) * den[g] > fabs(num[g]) * dc) {
      num[g] = f;
      den[g] = dc;
    }
  }
  if (fabs(num[1]) * den[0] > fabs(num[0]) * den[1]) {
    num[0] = num[1];
    den[0] = den[1];
  }
  const double rh = fabs(num[0]) * recip(den[0]) * S.inv_hinit;
  double absh = S.hcap;
  if (absh * rh > 1.0) absh = recip(rh);
  L.absh = fmax(absh, S.hmin0);
  L.status = finite ? 0 : AI_ST_NONFINITE;

  const double w = fma(dz, L.v[2] - L.v[5], fma(dy, L.v[1] - L.v[4], dx * (L.v[0] - L.v[3])));
  L.approached = (w >= 0.0);
  L.w_prev = w;
  L.t_first = L.t_last = L.position = 0.0;
  L.rmin2 = r2;
}

// Step set-up of ode45: floor and cap the step, stretch it onto tf when within
// 10% of the remaining span.
template <class LN>
__device__ __forceinline__ void begin_step(const Ctl& K, LN& L) {
  const double hmin = 16.0 * spacing(L.t);
  L.absh = vmin(K.hmax, vmax(hmin, L.absh));
  L.done = false;
  if (1.1 * L.absh >= K.tf - L.t) {
    L.absh = K.tf - L.t;
    L.done = true;
  }
  L.nofailed = true;
}

// Trap phase at the stage times t + c h, c = 1/5, 3/10, 4/5, 8/9, 1: cos for
// each and sin for the last, from the tracked (cos, sin)(omega t).
__device__ __forceinline__ void stage_phases(const Ctl& K, double cph, double sph, double t,
                                             double h, double& cs2, double& cs3, double& cs4,
                                             double& cs5, double& cs6, double& sn6) {
  // trap phase at the stage times: rotations of (cos, sin)(omega t) by
  // c omega (t_new - t), the exact step span of the double t_new (it differs
  // from h by the rounding of t + h, a stage-time shift no larger than the
  // rounding of t + c h itself).  The angles are built from theta = d/10 and
  // phi = d/9 (d = omega (t_new - t)): 2, 3, 8 and 10 theta by doubling and
  // addition; the phase at 8/9 d is the end phase (10 theta) turned back by
  // phi.  The stage-6 rotation also advances the
  // phase on acceptance.  A lane whose step spans more than SMALL_ANGLE
  // radians evaluates each phase directly instead.
  const double tn = t + h;
  const double omega = K.omega;
  const double d6 = omega * (tn - t);
  {
    const Rot r1 = rot_small(0.1 * d6), phi = rot_small((1.0 / 9.0) * d6);
    const Rot r2 = rot_twice(r1), r3 = rot_add(r2, r1), r4 = rot_twice(r2);
    const Rot r8 = rot_twice(r4), r10 = rot_add(r8, r2);
    const double C = cph, S = sph;
    cs2 = fma(C, r2.c, -(S * r2.s));
    cs3 = fma(C, r3.c, -(S * r3.s));
    cs4 = fma(C, r8.c, -(S * r8.s));
    cs6 = fma(C, r10.c, -(S * r10.s));
    sn6 = fma(S, r10.c, C * r10.s);
    cs5 = fma(cs6, phi.c, sn6 * phi.s);  // the end phase turned back by d/9
    if (!(fabs(d6) <= SMALL_ANGLE)) {
      cs2 = cos_rf(omega * fma(C2, h, t));
      cs3 = cos_rf(omega * fma(C3, h, t));
      cs4 = cos_rf(omega * fma(C4, h, t));
      cs5 = cos_rf(omega * fma(C5, h, t));
      sincos_rf(omega * tn, cs6, sn6);
    }
  }
}

// dst = src by one move into dst's own register (executed by the lanes of the
// current branch only), so that a value carried around the loop keeps its
// register on both sides of a divergent branch.
__device__ __forceinline__ void move_into(double& dst, double src) {
  asm volatile("v_mov_b64 %0, %1" : "+v"(dst) : "v"(src));
}
__device__ __forceinline__ void move_into(float& dst, float src) {
  asm volatile("v_mov_b32 %0, %1" : "+v"(dst) : "v"(src));
}

// Of two error components (signed value, positive scale), the one with the
// larger ratio |value| / scale, compared by cross-multiplication; the first on
// a tie (the initial step's largest weighted derivative).
__device__ __forceinline__ void pick(double& na, double& da, double nb, double db) {
  if (fabs(nb) * da > fabs(na) * db) {
    na = nb;
    da = db;
  }
}

// |e| / s for the error norm: the hardware reciprocal estimate (relative
// error below 2^-23) refined by one Newton step, r (1 + (1 - s r)), to a
// relative error below 2^-46, times |e|.  The norm's largest ratio then
// differs from the quotients' by at most that much (ties within it may pick
// either component, which changes the norm by no more), so an accept/reject
// decision differs from the exact division's only where err lies within
// ~1e-14 of RelTol.  (The estimate alone, 2^-23, flipped such decisions: one
// of 95 non-chaotic trajectories of a 10 uK ensemble then took another step
// sequence and ended 5e-5 away.)  s = inf gives NaN, which only a non-finite
// solution can produce (the attempt then ends as non-finite either way).
__device__ __forceinline__ double ratio(double e, double s) {
  const double r = __builtin_amdgcn_rcp(s);
  return fabs(e) * fma(r, fma(-s, r, 1.0), r);
}

// The error norm err = h max_c |e_c| / max(|y_c|, |ynew_c|, AbsTol/RelTol)
// over the twelve components, as a maximum of per-component ratios (exact, so
// in any order; the paths below all take it the same way: for each half, the
// ion's and the atom's ratio of each axis, then the axes as ((x, y), z); then
// the position half's against the velocity half's).  The position half is
// reduced before the last force evaluation, which keeps few of its values
// live across it.  half_norm() reduces one half: e the error components, y
// and yn the solution before and after; m receives the half's largest ratio.
// The maximum instructions drop NaN operands; a NaN or infinite error
// component comes with a non-finite new state, which conclude() catches.
template <class RE>
__device__ __forceinline__ void half_norm(const Ctl& K, const RE* e, const double* y,
                                          const double* yn, double& m) {
  double ax[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double r0 = ratio((double)e[k], max_abs(max_abs(y[k], yn[k]), K.thr));
    const double r1 = ratio((double)e[3 + k], max_abs(max_abs(y[3 + k], yn[3 + k]), K.thr));
    ax[k] = vmax(r0, r1);
  }
  m = vmax(vmax(ax[0], ax[1]), ax[2]);
}

// The error norm's largest ratio given the position half's, mx: mx against
// the velocity half's.  Every velocity scale is at least AbsTol/RelTol, so a
// velocity ratio as ratio() forms it (within 2^-45 of |e| RelTol/AbsTol) is
// below max_c |e_c| vbound; when that bound is at most mx the maximum is mx
// itself, and the velocity half's scales and reciprocals are not formed (for
// thermal collisions the velocity scales sit at the floor AbsTol/RelTol, far
// above |v|, and the position half decides every step).  The result is the
// same either way.
template <class RE>
__device__ __forceinline__ double with_velocity_half(const Ctl& K, const RE* e, const double* v,
                                                     const double* vn, double mx) {
  double a[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) a[c] = (double)e[c];
  const double big = max_abs(max_abs(max_abs(a[0], a[3]), max_abs(a[1], a[4])), max_abs(a[2], a[5]));
  if (big * K.vbound <= mx) return mx;
  double mv;
  half_norm(K, e, v, vn, mv);
  return vmax(mx, mv);
}

// The rest of an attempt, the same in every path: the error test and ode45's
// step-size control; on acceptance advance() moves the lane's state to tnew
// (the phase is rotated here), and the observables and exits are updated from
// w() = d . (v_ion - v_atom) and r2n = |d|^2 at tnew; ion_distance() gives
// |x_ion| at tnew for the first bounce.
//
// The attempt ends the trajectory as non-finite when an error component is
// NaN or infinite, tested without looking at each of the twelve components:
// the first-stage force is finite (the previous attempt would have ended
// otherwise), stages 3-6 enter the new velocity with nonzero weights and
// stage 2 enters the positions of stages 4-6, so a non-finite force of stages
// 2-6 (the only way the components without stage 7 can be non-finite) makes
// the new velocity, and with it w(), non-finite.  Stage 7's force, from the
// new position, is NaN only if that position is or r2n is 0, and infinite
// otherwise, which makes err infinite.  Hence the test on err, w and r2n.
template <class LN, class Advance, class W, class IonDistance>
__device__ __forceinline__ void conclude(const Ctl& K, LN& L, double t, double h, double tnew,
                                         double err, double cs6, double sn6, double r2n,
                                         Advance advance, W w_of, IonDistance ion_distance) {
  const double w = w_of();
  if (!isfinite(err) || !isfinite(w) || !(r2n > 0.0)) {
    L.status = AI_ST_NONFINITE;
    return;
  }
  const double w5 = inv_fifth_root(err * K.inv_rtol);  // (err/rtol)^(-1/5)
  if (err > K.rtol) {
    L.nfailed += 1;
    const double hmin = 16.0 * spacing(t);
    if (h <= hmin) {
      L.status = AI_ST_HMIN;
      return;
    }
    move_into(L.absh, L.nofailed ? fmax(hmin, h * fmax(0.1, 0.8 * w5)) : fmax(hmin, 0.5 * h));
    L.nofailed = false;
    L.done = false;
    L.fresh = false;
    return;
  }

  // accepted
  L.nsteps += 1;
  move_into(L.t, tnew);
  move_into(L.cph, cs6);
  move_into(L.sph, sn6);
  advance();
  // growth 1/(1.25 (err/rtol)^(1/5)), at most 5x
  if (L.nofailed) move_into(L.absh, (w5 < 6.25) ? h * (0.8 * w5) : 5.0 * h);
  L.fresh = true;

  // observables: closest approach = sign change of r r' from - to +
  if (L.w_prev < 0.0 && w >= 0.0) {
    L.approached = true;
    if (r2n < K.r_bounce2) {
      L.bounces += 1;
      if (L.bounces == 1) {
        L.t_first = tnew;
        L.position = ion_distance();
      }
      L.t_last = tnew;
    }
  }
  L.w_prev = w;
  L.rmin2 = vmin(L.rmin2, r2n);

  if (L.approached && K.exit_on && r2n > K.r_exit2)
    L.status = AI_ST_ESCAPED;
  else if (L.done)
    L.status = AI_ST_TMAX;
  else if (L.nsteps >= K.max_steps)
    L.status = AI_ST_MAXSTEPS;
}

// conclude() for a one-lane attempt: the new state xn, vn, F7 and the
// separation d = (dx, dy, dz) at tnew.
template <class R, class R7>
__device__ __forceinline__ void conclude_lane(const Ctl& K, LaneT<R>& L, double t, double h,
                                              double tnew, double err, const double* xn,
                                              const double* vn, const R7* F7, double cs6,
                                              double sn6, double dx, double dy, double dz,
                                              double r2n) {
  conclude(
      K, L, t, h, tnew, err, cs6, sn6, r2n,
      [&] {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          move_into(L.x[c], xn[c]);
          move_into(L.v[c], vn[c]);
          move_into(L.F1[c], (R)F7[c]);
        }
      },
      [&] { return fma(dz, vn[2] - vn[5], fma(dy, vn[1] - vn[4], dx * (vn[0] - vn[3]))); },
      [&] { return sqrt(fma(xn[2], xn[2], fma(xn[1], xn[1], xn[0] * xn[0]))); });
}

// One Dormand-Prince attempt of size h = absh from (t, x, v), the error test
// and the controller; on acceptance the state advances and the observables
// and exits are updated.
template <class F>
__device__ __forceinline__ void attempt(const F& P, const Ctl& K, Lane& L) {
  const double t = L.t, h = L.absh, hh = h * h;
  const double tnew = L.done ? K.tf : t + h;  // t + h is also tn below
  const double* x = L.x;
  const double* v = L.v;
  const double* F1 = L.F1;
  double X[6], F2[6], F3[6], F4[6], F5[6], F6[6], F7[6];
  double dx, dy, dz;

  double cs2, cs3, cs4, cs5, cs6, sn6;
  stage_phases(K, L.cph, L.sph, t, h, cs2, cs3, cs4, cs5, cs6, sn6);
  {
    const double a = C2 * h;
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = fma(a, v[c], x[c]);
    accel(P, cs2, X, F2, dx, dy, dz);
  }
  {
    const double a = C3 * h, q1 = Q31 * hh;
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = fma(q1, F1[c], fma(a, v[c], x[c]));
    accel(P, cs3, X, F3, dx, dy, dz);
  }
  {
    const double a = C4 * h, q1 = Q41 * hh, q2 = Q42 * hh;
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = fma(q2, F2[c], fma(q1, F1[c], fma(a, v[c], x[c])));
    accel(P, cs4, X, F4, dx, dy, dz);
  }
  {
    const double a = C5 * h, q1 = Q51 * hh, q2 = Q52 * hh, q3 = Q53 * hh;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      X[c] = fma(q3, F3[c], fma(q2, F2[c], fma(q1, F1[c], fma(a, v[c], x[c]))));
    accel(P, cs5, X, F5, dx, dy, dz);
  }
  {
    const double q1 = Q61 * hh, q2 = Q62 * hh, q3 = Q63 * hh, q4 = Q64 * hh;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      X[c] = fma(q4, F4[c], fma(q3, F3[c], fma(q2, F2[c], fma(q1, F1[c], fma(h, v[c], x[c])))));
    accel(P, cs6, X, F6, dx, dy, dz);
  }
  // new solution, error vector (without F7) and stage 7
  double xn[6], vn[6], ex[6], ev[6];
  {
    const double q1 = Q71 * hh, q3 = Q73 * hh, q4 = Q74 * hh, q5 = Q75 * hh;
    const double b1 = B1 * h, b3 = B3 * h, b4 = B4 * h, b5 = B5 * h, b6 = B6 * h;
    const double p1 = P1 * h, p3 = P3 * h, p4 = P4 * h, p5 = P5 * h, p6 = P6 * h;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      xn[c] = fma(q5, F5[c], fma(q4, F4[c], fma(q3, F3[c], fma(q1, F1[c], fma(h, v[c], x[c])))));
      vn[c] = fma(b6, F6[c], fma(b5, F5[c], fma(b4, F4[c], fma(b3, F3[c], fma(b1, F1[c], v[c])))));
      ex[c] = fma(p6, F6[c], fma(p5, F5[c], fma(p4, F4[c], fma(p3, F3[c], p1 * F1[c]))));
      ev[c] = fma(E6, F6[c], fma(E5, F5[c], fma(E4, F4[c], fma(E3, F3[c], E1 * F1[c]))));
    }
  }
  // stage 7 at tnew; tnew == t + h unless the step was stretched onto tf
  const double cos7 = L.done ? cos_rf(K.omega * tnew) : cs6;
  // error norm (order in half_norm()): the position half, stage 7, the
  // velocity half
  double mx;
  half_norm(K, ex, x, xn, mx);
  const double r2n = accel(P, cos7, xn, F7, dx, dy, dz);
  double ev7[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) ev7[c] = fma(E7, F7[c], ev[c]);
  const double m = with_velocity_half(K, ev7, v, vn, mx);
  const double err = h * m;
  conclude_lane(K, L, t, h, tnew, err, xn, vn, F7, cs6, sn6, dx, dy, dz, r2n);
}

// Dormand-Prince coefficients in single precision for the variant below.
constexpr float C2f = (float)C2, C3f = (float)C3, C4f = (float)C4, C5f = (float)C5;
constexpr float B1f = (float)B1, B3f = (float)B3, B4f = (float)B4, B5f = (float)B5,
                B6f = (float)B6;
constexpr float E1f = (float)E1, E3f = (float)E3, E4f = (float)E4, E5f = (float)E5,
                E6f = (float)E6, E7f = (float)E7;
constexpr float Q31f = (float)Q31, Q41f = (float)Q41, Q42f = (float)Q42, Q51f = (float)Q51,
                Q52f = (float)Q52, Q53f = (float)Q53, Q61f = (float)Q61, Q62f = (float)Q62,
                Q63f = (float)Q63, Q64f = (float)Q64, Q71f = (float)Q71, Q73f = (float)Q73,
                Q74f = (float)Q74, Q75f = (float)Q75;
constexpr float P1f = (float)P1, P3f = (float)P3, P4f = (float)P4, P5f = (float)P5,
                P6f = (float)P6;

// One attempt with single-precision stages: the stage increments, forces and
// error sums are float; the state, t, h, the trap phase and the error norm
// stay double, as does the h v term of every stage position and of the new
// position.  A stage position is the double state plus a float increment
// D_s = h^2 sum_l (A^2)_sl F_l (+ c_s h v, narrowed); the ion-atom separation
// is x_ion - x_atom formed in double once per attempt, narrowed, plus
// D_s(ion) - D_s(atom), so r keeps its precision at short range.  The error
// estimate's float rounding (a relative 6e-8 of the cancelling sums) stays far
// below RelTol for the configured tolerances.
__device__ __forceinline__ void attempt32(const Force32& P, const Ctl& K, Lane& L) {
  const double t = L.t, h = L.absh, hh = h * h;
  const double tnew = L.done ? K.tf : t + h;
  const double* x = L.x;
  const double* v = L.v;
  float F1[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) F1[c] = (float)L.F1[c];
  double cs2, cs3, cs4, cs5, cs6, sn6;
  stage_phases(K, L.cph, L.sph, t, h, cs2, cs3, cs4, cs5, cs6, sn6);

  float d0[3], xi[3], hv[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d0[k] = (float)(x[k] - x[3 + k]);
    xi[k] = (float)x[k];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) hv[c] = (float)(h * v[c]);
  const float hf = (float)h, hhf = (float)hh;
  float D[6], d[3], Xi[3], F2[6], F3[6], F4[6], F5[6], F6[6], F7[6];
  auto stage = [&](double cs, float* F) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d[k] = d0[k] + (D[k] - D[3 + k]);
      Xi[k] = xi[k] + D[k];
    }
    accel32(P, (float)cs, d, Xi, F);
  };
#pragma unroll
  for (int c = 0; c < 6; ++c) D[c] = C2f * hv[c];
  stage(cs2, F2);
  {
    const float q1 = Q31f * hhf;
#pragma unroll
    for (int c = 0; c < 6; ++c) D[c] = fmaf(q1, F1[c], C3f * hv[c]);
    stage(cs3, F3);
  }
  {
    const float q1 = Q41f * hhf, q2 = Q42f * hhf;
#pragma unroll
    for (int c = 0; c < 6; ++c) D[c] = fmaf(q2, F2[c], fmaf(q1, F1[c], C4f * hv[c]));
    stage(cs4, F4);
  }
  {
    const float q1 = Q51f * hhf, q2 = Q52f * hhf, q3 = Q53f * hhf;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      D[c] = fmaf(q3, F3[c], fmaf(q2, F2[c], fmaf(q1, F1[c], C5f * hv[c])));
    stage(cs5, F5);
  }
  {
    const float q1 = Q61f * hhf, q2 = Q62f * hhf, q3 = Q63f * hhf, q4 = Q64f * hhf;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      D[c] = fmaf(q4, F4[c], fmaf(q3, F3[c], fmaf(q2, F2[c], fmaf(q1, F1[c], hv[c]))));
    stage(cs6, F6);
  }
  // new solution (double state plus float sums), error sums without F7
  double xn[6], vn[6];
  float ex[6], ev[6];
  {
    const float q1 = Q71f * hhf, q3 = Q73f * hhf, q4 = Q74f * hhf, q5 = Q75f * hhf;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float G = fmaf(q5, F5[c], fmaf(q4, F4[c], fmaf(q3, F3[c], q1 * F1[c])));
      const float B =
          fmaf(B6f, F6[c], fmaf(B5f, F5[c], fmaf(B4f, F4[c], fmaf(B3f, F3[c], B1f * F1[c]))));
      xn[c] = fma(h, v[c], x[c]) + (double)G;
      vn[c] = fma(h, (double)B, v[c]);
      ex[c] = hf * fmaf(P6f, F6[c], fmaf(P5f, F5[c], fmaf(P4f, F4[c], fmaf(P3f, F3[c], P1f * F1[c]))));
      ev[c] = fmaf(E6f, F6[c], fmaf(E5f, F5[c], fmaf(E4f, F4[c], fmaf(E3f, F3[c], E1f * F1[c]))));
    }
  }
  // error norm in double, as in attempt(): the position half, stage 7 at tnew
  // from the new double state, the velocity half
  double mx;
  half_norm(K, ex, x, xn, mx);
  const double cos7 = L.done ? cos_rf(K.omega * tnew) : cs6;
  const double dx = xn[0] - xn[3], dy = xn[1] - xn[4], dz = xn[2] - xn[5];
  float r2f;
  {
    const float dn[3] = {(float)dx, (float)dy, (float)dz};
    const float xin[3] = {(float)xn[0], (float)xn[1], (float)xn[2]};
    r2f = accel32(P, (float)cos7, dn, xin, F7);
  }
  const double r2n = fma(dz, dz, fma(dy, dy, dx * dx));
  float ev7[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) ev7[c] = fmaf(E7f, F7[c], ev[c]);
  const double m = with_velocity_half(K, ev7, v, vn, mx);
  // stage 7's single-precision force is not finite also when the separation's
  // square underflows in single precision (r2f = 0 with r2n > 0)
  const double err = (r2f > 0.0f) ? h * m : __builtin_nan("");
  conclude_lane(K, L, t, h, tnew, err, xn, vn, F7, cs6, sn6, dx, dy, dz, r2n);
}

// End of trajectory idx: store the final state and the raw accumulators.
// Derived observables are formed afterwards by ai_finalize_kernel from these
// planes (the plain and batched kernels form them at the end instead:
// finish_derived), so the integration loops carry no atan2 or square roots;
// until then the lifetime, angle, transfer, dist, ke and rmin planes hold
// t_first, t_last, the atom's initial velocity (3 planes) and rmin^2.
// va0 is the atom's initial velocity (kept by the caller: final_state may be
// the y0 buffer itself).
template <class R>
__device__ __forceinline__ void finish(double* yf, double* obs, long long ld, const LaneT<R>& L,
                                       long long idx, double va0x, double va0y, double va0z) {
  double o[AI_NOBS];
  o[AI_OBS_TEND] = L.t;
  o[AI_OBS_STATUS] = (double)L.status;
  o[AI_OBS_NSTEPS] = (double)L.nsteps;
  o[AI_OBS_NFAILED] = (double)L.nfailed;
  o[AI_OBS_BOUNCES] = (double)L.bounces;
  o[AI_OBS_LIFETIME] = L.t_first;
  o[AI_OBS_ANGLE] = L.t_last;
  o[AI_OBS_TRANSFER] = va0x;
  o[AI_OBS_POSITION] = L.position;
  o[AI_OBS_DIST] = va0y;
  o[AI_OBS_KE] = va0z;
  o[AI_OBS_RMIN] = L.rmin2;
  o[AI_OBS_HNEXT] = L.absh;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    yf[k * ld + idx] = L.x[k];
    yf[(3 + k) * ld + idx] = L.v[k];
    yf[(6 + k) * ld + idx] = L.x[3 + k];
    yf[(9 + k) * ld + idx] = L.v[3 + k];
  }
#pragma unroll
  for (int c = 0; c < AI_NOBS; ++c) obs[c * ld + idx] = o[c];
}

// Observables of Sec. 4.1 from the final state and the raw accumulators:
// lifetime = t_last - t_first for two or more bounces, scattering angle
// between the atom's initial and final velocity, momentum transfer
// m_atom |v - v0|, final distance, final ion kinetic energy, smallest distance.
struct Derived {
  double lifetime, angle, transfer, dist, ke, rmin;
};

// From the raw accumulators, the atom's initial and final velocity va0, va,
// the ion's final velocity vi and the final separation d = x_ion - x_atom.
__device__ __forceinline__ Derived derive_from(double t_first, double t_last, double va0x,
                                               double va0y, double va0z, double rmin2,
                                               double bounces, double vix, double viy, double viz,
                                               double vax, double vay, double vaz, double dx,
                                               double dy, double dz, double m_atom,
                                               double half_mi) {
  const double cx = fma(va0y, vaz, -(va0z * vay));
  const double cy = fma(va0z, vax, -(va0x * vaz));
  const double cz = fma(va0x, vay, -(va0y * vax));
  const double dot = fma(va0z, vaz, fma(va0y, vay, va0x * vax));
  const double dvx = vax - va0x, dvy = vay - va0y, dvz = vaz - va0z;
  Derived d;
  d.lifetime = bounces >= 2.0 ? t_last - t_first : 0.0;
  d.angle = atan2(sqrt(fma(cz, cz, fma(cy, cy, cx * cx))), dot);
  d.transfer = m_atom * sqrt(fma(dvz, dvz, fma(dvy, dvy, dvx * dvx)));
  d.dist = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
  d.ke = half_mi * fma(viz, viz, fma(viy, viy, vix * vix));
  d.rmin = sqrt(rmin2);
  return d;
}

__device__ __forceinline__ Derived derive(double t_first, double t_last, double va0x, double va0y,
                                          double va0z, double rmin2, double bounces,
                                          const double* y, double m_atom, double half_mi) {
  return derive_from(t_first, t_last, va0x, va0y, va0z, rmin2, bounces, y[3], y[4], y[5], y[9],
                     y[10], y[11], y[0] - y[6], y[1] - y[7], y[2] - y[8], m_atom, half_mi);
}

__device__ __forceinline__ void finalize_one(const Launch& P, const double* __restrict__ yf,
                                             double* __restrict__ obs, long long i) {
  const long long ld = P.ld;
  double y[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = yf[c * ld + i];
  const Derived d = derive(obs[AI_OBS_LIFETIME * ld + i], obs[AI_OBS_ANGLE * ld + i],
                           obs[AI_OBS_TRANSFER * ld + i], obs[AI_OBS_DIST * ld + i],
                           obs[AI_OBS_KE * ld + i], obs[AI_OBS_RMIN * ld + i],
                           obs[AI_OBS_BOUNCES * ld + i], y, P.m_atom, P.half_mi);
  obs[AI_OBS_LIFETIME * ld + i] = d.lifetime;
  obs[AI_OBS_ANGLE * ld + i] = d.angle;
  obs[AI_OBS_TRANSFER * ld + i] = d.transfer;
  obs[AI_OBS_DIST * ld + i] = d.dist;
  obs[AI_OBS_KE * ld + i] = d.ke;
  obs[AI_OBS_RMIN * ld + i] = d.rmin;
}

__global__ __launch_bounds__(256) void ai_finalize_kernel(Launch P, const double* __restrict__ yf,
                                                          double* __restrict__ obs) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= P.n) return;
  finalize_one(P, yf, obs, i);
}

// One ensemble of a batched call and the global index of its first
// trajectory; a batch lists them with increasing offsets.
struct BatchEntry {
  Launch P;
  long long offset;
};

// A batched call: its ensembles (device memory), their total trajectory
// count and the optional longest-first order over global indices.
struct BatchLaunch {
  const BatchEntry* entries;
  int count;
  long long total;
  const unsigned* order;
  const unsigned* key;
  long long wide;   // with the order: leading positions integrated four lanes each
  int wide_waves;   // the waves at the start of the grid that hold them
};

// The ensemble holding global index j: the last entry with offset <= j.
__device__ __forceinline__ int batch_entry(const BatchEntry* E, int count, long long j) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (E[mid].offset <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Wave priority from the predicted duration of the wave's longest trajectory
// relative to the longest in the ensemble (both from the longest-first
// schedule).  The longest trajectories set the end of the launch; while they
// share a SIMD with other waves, the higher priority lets them issue first
// and the others fill the gaps.  frac must be uniform across the wave.
__device__ __forceinline__ void set_wave_priority(float frac) {
  if (frac >= 0.5f)
    __builtin_amdgcn_s_setprio(3);
  else if (frac >= 0.25f)
    __builtin_amdgcn_s_setprio(2);
  else if (frac >= 0.125f)
    __builtin_amdgcn_s_setprio(1);
  else
    __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The derived observables out of line, for the resident kernel, where a
// lane ends trajectories inside its loop: inlined there, the temporaries of
// atan2 and the square roots added ~40 registers spilled to scratch.
__device__ __attribute__((noinline)) Derived derive_at_end(
    double t_first, double t_last, double va0x, double va0y, double va0z, double rmin2,
    double bounces, double vix, double viy, double viz, double vax, double vay, double vaz,
    double dx, double dy, double dz, double m_atom, double half_mi) {
  return derive_from(t_first, t_last, va0x, va0y, va0z, rmin2, bounces, vix, viy, viz, vax, vay,
                     vaz, dx, dy, dz, m_atom, half_mi);
}

// finish() with the derived observables formed here, from the same values
// ai_finalize_kernel would read back (so the results are bitwise the same),
// instead of by that kernel afterwards.  Called after the integration loop,
// inline: the loop's registers are free by then.
template <class R>
__device__ __forceinline__ void finish_derived(const Launch& P, const LaneT<R>& L, long long idx,
                                               double va0x, double va0y, double va0z) {
  const Derived d = derive_from(L.t_first, L.t_last, va0x, va0y, va0z, L.rmin2,
                                  (double)L.bounces, L.v[0], L.v[1], L.v[2], L.v[3], L.v[4],
                                  L.v[5], L.x[0] - L.x[3], L.x[1] - L.x[4], L.x[2] - L.x[5],
                                  P.m_atom, P.half_mi);
  const long long ld = P.ld;
  double o[AI_NOBS];
  o[AI_OBS_TEND] = L.t;
  o[AI_OBS_STATUS] = (double)L.status;
  o[AI_OBS_NSTEPS] = (double)L.nsteps;
  o[AI_OBS_NFAILED] = (double)L.nfailed;
  o[AI_OBS_BOUNCES] = (double)L.bounces;
  o[AI_OBS_LIFETIME] = d.lifetime;
  o[AI_OBS_ANGLE] = d.angle;
  o[AI_OBS_TRANSFER] = d.transfer;
  o[AI_OBS_POSITION] = L.position;
  o[AI_OBS_DIST] = d.dist;
  o[AI_OBS_KE] = d.ke;
  o[AI_OBS_RMIN] = d.rmin;
  o[AI_OBS_HNEXT] = L.absh;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.yf[k * ld + idx] = L.x[k];
    P.yf[(3 + k) * ld + idx] = L.v[k];
    P.yf[(6 + k) * ld + idx] = L.x[3 + k];
    P.yf[(9 + k) * ld + idx] = L.v[3 + k];
  }
#pragma unroll
  for (int c = 0; c < AI_NOBS; ++c) P.obs[c * ld + idx] = o[c];
}

// Trajectory idx of the ensemble P, start to end, by one lane.  DERIVE: form
// the derived observables here (finish_derived) rather than leave the raw
// accumulators for ai_finalize_kernel (finish).
template <class R, class F = Force, bool DERIVE = false>
__device__ __forceinline__ void integrate_one(const Launch& P, long long idx) {
  const Ctl K = lane_ctl(P);
  const F Fc = lane_force_of(P, (const F*)nullptr);
  Lane L;
  double y[12];
  load_column(P, idx, y);
  start(Fc, start_const(P), y, L);
  if constexpr (sizeof(R) == sizeof(double)) {
    while (L.status == 0) {
      if (L.fresh) begin_step(K, L);
      attempt(Fc, K, L);
    }
  } else {
    // single-precision stages while the lane's atom is farther than r_near
    // from its ion, the double attempt closer, so collisions are integrated in
    // double.  The choice is the lane's own (a wave with lanes on both sides
    // runs both branches), so results do not depend on which trajectories
    // share a wave.
    const Force32 F32 = lane_force32(P);
    const double near2 = in_vgpr(P.near2);
    while (L.status == 0) {
      if (L.fresh) begin_step(K, L);
      const double dx = L.x[0] - L.x[3], dy = L.x[1] - L.x[4], dz = L.x[2] - L.x[5];
      if (fma(dz, dz, fma(dy, dy, dx * dx)) < near2)
        attempt(Fc, K, L);
      else
        attempt32(F32, K, L);
    }
  }
  // the initial atom velocity is read before final_state (possibly y0) is written
  const double* va0 = P.y0 + 9 * P.ld + idx;
  if constexpr (DERIVE)
    finish_derived(P, L, idx, va0[0], va0[P.ld], va0[2 * P.ld]);
  else
    finish(P.yf, P.obs, P.ld, L, idx, va0[0], va0[P.ld], va0[2 * P.ld]);
}

// ---- Four lanes per trajectory ----
//
// A scheduled launch ends with its longest trajectories (thousands of
// attempts where the bulk needs hundreds), and one lane runs an attempt no
// faster than its wave issues the ~700 instructions of the loop.  The leading
// positions of the longest-first order therefore run four lanes each: lane a
// of a quad holds axis a (lane 3 repeats axis 2) of the ion's and the atom's
// position, velocity and acceleration, and does that axis's share of the stage
// sums, the forces and the error components, about a third of the
// arithmetic.  The separation components, the velocity differences and the
// per-axis error maxima pass between the quad's lanes by DPP; everything that
// depends on all three axes (|d|^2, the force magnitude, the step-size
// control, the observables) is computed by each lane from the same operands
// in the same order as the one-lane path, so every lane of the quad takes the
// same decisions and the results are bitwise those of one lane.

// v of lane SRC of this lane's quad (quad_perm [SRC, SRC, SRC, SRC]).  Every
// lane of a quad is active whenever one is: they integrate one trajectory and
// take the same decisions.
template <int SRC>
__device__ __forceinline__ int from_quad_lane(int v) {
  return __builtin_amdgcn_mov_dpp(v, SRC * 0x55, 0xf, 0xf, true);
}
template <int SRC>
__device__ __forceinline__ double from_quad_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = from_quad_lane<SRC>((int)b), hi = from_quad_lane<SRC>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double axis_value(int ax, double a0, double a1, double a2) {
  return ax == 0 ? a0 : (ax == 1 ? a1 : a2);
}

// One lane's share of a trajectory: axis ax of the ion's and the atom's
// position, velocity and acceleration; the rest as in Lane.
struct WideLane {
  double xi, xa, vi, va, Fi, Fa;
  double t, absh;
  double cph, sph;
  double w_prev, t_first, t_last, position, rmin2;
  long long nfailed;
  int nsteps, bounces, status;
  int done, nofailed, fresh, approached;
};

// accel() for axis ax of the stage position (Xi, Xa): the trap coefficients of
// that axis are ka, kq.  Returns r^2, the separation (dx, dy, dz) and the
// axis's accelerations.
template <class F>
__device__ __forceinline__ double accel_wide(const F& P, double ka, double kq, double cosrf,
                                             double Xi, double Xa, double& Fi, double& Fa,
                                             double& dx, double& dy, double& dz) {
  const double d = Xi - Xa;
  dx = from_quad_lane<0>(d);
  dy = from_quad_lane<1>(d);
  dz = from_quad_lane<2>(d);
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double s = recip_force(r2);
  const double ga = force_g(P, s);
  Fa = ga * d;
  Fi = -fma(P.mr, Fa, fma(kq, cosrf, ka) * Xi);
  return r2;
}

// attempt() on one axis per lane.
template <class F>
__device__ __forceinline__ void attempt_wide(const F& P, double ka, double kq, const Ctl& K,
                                             WideLane& L) {
  const double t = L.t, h = L.absh, hh = h * h;
  const double tnew = L.done ? K.tf : t + h;
  const double xi = L.xi, xa = L.xa, vi = L.vi, va = L.va, F1i = L.Fi, F1a = L.Fa;
  double F2i, F2a, F3i, F3a, F4i, F4a, F5i, F5a, F6i, F6a, F7i, F7a;
  double dx, dy, dz;

  double cs2, cs3, cs4, cs5, cs6, sn6;
  stage_phases(K, L.cph, L.sph, t, h, cs2, cs3, cs4, cs5, cs6, sn6);
  {
    const double a = C2 * h;
    accel_wide(P, ka, kq, cs2, fma(a, vi, xi), fma(a, va, xa), F2i, F2a, dx, dy, dz);
  }
  {
    const double a = C3 * h, q1 = Q31 * hh;
    accel_wide(P, ka, kq, cs3, fma(q1, F1i, fma(a, vi, xi)), fma(q1, F1a, fma(a, va, xa)), F3i,
               F3a, dx, dy, dz);
  }
  {
    const double a = C4 * h, q1 = Q41 * hh, q2 = Q42 * hh;
    accel_wide(P, ka, kq, cs4, fma(q2, F2i, fma(q1, F1i, fma(a, vi, xi))),
               fma(q2, F2a, fma(q1, F1a, fma(a, va, xa))), F4i, F4a, dx, dy, dz);
  }
  {
    const double a = C5 * h, q1 = Q51 * hh, q2 = Q52 * hh, q3 = Q53 * hh;
    accel_wide(P, ka, kq, cs5, fma(q3, F3i, fma(q2, F2i, fma(q1, F1i, fma(a, vi, xi)))),
               fma(q3, F3a, fma(q2, F2a, fma(q1, F1a, fma(a, va, xa)))), F5i, F5a, dx, dy, dz);
  }
  {
    const double q1 = Q61 * hh, q2 = Q62 * hh, q3 = Q63 * hh, q4 = Q64 * hh;
    accel_wide(P, ka, kq, cs6,
               fma(q4, F4i, fma(q3, F3i, fma(q2, F2i, fma(q1, F1i, fma(h, vi, xi))))),
               fma(q4, F4a, fma(q3, F3a, fma(q2, F2a, fma(q1, F1a, fma(h, va, xa))))), F6i, F6a,
               dx, dy, dz);
  }
  double xni, xna, vni, vna, exi, exa, evi, eva;
  {
    const double q1 = Q71 * hh, q3 = Q73 * hh, q4 = Q74 * hh, q5 = Q75 * hh;
    const double b1 = B1 * h, b3 = B3 * h, b4 = B4 * h, b5 = B5 * h, b6 = B6 * h;
    const double p1 = P1 * h, p3 = P3 * h, p4 = P4 * h, p5 = P5 * h, p6 = P6 * h;
    xni = fma(q5, F5i, fma(q4, F4i, fma(q3, F3i, fma(q1, F1i, fma(h, vi, xi)))));
    xna = fma(q5, F5a, fma(q4, F4a, fma(q3, F3a, fma(q1, F1a, fma(h, va, xa)))));
    vni = fma(b6, F6i, fma(b5, F5i, fma(b4, F4i, fma(b3, F3i, fma(b1, F1i, vi)))));
    vna = fma(b6, F6a, fma(b5, F5a, fma(b4, F4a, fma(b3, F3a, fma(b1, F1a, va)))));
    exi = fma(p6, F6i, fma(p5, F5i, fma(p4, F4i, fma(p3, F3i, p1 * F1i))));
    exa = fma(p6, F6a, fma(p5, F5a, fma(p4, F4a, fma(p3, F3a, p1 * F1a))));
    evi = fma(E6, F6i, fma(E5, F5i, fma(E4, F4i, fma(E3, F3i, E1 * F1i))));
    eva = fma(E6, F6a, fma(E5, F5a, fma(E4, F4a, fma(E3, F3a, E1 * F1a))));
  }
  // error norm as in half_norm(): this axis's ion and atom ratios on this
  // lane, the axes across the quad
  double mx = vmax(ratio(exi, max_abs(max_abs(xi, xni), K.thr)),
                   ratio(exa, max_abs(max_abs(xa, xna), K.thr)));
  {
    const double my = from_quad_lane<1>(mx), mz = from_quad_lane<2>(mx);
    mx = vmax(vmax(from_quad_lane<0>(mx), my), mz);
  }

  const double cos7 = L.done ? cos_rf(K.omega * tnew) : cs6;
  const double r2n = accel_wide(P, ka, kq, cos7, xni, xna, F7i, F7a, dx, dy, dz);

  const double e7i = fma(E7, F7i, evi), e7a = fma(E7, F7a, eva);
  // the velocity half as in with_velocity_half(): skipped when each axis's
  // bound max(|e|) vbound is at most mx (decided per quad, so that the quad's
  // lanes stay together for the exchanges below)
  int need_v = !(max_abs(e7i, e7a) * K.vbound <= mx);
  need_v = from_quad_lane<0>(need_v) | from_quad_lane<1>(need_v) | from_quad_lane<2>(need_v);
  double m = mx;
  if (need_v) {
    double mv = vmax(ratio(e7i, max_abs(max_abs(vi, vni), K.thr)),
                     ratio(e7a, max_abs(max_abs(va, vna), K.thr)));
    const double my = from_quad_lane<1>(mv), mz = from_quad_lane<2>(mv);
    mv = vmax(vmax(from_quad_lane<0>(mv), my), mz);
    m = vmax(mx, mv);
  }
  const double err = h * m;

  conclude(
      K, L, t, h, tnew, err, cs6, sn6, r2n,
      [&] {
        move_into(L.xi, xni);
        move_into(L.xa, xna);
        move_into(L.vi, vni);
        move_into(L.va, vna);
        move_into(L.Fi, F7i);
        move_into(L.Fa, F7a);
      },
      [&] {
        const double dv = vni - vna;
        const double dvx = from_quad_lane<0>(dv), dvy = from_quad_lane<1>(dv),
                     dvz = from_quad_lane<2>(dv);
        return fma(dz, dvz, fma(dy, dvy, dx * dvx));
      },
      [&] {
        const double x0 = from_quad_lane<0>(xni), x1 = from_quad_lane<1>(xni),
                     x2 = from_quad_lane<2>(xni);
        return sqrt(fma(x2, x2, fma(x1, x1, x0 * x0)));
      });
}

// Trajectory idx by the four lanes of a quad; this lane holds axis ax and, if
// it is the quad's lane q < 3, stores that axis's final state (q = 0 also the
// observables, with DERIVE the derived ones as finish_derived forms them).
// The start is the one-lane start on every lane.
template <class F, bool DERIVE = false>
__device__ __forceinline__ void integrate_wide(const Launch& P, long long idx, int q) {
  const int ax = q < 3 ? q : 2;
  const Ctl K = lane_ctl(P);
  const F Fc = lane_force_of(P, (const F*)nullptr);
  double y[12];
  load_column(P, idx, y);
  WideLane W;
  {
    Lane L;
    start(Fc, start_const(P), y, L);
    W.xi = axis_value(ax, L.x[0], L.x[1], L.x[2]);
    W.xa = axis_value(ax, L.x[3], L.x[4], L.x[5]);
    W.vi = axis_value(ax, L.v[0], L.v[1], L.v[2]);
    W.va = axis_value(ax, L.v[3], L.v[4], L.v[5]);
    W.Fi = axis_value(ax, L.F1[0], L.F1[1], L.F1[2]);
    W.Fa = axis_value(ax, L.F1[3], L.F1[4], L.F1[5]);
    W.t = L.t;
    W.absh = L.absh;
    W.cph = L.cph;
    W.sph = L.sph;
    W.w_prev = L.w_prev;
    W.t_first = L.t_first;
    W.t_last = L.t_last;
    W.position = L.position;
    W.rmin2 = L.rmin2;
    W.nfailed = L.nfailed;
    W.nsteps = L.nsteps;
    W.bounces = L.bounces;
    W.status = L.status;
    W.done = L.done;
    W.nofailed = L.nofailed;
    W.fresh = L.fresh;
    W.approached = L.approached;
  }
  const double ka = in_vgpr(axis_value(ax, Fc.ka[0], Fc.ka[1], Fc.ka[2]));
  const double kq = in_vgpr(axis_value(ax, Fc.kq[0], Fc.kq[1], Fc.kq[2]));
  while (W.status == 0) {
    if (W.fresh) begin_step(K, W);
    attempt_wide(Fc, ka, kq, K, W);
  }
  // the initial atom velocity y[9..11] was read before final_state (possibly
  // y0) is written
  const long long ld = P.ld;
  if (q < 3) {
    P.yf[ax * ld + idx] = W.xi;
    P.yf[(3 + ax) * ld + idx] = W.vi;
    P.yf[(6 + ax) * ld + idx] = W.xa;
    P.yf[(9 + ax) * ld + idx] = W.va;
  }
  // DERIVE: lane q = 0 gathers the other axes' final values from lanes 1
  // and 2 of its quad and forms the derived observables (as finish_derived)
  double vi[3], va[3], d[3];
  if constexpr (DERIVE) {
    const double dq = W.xi - W.xa;
    vi[0] = from_quad_lane<0>(W.vi);
    vi[1] = from_quad_lane<1>(W.vi);
    vi[2] = from_quad_lane<2>(W.vi);
    va[0] = from_quad_lane<0>(W.va);
    va[1] = from_quad_lane<1>(W.va);
    va[2] = from_quad_lane<2>(W.va);
    d[0] = from_quad_lane<0>(dq);
    d[1] = from_quad_lane<1>(dq);
    d[2] = from_quad_lane<2>(dq);
  }
  if (q == 0) {
    double o[AI_NOBS];
    o[AI_OBS_TEND] = W.t;
    o[AI_OBS_STATUS] = (double)W.status;
    o[AI_OBS_NSTEPS] = (double)W.nsteps;
    o[AI_OBS_NFAILED] = (double)W.nfailed;
    o[AI_OBS_BOUNCES] = (double)W.bounces;
    o[AI_OBS_LIFETIME] = W.t_first;
    o[AI_OBS_ANGLE] = W.t_last;
    o[AI_OBS_TRANSFER] = y[9];
    o[AI_OBS_POSITION] = W.position;
    o[AI_OBS_DIST] = y[10];
    o[AI_OBS_KE] = y[11];
    o[AI_OBS_RMIN] = W.rmin2;
    o[AI_OBS_HNEXT] = W.absh;
    if constexpr (DERIVE) {
      const Derived dv = derive_from(W.t_first, W.t_last, y[9], y[10], y[11], W.rmin2,
                                       (double)W.bounces, vi[0], vi[1], vi[2], va[0], va[1], va[2],
                                       d[0], d[1], d[2], P.m_atom, P.half_mi);
      o[AI_OBS_LIFETIME] = dv.lifetime;
      o[AI_OBS_ANGLE] = dv.angle;
      o[AI_OBS_TRANSFER] = dv.transfer;
      o[AI_OBS_DIST] = dv.dist;
      o[AI_OBS_KE] = dv.ke;
      o[AI_OBS_RMIN] = dv.rmin;
    }
#pragma unroll
    for (int c = 0; c < AI_NOBS; ++c) P.obs[c * ld + idx] = o[c];
  }
}

// With the schedule's keys a wave takes the priority of its first (longest)
// trajectory, the one at schedule position first.
__device__ __forceinline__ void wave_priority_from_keys(const unsigned* key, long long first) {
  if (key) {
    const float top = (float)key[0], mine = (float)key[first];
    set_wave_priority(wave_uniform(top > 0.0f ? mine / top : 0.0f));
  }
}

// The plain kernels' grid: P.wide_waves waves of WAVE/4 trajectories each
// (schedule positions 0 .. P.wide - 1, four lanes per trajectory), then one
// trajectory per lane for positions P.wide .. n - 1.  Position g holds
// trajectory order[g] (g itself without a schedule).
template <class R, class F = Force>
__device__ __forceinline__ void plain_body(const Launch& P) {
  const long long w = blockIdx.x;
  if constexpr (sizeof(R) == sizeof(double)) {
    if (w < P.wide_waves) {
      const long long first = w * (WAVE / 4);
      wave_priority_from_keys(P.key, first);
      const long long g = first + (threadIdx.x >> 2);
      if (g >= P.wide) return;
      integrate_wide<F, true>(P, (long long)P.order[g], (int)(threadIdx.x & 3));
      return;
    }
  }
  const long long first = P.wide + (w - P.wide_waves) * BLOCK;
  wave_priority_from_keys(P.key, first);
  const long long g = first + threadIdx.x;
  if (g >= P.n) return;
  integrate_one<R, F, true>(P, P.order ? (long long)P.order[g] : g);
}

__global__ __launch_bounds__(BLOCK) void ai_plain_kernel(Launch P) { plain_body<double>(P); }

// The same with single-precision stages (AI_FP32_STAGES).
__global__ __launch_bounds__(BLOCK) void ai_plain32_kernel(Launch P) { plain_body<float>(P); }

// One trajectory (the lane 0 of one wave) with the ensemble kernels' attempt,
// recording (t, y) at t0 and at `refine` points per accepted step, the last at
// the step's end: point k at t_out[k] and y_out[c * cap + k], for the first
// cap points.  Points inside a step come from the quintic Hermite interpolant
// of the positions through (x, v, a) at both ends of the step (a = the
// first-same-as-last accelerations), velocities from its derivative.  Initial
// state y0[c], final state yf[c] and observables obs[c] are 12 and AI_NOBS
// consecutive doubles (P.ld = 1).
template <class F>
__device__ __forceinline__ void trace_body(const Launch& P, int refine, long long cap,
                                           double* t_out, double* y_out) {
  if (threadIdx.x != 0) return;
  const Ctl K = lane_ctl(P);
  const F Fc = lane_force_of(P, (const F*)nullptr);
  Lane L;
  double y[12];
  load_column(P, 0, y);
  start(Fc, start_const(P), y, L);
  long long k = 0;
  auto store = [&](double t, const double* x, const double* v) {
    if (k < cap) {
      t_out[k] = t;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        y_out[c * cap + k] = x[c];            // x_ion
        y_out[(3 + c) * cap + k] = v[c];      // v_ion
        y_out[(6 + c) * cap + k] = x[3 + c];  // x_atom
        y_out[(9 + c) * cap + k] = v[3 + c];  // v_atom
      }
    }
    ++k;
  };
  store(L.t, L.x, L.v);
  double t0 = L.t, x0[6], v0[6], a0[6];
  auto keep = [&]() {
    t0 = L.t;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      x0[c] = L.x[c];
      v0[c] = L.v[c];
      a0[c] = L.F1[c];
    }
  };
  keep();
  int seen = 0;
  while (L.status == 0) {
    if (L.fresh) begin_step(K, L);
    attempt(Fc, K, L);
    if (L.nsteps != seen) {
      seen = L.nsteps;
      const double h = L.t - t0;
      for (int j = 1; j < refine; ++j) {
        const double u = (double)j / refine, u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
        const double h0 = 1.0 - 10.0 * u3 + 15.0 * u4 - 6.0 * u5, h3 = 1.0 - h0;
        const double h1 = u - 6.0 * u3 + 8.0 * u4 - 3.0 * u5;
        const double h2 = 0.5 * (u2 - 3.0 * u3 + 3.0 * u4 - u5);
        const double h4 = -4.0 * u3 + 7.0 * u4 - 3.0 * u5;
        const double h5 = 0.5 * (u3 - 2.0 * u4 + u5);
        const double d0 = -30.0 * u2 + 60.0 * u3 - 30.0 * u4;  // derivatives in u
        const double d1 = 1.0 - 18.0 * u2 + 32.0 * u3 - 15.0 * u4;
        const double d2 = u - 4.5 * u2 + 6.0 * u3 - 2.5 * u4;
        const double d4 = -12.0 * u2 + 28.0 * u3 - 15.0 * u4;
        const double d5 = 1.5 * u2 - 4.0 * u3 + 2.5 * u4;
        double xi[6], vi[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double dx = L.x[c] - x0[c];
          xi[c] = x0[c] + h3 * dx + h * (h1 * v0[c] + h4 * L.v[c]) +
                  h * h * (h2 * a0[c] + h5 * L.F1[c]);
          vi[c] = (-d0) * dx / h + d1 * v0[c] + d4 * L.v[c] + h * (d2 * a0[c] + d5 * L.F1[c]);
        }
        store(t0 + u * h, xi, vi);
      }
      store(L.t, L.x, L.v);
      keep();
    }
  }
  finish(P.yf, P.obs, 1, L, 0, y[9], y[10], y[11]);
}

__global__ __launch_bounds__(BLOCK) void ai_trace_kernel(Launch P, int refine, long long cap,
                                                         double* t_out, double* y_out) {
  trace_body<Force>(P, refine, cap, t_out, y_out);
}

__global__ __launch_bounds__(BLOCK) void ai_trace_nm_kernel(Launch P, int refine, long long cap,
                                                            double* t_out, double* y_out) {
  trace_body<ForceNM>(P, refine, cap, t_out, y_out);
}

// The same for potentials with exponents other than n = 4, m = 8.
__global__ __launch_bounds__(BLOCK) void ai_plain_nm_kernel(Launch P) {
  plain_body<double, ForceNM>(P);
}

// A batch of ensembles in one index space: lane g integrates global index
// order[g] (g without a schedule) of the ensemble that holds it, with that
// ensemble's constants, buffers and tolerances.
// The grid is laid out as the plain kernel's: B.wide_waves waves of four-lane
// trajectories (positions 0 .. B.wide - 1 of the order), then one trajectory
// per lane; as there, the derived observables are formed at each
// trajectory's end.
__global__ __launch_bounds__(BLOCK) void ai_plain_batch_kernel(BatchLaunch B) {
  const long long w = blockIdx.x;
  if (w < B.wide_waves) {
    const long long first = w * (WAVE / 4);
    wave_priority_from_keys(B.key, first);
    const long long g = first + (threadIdx.x >> 2);
    if (g >= B.wide) return;
    const long long j = (long long)B.order[g];
    const BatchEntry& E = B.entries[batch_entry(B.entries, B.count, j)];
    integrate_wide<Force, true>(E.P, j - E.offset, (int)(threadIdx.x & 3));
    return;
  }
  const long long first = B.wide + (w - B.wide_waves) * BLOCK;
  wave_priority_from_keys(B.key, first);
  const long long g = first + threadIdx.x;
  if (g >= B.total) return;
  const long long j = B.order ? (long long)B.order[g] : g;
  const BatchEntry& E = B.entries[batch_entry(B.entries, B.count, j)];
  integrate_one<double, Force, true>(E.P, j - E.offset);
}

__global__ void ai_queue_reset_kernel(unsigned long long* queue) { *queue = 0ull; }

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Positions a wave claims from the queue at a time, and near the queue's end
// (when fewer than TAIL_ROUNDS chunks per wave remain), so that no wave holds
// much unstarted work while others run dry.
constexpr int CHUNK = 32;
constexpr int CHUNK_TAIL = 8;
constexpr int TAIL_ROUNDS = 8;

// Resident waves.  Positions below P.first_dynamic are assigned statically
// (lane g of the grid starts position g); the rest are claimed from the device
// queue in chunks: one atomic per chunk, and the chunk's initial states are
// loaded into LDS at once.  Lanes whose trajectory has ended take staged
// entries from LDS, so a refill waits on memory once per chunk rather than on
// three dependent round trips (queue, schedule, y0) per trajectory.  Position
// p is trajectory order[p] (p itself when order is null).  Each outer
// iteration: busy lanes make attempts until enough lanes are free, ended
// trajectories are stored, and free lanes start staged trajectories.
__global__ __launch_bounds__(BLOCK, 2) void ai_persistent_kernel(Launch P) {
  // the leading positions of a longest-first order: four lanes per
  // trajectory, as in the plain kernel (these waves then leave)
  if ((long long)blockIdx.x < P.wide_waves) {
    const long long first = (long long)blockIdx.x * (WAVE / 4);
    wave_priority_from_keys(P.key, first);
    const long long g = first + (threadIdx.x >> 2);
    if (g < P.wide) integrate_wide<Force>(P, (long long)P.order[g], (int)(threadIdx.x & 3));
    return;
  }
  __shared__ double stage_y[12][WAVE];  // staged initial states, component-major
  __shared__ long long stage_idx[WAVE];
  __shared__ float stage_key[WAVE];
  __shared__ double lane_va0[3][WAVE];  // each lane's initial atom velocity
  // The launch fields and start constants the refill, start and store code
  // uses, read from LDS where used (through an opaque pointer, so the loads
  // stay there) instead of being held in scalar registers across the
  // attempt loop, where they would be spilled to vector-register lanes.
  __shared__ Launch lds_P;
  __shared__ StartConst lds_S;
  const int lane = (int)threadIdx.x;    // BLOCK == WAVE: one wave per workgroup
  if (lane == 0) {
    lds_P = P;
    lds_S = start_const(P);
  }
  __syncthreads();
  const float top = P.key ? (float)P.key[0] : 0.0f;
  const int refill_min = in_vgpr(P.refill_min);
  const Ctl K = lane_ctl(P);
  const Force Fc = lane_force(P);
  Lane L;
  // statically assigned: the positions after the four-lane ones, a wave's worth each
  const long long static_first = P.wide + ((long long)blockIdx.x - P.wide_waves) * BLOCK;
  long long idx = static_first + lane;
  int busy = 0;                             // integrating, or ended and not yet stored
  bool critical = false;                    // wave-uniform
  bool drained = P.first_dynamic >= P.n;    // wave-uniform: no more claims succeed
  long long front = P.first_dynamic;        // wave-uniform: queue front as last seen
  int avail = 0, head = 0;                  // wave-uniform: staged entries, next to take

  using LdsLaunch = const __attribute__((address_space(3))) Launch*;
  using LdsStart = const __attribute__((address_space(3))) StartConst*;
  auto launch = [&]() {
    LdsLaunch q = (LdsLaunch)&lds_P;
    asm volatile("" : "+v"(q));
    return q;
  };
  auto begin = [&](const double* y) {
    lane_va0[0][lane] = y[9];
    lane_va0[1][lane] = y[10];
    lane_va0[2][lane] = y[11];
    LdsStart q = (LdsStart)&lds_S;
    asm volatile("" : "+v"(q));
    StartConst S;
    S.t0 = q->t0;
    S.cph0 = q->cph0;
    S.sph0 = q->sph0;
    S.hcap = q->hcap;
    S.hmin0 = q->hmin0;
    S.thr = q->thr;
    S.inv_hinit = q->inv_hinit;
    start(Fc, S, y, L);
    busy = 1;
  };
  // priority from the wave's longest predicted trajectory (as a fraction of
  // the longest overall); a wave holding one predicted to last at least half
  // as long carries the critical path and refills only once all its lanes are
  // free.  Positions are handed out in decreasing order of predicted
  // duration, so the wave's first position is its longest, and after a
  // critical wave drains, the first of its new ones is.
  auto set_priority = [&](float k) {
    const float frac = top > 0.0f ? k / top : 0.0f;
    set_wave_priority(frac);
    critical = frac >= 0.5f;
  };

  if (P.key) set_priority(P.key[static_first]);  // the grid never exceeds the positions
  if (idx < P.n) {
    idx = P.order ? (long long)P.order[idx] : idx;
    double y[12];
    load_column(P, idx, y);
    begin(y);
  }

  for (;;) {
    // integrate until enough lanes are free for a refill: refill_min of them
    // (idle lanes included), or all of them once nothing is left to start or
    // while the wave is critical.  Ended lanes wait, frozen, for their store.
    for (;;) {
      if (busy && L.status == 0) {
        if (L.fresh) begin_step(K, L);
        attempt(Fc, K, L);
      }
      const unsigned long long live = __ballot(busy && L.status == 0);
      if (live == 0ull) break;
      if ((!drained || head < avail) && !critical && __popcll(~live) >= refill_min) break;
    }
    if (busy && L.status != 0) {
      const LdsLaunch Q = launch();
      finish(Q->yf, Q->obs, Q->ld, L, idx, lane_va0[0][lane], lane_va0[1][lane], lane_va0[2][lane]);
      busy = 0;
    }
    const bool was_drained = __ballot(busy) == 0ull;
    float first_key = -1.0f;  // key of the first entry taken
    // free lanes take staged entries; a new chunk is claimed when none are left
    for (;;) {
      const unsigned long long idle = __ballot(!busy);
      if (idle == 0ull) break;
      if (head >= avail) {
        if (drained) break;
        const LdsLaunch Q = launch();
        const long long n = Q->n;
        const long long left = n - front;
        const int want =
            left > (long long)CHUNK * TAIL_ROUNDS * (long long)gridDim.x ? CHUNK : CHUNK_TAIL;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(Q->queue, (unsigned long long)want);
        base = __shfl(base, 0, WAVE);
        const long long first = Q->first_dynamic + (long long)base;
        long long cnt = n - first;
        cnt = cnt < 0 ? 0 : (cnt > want ? want : cnt);
        front = first + want;
        if (front >= n) drained = true;
        __syncthreads();  // earlier reads of the staging area are complete
        if (lane < cnt) {
          const long long pos = first + lane;
          const unsigned* order = Q->order;
          const unsigned* key = Q->key;
          const double* y0 = Q->y0;
          const long long ld = Q->ld;
          const long long t = order ? (long long)order[pos] : pos;
          stage_idx[lane] = t;
          stage_key[lane] = key ? (float)key[pos] : 0.0f;
#pragma unroll
          for (int c = 0; c < 12; ++c) stage_y[c][lane] = y0[c * ld + t];
        }
        __syncthreads();  // staged entries visible to every lane
        avail = (int)cnt;
        head = 0;
        if (avail == 0) break;
      }
      if (first_key < 0.0f) first_key = stage_key[head];
      const int e = head + (int)lanes_below(idle);
      if (!busy && e < avail) {
        idx = stage_idx[e];
        double y[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = stage_y[c][e];
        begin(y);
      }
      const int took = __popcll(idle);
      head = head + took < avail ? head + took : avail;
    }
    if (__ballot(busy) == 0ull) break;  // nothing running and nothing left to start
    if (critical && was_drained && first_key >= 0.0f) set_priority(first_key);
  }
}

// ---- Resident serving kernel ----
//
// Waves that stay resident while a server publishes requests (see internal.h
// for the protocol).  Lanes of one wave may hold trajectories of different
// requests: every lane keeps its request's loop constants in its own
// registers, its output addresses in LDS, and takes the double or the
// single-precision-stage attempt as its request asks (the single-precision
// variant's per-lane choice of integrate_one), so each trajectory's result is
// bitwise what ai_integrate gives for its request alone.  A wave claims
// trajectories of the oldest request with work left when enough of its lanes
// are free, stores each finished trajectory's final state and observables
// with stores written through to memory, then adds the finished count of each
// request to its slot's counter; the add that reaches a request's target
// signals its completion to the host.  Idle waves poll for new requests and
// exit once the host asks them to stop or they have been idle for
// idle_ticks.  Every trajectory ends (step cap, step floor, non-finite
// check) and claims only succeed for published work, so every wave exits
// once the host stops publishing.

struct ResidentDesc {
  Launch P;        // the request's constants; y0, yf, obs planes in the slab
  long long seq;   // request number
  long long target;  // done count of its ring slot once the request has completed
  int fp32;        // single-precision stages
};
static_assert(sizeof(ResidentDesc) <= sizeof(ai_resident_desc), "resident descriptor size");
constexpr int RES_DESC_WORDS = (int)((sizeof(ResidentDesc) + 7) / 8);
static_assert(RES_DESC_WORDS <= WAVE, "one word per lane");
constexpr int RES_BACKOFF = 64;
// Trajectories a wave claims at a time (fewer at a request's end); it keeps
// the unstarted ones of a claim and hands them to its lanes as they free up,
// so the claim word sees one compare-and-swap per chunk.
constexpr int RES_CHUNK = 32;
// How far past the oldest request with work left a wave looks for a request
// of its own precision, and how many of its lanes must be running for it to
// look only for that precision (see claim()).
constexpr int RES_CLASS_WINDOW = 16;
constexpr int RES_CLASS_KEEP = 32;
static_assert(offsetof(ResidentDesc, fp32) % 8 == 0, "precision flag in a word of its own");

__device__ __forceinline__ unsigned long long load_system(const uint64_t* p) {
  return __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

// A store that is written through to memory (system scope), so the server's
// copy engine reads it once the store has completed.
__device__ __forceinline__ void store_through(double* p, double v) {
  __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A load that is not served from a stale cache line (system scope): the slab's
// initial states were written by a copy engine, possibly over lines an earlier
// request left in this die's L2.
__device__ __forceinline__ double load_through(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      (const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
}

// Wait until this wave's memory operations have completed: its stores written
// through above are then in memory.  (A release or acquire fence at system or
// device scope would write back or invalidate the whole L2 of the die, at every
// finished trajectory and every claim; the kernel needs neither, since the data
// it shares bypasses the L2 both ways.)
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ Force32 force32_of(const Force& F) {
  Force32 f;
  f.mr = (float)F.mr;
  f.nCa = (float)F.nCa;
  f.mCa = (float)F.mCa;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f.ka[k] = (float)F.ka[k];
    f.kq[k] = (float)F.kq[k];
  }
  return f;
}

// The leader lane's claim: up to `want` trajectories of the oldest published
// request with work left, as (request, first index, count); false if there is
// none.  Each ring slot has a claim counter packing (request << 32 | claimed),
// which the host sets to (request << 32) when it publishes the request there;
// a claim is one fetch-and-add of `want` on the counter of the request the
// current-request word names, so claims never retry against each other.  The
// counter's old value says which request the trajectories belong to (and so
// which descriptor: the ring slot's, copied before the counter was set) and
// whether any were left; a claim that finds a request exhausted moves the
// current-request word on (one compare-and-swap, if the next request is
// published) and tries again.  Counts past a request's size are claims of
// nothing; a claim looks at the counter before adding to it, so only claims
// racing at a request's end add past its size.  n_of(seq) gives a request's
// size.  Bounded: gives up after a few rounds (and is retried later).
//
// Precision: a lane runs the double or the single-precision-stage attempt as
// its request asks, so a wave holding lanes of both kinds issues both every
// iteration.  A wave with at least RES_CLASS_KEEP lanes running requests of
// one kind (cls: 0 double, 1 single-precision stages; -1 for any other wave)
// therefore claims only requests of that kind: when the oldest request with
// work left is of the other kind it takes the next one of its own kind within
// RES_CLASS_WINDOW requests (claim_ahead), or nothing.  A wave with fewer
// running lanes (one kept alive by a few long trajectories, say) takes the
// oldest request whatever its kind, so mixing costs a wave at most half its
// issue slots and the oldest request always has waves that take it.
// cls_of(seq) gives a request's kind.
template <class SizeOf, class ClassOf>
__device__ bool claim_ahead(const ai_resident_args& A, int want, int cls, unsigned long long s,
                            unsigned long long pub, long long& seq, long long& first, int& count,
                            SizeOf n_of, ClassOf cls_of) {
  const unsigned long long reach =
      (unsigned long long)(RES_CLASS_WINDOW < A.ring - 1 ? RES_CLASS_WINDOW : A.ring - 1);
  const unsigned long long end = s + 1 + reach < pub ? s + 1 + reach : pub;
  for (unsigned long long t = s + 1; t < end; ++t) {
    unsigned long long* counter = (unsigned long long*)A.claimed + t % (unsigned long long)A.ring;
    const unsigned long long seen =
        __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the slot holds request t (its descriptor was copied before its counter
    // was set), of this kind, with trajectories left
    if ((long long)(seen >> 32) != (long long)t || cls_of((long long)t) != cls) continue;
    const long long n = n_of((long long)t);
    if ((long long)(seen & 0xffffffffull) >= n) continue;
    const unsigned long long v = __hip_atomic_fetch_add(counter, (unsigned long long)want,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long sv = (long long)(v >> 32), k = (long long)(v & 0xffffffffull);
    if (sv == (long long)t && k < n) {
      seq = sv;
      first = k;
      count = (int)(n - k < want ? n - k : want);
      return true;
    }
  }
  return false;
}

template <class SizeOf, class ClassOf>
__device__ bool claim(const ai_resident_args& A, int want, int cls, long long& seq,
                      long long& first, int& count, SizeOf n_of, ClassOf cls_of) {
  for (int tries = 0; tries < 8; ++tries) {
    const unsigned long long pub = load_system(A.pub);
    unsigned long long s =
        __hip_atomic_load((unsigned long long*)A.cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s >= pub) return false;
    unsigned long long* counter =
        (unsigned long long*)A.claimed + s % (unsigned long long)A.ring;
    // a look first: idle waves polling an exhausted request must not keep
    // adding to its counter (2,000 waves adding 32 every look would carry the
    // 32-bit claimed count into the request number within seconds, and the
    // counter would then name a request it does not hold)
    const unsigned long long seen =
        __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((long long)(seen >> 32) == (long long)s &&
        (long long)(seen & 0xffffffffull) >= n_of((long long)s)) {
      if (s + 1 < pub) {
        __hip_atomic_compare_exchange_strong((unsigned long long*)A.cur, &s, s + 1,
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        continue;
      }
      return false;
    }
    if (cls >= 0 && (long long)(seen >> 32) == (long long)s && cls_of((long long)s) != cls)
      return claim_ahead(A, want, cls, s, pub, seq, first, count, n_of, cls_of);
    const unsigned long long v = __hip_atomic_fetch_add(counter, (unsigned long long)want,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long sv = (long long)(v >> 32), k = (long long)(v & 0xffffffffull);
    if (sv < (long long)s) return false;  // the slot not yet set for s (cannot happen)
    const long long n = n_of(sv);
    if (k < n) {
      seq = sv;
      first = k;
      count = (int)(n - k < want ? n - k : want);
      return true;
    }
    // the request is exhausted (or its slot already holds a later one):
    // move the current-request word past it
    if (s + 1 < pub)
      __hip_atomic_compare_exchange_strong((unsigned long long*)A.cur, &s, s + 1,
                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    else
      return false;
  }
  return false;
}

__global__ __launch_bounds__(BLOCK, 2) void ai_resident_kernel(ai_resident_args A) {
  __shared__ ResidentDesc lds_desc;     // descriptor of the request claimed last
  __shared__ StartConst lds_S;
  __shared__ double* lane_yf[WAVE];
  __shared__ double* lane_obs[WAVE];
  __shared__ long long lane_ld[WAVE], lane_idx[WAVE], lane_seq[WAVE], lane_target[WAVE];
  __shared__ int lane_slot[WAVE];
  __shared__ double lane_va0[3][WAVE], lane_m_atom[WAVE], lane_half_mi[WAVE];
  __shared__ long long claim_info[3];   // leader's claim broadcast: seq, first, count
  // each lane's loop and force constants (its request's), read from LDS at
  // every attempt rather than held in registers across the loop: they would
  // add ~40 registers to the ones the loop carries, which the rare start and
  // store paths then push into scratch
  __shared__ Ctl lane_K[WAVE];
  __shared__ Force lane_F[WAVE];
  __shared__ double lane_near2[WAVE];
  const int lane = (int)threadIdx.x;    // BLOCK == WAVE
  using LdsCtl = __attribute__((address_space(3))) Ctl*;
  using LdsForce = __attribute__((address_space(3))) Force*;
  using LdsDouble = __attribute__((address_space(3))) double*;
  Lane L;
  int busy = 0;
  long long cur_seq = -1;               // wave-uniform: request in lds_desc
  long long cur_n = 0;
  long long st_next = 0, st_end = 0;    // wave-uniform: claimed, unstarted positions of cur_seq
  unsigned long long idle_since = 0;
  bool idle = false;
  int backoff = 0;                      // attempts before the next claim
  int wave_cls = -1;                    // wave-uniform: kind of the running lanes' requests
  const int refill_min = A.refill_min;

  for (;;) {
    // integrate until enough lanes are free to refill (a wave with nothing
    // left to run leaves at once); ended lanes wait, frozen, for their store
    // (after a claim found nothing, wait RES_BACKOFF attempts before asking
    // again)
    int since = 0;
    for (;;) {
      if (busy && L.status == 0) {
        // opaque addresses: the loads stay inside the loop
        LdsCtl kp = (LdsCtl)&lane_K[lane];
        LdsForce fp = (LdsForce)&lane_F[lane];
        LdsDouble np = (LdsDouble)&lane_near2[lane];
        asm volatile("" : "+v"(kp), "+v"(fp), "+v"(np));
        Ctl K;
        K.tf = kp->tf;
        K.hmax = kp->hmax;
        K.rtol = kp->rtol;
        K.inv_rtol = kp->inv_rtol;
        K.thr = kp->thr;
        K.vbound = kp->vbound;
        K.r_exit2 = kp->r_exit2;
        K.r_bounce2 = kp->r_bounce2;
        K.omega = kp->omega;
        K.max_steps = kp->max_steps;
        K.exit_on = kp->exit_on;
        Force F;
        F.mr = fp->mr;
        F.nCa = fp->nCa;
        F.mCa = fp->mCa;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          F.ka[k] = fp->ka[k];
          F.kq[k] = fp->kq[k];
        }
        if (L.fresh) begin_step(K, L);
        const double dx = L.x[0] - L.x[3], dy = L.x[1] - L.x[4], dz = L.x[2] - L.x[5];
        if (fma(dz, dz, fma(dy, dy, dx * dx)) < *np)
          attempt(F, K, L);
        else
          attempt32(force32_of(F), K, L);
      }
      const unsigned long long live = __ballot(busy && L.status == 0);
      if (live == 0ull) break;
      ++since;
      const int free_lanes = __popcll(~live);
      if (free_lanes > 0 && since >= backoff && (free_lanes >= refill_min || since >= RES_BACKOFF))
        break;
    }

    // store ended trajectories, then count them per request
    const unsigned long long ended = __ballot(busy && L.status != 0);
    if (ended) {
      if (busy && L.status != 0) {
        double* yf = lane_yf[lane];
        double* ob = lane_obs[lane];
        const long long ld = lane_ld[lane], i = lane_idx[lane];
        double y[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          y[k] = L.x[k];
          y[3 + k] = L.v[k];
          y[6 + k] = L.x[3 + k];
          y[9 + k] = L.v[3 + k];
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) store_through(yf + c * ld + i, y[c]);
        const double bounces = (double)L.bounces;
        const Derived d = derive_at_end(
            L.t_first, L.t_last, lane_va0[0][lane], lane_va0[1][lane], lane_va0[2][lane], L.rmin2,
            bounces, y[3], y[4], y[5], y[9], y[10], y[11], y[0] - y[6], y[1] - y[7], y[2] - y[8],
            lane_m_atom[lane], lane_half_mi[lane]);
        store_through(ob + AI_OBS_TEND * ld + i, L.t);
        store_through(ob + AI_OBS_STATUS * ld + i, (double)L.status);
        store_through(ob + AI_OBS_NSTEPS * ld + i, (double)L.nsteps);
        store_through(ob + AI_OBS_NFAILED * ld + i, (double)L.nfailed);
        store_through(ob + AI_OBS_BOUNCES * ld + i, bounces);
        store_through(ob + AI_OBS_LIFETIME * ld + i, d.lifetime);
        store_through(ob + AI_OBS_ANGLE * ld + i, d.angle);
        store_through(ob + AI_OBS_TRANSFER * ld + i, d.transfer);
        store_through(ob + AI_OBS_POSITION * ld + i, L.position);
        store_through(ob + AI_OBS_DIST * ld + i, d.dist);
        store_through(ob + AI_OBS_KE * ld + i, d.ke);
        store_through(ob + AI_OBS_RMIN * ld + i, d.rmin);
        store_through(ob + AI_OBS_HNEXT * ld + i, L.absh);
      }
      // the stores above are in memory before any count that includes them
      wait_memory();
      unsigned long long todo = ended;
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int slot = __shfl(lane_slot[lane], leader, WAVE);
        const unsigned long long group = __ballot(((todo >> lane) & 1ull) && lane_slot[lane] == slot);
        if (lane == leader) {
          const unsigned long long k = (unsigned long long)__popcll(group);
          const unsigned long long before = __hip_atomic_fetch_add(
              (unsigned long long*)A.done_cnt + slot, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          if (before + k == (unsigned long long)lane_target[lane])
            __hip_atomic_store((unsigned long long*)A.done_seq + slot,
                               (unsigned long long)lane_seq[lane] + 1ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
        todo &= ~group;
      }
      if (busy && L.status != 0) busy = 0;
    }

    // free lanes take trajectories of the oldest request with work left
    bool claimed_any = false;
    for (;;) {
      const unsigned long long freel = __ballot(!busy);
      if (freel == 0ull) break;
      if (st_next >= st_end) {
        const int cls = __popcll(__ballot(busy)) >= RES_CLASS_KEEP ? wave_cls : -1;
        if (lane == 0) {
          long long seq = -1, first = 0;
          int count = 0;
          const bool got = claim(
              A, RES_CHUNK, cls, seq, first, count,
              [&](long long s) {
                if (s == cur_seq) return cur_n;
                const ResidentDesc* d = (const ResidentDesc*)&A.desc[s % A.ring];
                return (long long)load_system((const uint64_t*)&d->P.n);
              },
              [&](long long s) {
                const ResidentDesc* d = (const ResidentDesc*)&A.desc[s % A.ring];
                return (load_system((const uint64_t*)&d->fp32) & 0xffffffffull) != 0ull ? 1 : 0;
              });
          claim_info[0] = got ? seq : -1;
          claim_info[1] = first;
          claim_info[2] = count;
        }
        __syncthreads();
        // the request's initial states, copied into the slab before it was
        // published, are read below with loads that bypass stale cache lines
        const long long seq = claim_info[0], first = claim_info[1];
        const int count = (int)claim_info[2];
        __syncthreads();
        if (seq < 0) {
          backoff = RES_BACKOFF;
          break;
        }
        backoff = 0;
        claimed_any = true;
        if (seq != cur_seq) {
          // the request's descriptor, one word per lane, from the device ring
          const uint64_t* src = A.desc[seq % A.ring].w;
          if (lane < RES_DESC_WORDS) ((unsigned long long*)&lds_desc)[lane] = load_system(src + lane);
          __syncthreads();
          if (lane == 0) lds_S = start_const(lds_desc.P);
          __syncthreads();
          cur_seq = seq;
          cur_n = lds_desc.P.n;
        }
        wave_cls = lds_desc.fp32 ? 1 : 0;
        st_next = first;
        st_end = first + count;
      }
      const long long seq = cur_seq;
      const long long first = st_next;
      const long long count = st_end - st_next;
      st_next += __popcll(freel) < count ? __popcll(freel) : count;
      const int e = (int)lanes_below(freel);
      if (!busy && e < count) {
        const Launch& P = lds_desc.P;
        // with the request's order (longest predicted first), position
        // first + e holds trajectory order[first + e]; written by the order's
        // kernels before the request was published, read past any line an
        // earlier request left in this die's L2
        const long long i =
            P.order ? (long long)__hip_atomic_load(P.order + first + e, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM)
                    : first + e;
        double y[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = load_through(P.y0 + c * P.ld + i);
        lane_K[lane] = lane_ctl(P);
        const Force F = lane_force(P);
        lane_F[lane] = F;
        lane_near2[lane] = lds_desc.fp32 ? P.near2 : INFINITY;
        lane_yf[lane] = P.yf;
        lane_obs[lane] = P.obs;
        lane_ld[lane] = P.ld;
        lane_idx[lane] = i;
        lane_seq[lane] = lds_desc.seq;
        lane_target[lane] = lds_desc.target;
        lane_slot[lane] = (int)(seq % A.ring);
        lane_va0[0][lane] = y[9];
        lane_va0[1][lane] = y[10];
        lane_va0[2][lane] = y[11];
        lane_m_atom[lane] = P.m_atom;
        lane_half_mi[lane] = P.half_mi;
        start(F, lds_S, y, L);
        busy = 1;
      }
    }

    if (__ballot(busy) != 0ull) {
      idle = false;
      continue;
    }
    // nothing to run: stop if asked, or after idle_ticks without work; else
    // wait ~100 us and look again (each look is a few loads of the request
    // words by each of ~2,000 waves)
    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
    if (claimed_any || !idle) {
      idle = true;
      idle_since = now;
    }
    int stop = 0;
    if (lane == 0) stop = load_system(A.stop) != 0ull;
    if (__shfl(stop, 0, WAVE)) break;
    if (now - idle_since > (unsigned long long)A.idle_ticks) break;
    for (int k = 0; k < 30; ++k) __builtin_amdgcn_s_sleep(127);
  }
}

// ---------------------------------------------------------------------------
// Host side.

thread_local std::string g_error;

int fail(int rc, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int rc, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return rc;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(AI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_params(const ai_params* p) {
  const double v[] = {p->m_ion, p->m_atom, p->Cn,   p->Cm,       p->a[0],
                      p->a[1],  p->a[2],   p->q[0], p->q[1],     p->q[2],
                      p->omega_rf, p->r_exit, p->r_bounce, p->hmax};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// A device pointer of the current device (hipMalloc, pool or managed memory).
bool on_current_device(const void* ptr, int dev) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return false;
  return attr.device == dev;
}

struct DeviceFacts {
  int cus = 0;
  int plain_blocks_per_cu = 0;
  int plain32_blocks_per_cu = 0;
  int persistent_blocks_per_cu = 0;
  hipFuncAttributes plain_attr{};
  hipFuncAttributes plain32_attr{};
  hipFuncAttributes persistent_attr{};
  bool ready = false;
};

std::mutex g_facts_mutex;
DeviceFacts g_facts[64];

int device_facts(int dev, DeviceFacts** out) {
  if (dev < 0 || dev >= 64) return fail(AI_EHIP, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_facts_mutex);
  DeviceFacts& f = g_facts[dev];
  if (!f.ready) {
    hipError_t e;
    if ((e = hipDeviceGetAttribute(&f.cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return hip_fail(e, "hipDeviceGetAttribute");
    if ((e = hipFuncGetAttributes(&f.plain_attr, (const void*)ai_plain_kernel)) != hipSuccess)
      return hip_fail(e, "hipFuncGetAttributes(plain)");
    if ((e = hipFuncGetAttributes(&f.plain32_attr, (const void*)ai_plain32_kernel)) != hipSuccess)
      return hip_fail(e, "hipFuncGetAttributes(plain32)");
    if ((e = hipFuncGetAttributes(&f.persistent_attr, (const void*)ai_persistent_kernel)) != hipSuccess)
      return hip_fail(e, "hipFuncGetAttributes(persistent)");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.plain_blocks_per_cu,
                                                          ai_plain_kernel, BLOCK, 0)) != hipSuccess)
      return hip_fail(e, "occupancy(plain)");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.plain32_blocks_per_cu,
                                                          ai_plain32_kernel, BLOCK, 0)) != hipSuccess)
      return hip_fail(e, "occupancy(plain32)");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.persistent_blocks_per_cu,
                                                          ai_persistent_kernel, BLOCK, 0)) != hipSuccess)
      return hip_fail(e, "occupancy(persistent)");
    if (f.persistent_blocks_per_cu < 1) f.persistent_blocks_per_cu = 1;
    f.ready = true;
  }
  *out = &f;
  return AI_OK;
}

// The static scratch of ai_integrate_static_async: its first
// AI_STATIC_QUEUE_BYTES hold the persistent kernel's queue counter, the rest
// the schedule's workspace.  Each device holds its own copy until the process
// ends; host code addresses it only through the device address
// hipGetSymbolAddress gives on that device (the array's host-side name is a
// stand-in, not device memory).
constexpr size_t AI_STATIC_QUEUE_BYTES = 256;
static_assert(AI_STATIC_SCRATCH_BYTES > AI_STATIC_QUEUE_BYTES, "scratch size");
static __device__ __align__(256) unsigned char scratch[AI_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mutex;
char* g_scratch[64] = {};

// The device address of this device's static scratch, looked up once per
// device (dev must be the current device).
int static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= 64) return fail(AI_EHIP, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_scratch[dev] = (char*)ptr;
  }
  *out = g_scratch[dev];
  return AI_OK;
}

// Host memory (pinned, registered or pageable), as opposed to device memory.
bool is_host_memory(const void* ptr) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // unknown to the runtime: pageable host memory
  }
  return attr.type == hipMemoryTypeHost || attr.type == hipMemoryTypeUnregistered;
}

int validate(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
             double tmax, double rtol, double atol, const double* yf, const double* obs,
             int32_t kernel, bool host_ok = false) {
  if (!p) return fail(AI_EINVAL, "params is NULL");
  if (n < 0) return fail(AI_EINVAL, "n = %lld < 0", (long long)n);
  if (ld < n) return fail(AI_EINVAL, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  const int32_t base_kernel = kernel & 0xf;
  if ((base_kernel != AI_KERNEL_PLAIN && base_kernel != AI_KERNEL_PERSISTENT) ||
      (kernel & ~(0xf | AI_SCHEDULE_LONGEST_FIRST | AI_FP32_STAGES | AI_TIME_KERNEL |
                  (0x7f << 8) | AI_WIDE(3))) != 0 ||
      ((kernel >> 8) & 0x7f) > 64)
    return fail(AI_EINVAL, "unknown kernel argument 0x%x", (unsigned)kernel);
  if ((kernel & AI_FP32_STAGES) && base_kernel != AI_KERNEL_PLAIN)
    return fail(AI_EUNSUPPORTED, "single-precision stages run in the plain kernel only");
  if (!finite_params(p)) return fail(AI_EINVAL, "non-finite system constant");
  if (!(p->m_ion > 0.0) || !(p->m_atom > 0.0)) return fail(AI_EINVAL, "masses must be > 0");
  if (p->n < 1 || p->n >= p->m) return fail(AI_EINVAL, "need 1 <= n < m");
  if (p->hmax < 0.0 || p->r_exit < 0.0 || p->r_bounce < 0.0)
    return fail(AI_EINVAL, "hmax, r_exit and r_bounce must be >= 0");
  if (p->max_steps < 1 || p->max_steps > 2147483647LL)
    return fail(AI_EINVAL, "max_steps must be in [1, 2^31 - 1]");
  if (!std::isfinite(t0) || !std::isfinite(tmax) || !(tmax > t0))
    return fail(AI_EINVAL, "need finite t0 < tmax");
  if (!std::isfinite(rtol) || !(rtol > 0.0) || !std::isfinite(atol) || !(atol > 0.0))
    return fail(AI_EINVAL, "rtol and atol must be finite and > 0");
  if (p->n != 4 || p->m != 8) {
    if (p->m > 16)
      return fail(AI_EUNSUPPORTED, "exponents n=%d, m=%d: this build integrates m <= 16",
                  p->n, p->m);
    if (base_kernel != AI_KERNEL_PLAIN || (kernel & AI_FP32_STAGES))
      return fail(AI_EUNSUPPORTED, "exponents other than n=4, m=8 run in the plain double "
                  "kernel only");
  }
  // the trap phase omega t is reduced with a two-part pi/2 valid below 2^31 pi/2
  if (std::fabs(p->omega_rf) * std::fmax(std::fabs(t0), std::fabs(tmax)) >= 3.0e9)
    return fail(AI_EUNSUPPORTED, "|omega_rf t| reaches %.3g rad; this build evaluates the trap "
                "phase below 3e9 rad", std::fabs(p->omega_rf) * std::fmax(std::fabs(t0), std::fabs(tmax)));
  if (n == 0) return AI_OK;
  if (!y0 || !yf || !obs) return fail(AI_EINVAL, "NULL buffer with n > 0");
  // plane extents, in elements
  if (ld > (int64_t)(INT64_MAX / 8 / AI_NOBS)) return fail(AI_EINVAL, "ld too large");
  const char* lo[3] = {(const char*)y0, (const char*)yf, (const char*)obs};
  const int64_t ext[3] = {12 * ld * 8, 12 * ld * 8, AI_NOBS * ld * 8};
  // obs must not overlap the states; final_state equals y0 or is disjoint
  for (int i = 1; i < 3; ++i)
    for (int j = 0; j < i; ++j) {
      if (i == 1 && j == 0 && lo[0] == lo[1]) continue;
      if (lo[i] < lo[j] + ext[j] && lo[j] < lo[i] + ext[i])
        return fail(AI_EINVAL, "output buffers overlap");
    }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (host_ok) {
    for (const void* ptr : {(const void*)y0, (const void*)yf, (const void*)obs})
      if (!on_current_device(ptr, dev) && !is_host_memory(ptr))
        return fail(AI_EINVAL, "y0, final_state and obs must be host memory or device memory "
                               "of the current device");
    return AI_OK;
  }
  if (!on_current_device(y0, dev) || !on_current_device(yf, dev) || !on_current_device(obs, dev))
    return fail(AI_EINVAL, "y0, final_state and obs must be device memory of the current device");
  return AI_OK;
}

Launch launch_constants(const ai_params* p, int64_t n, int64_t ld, double t0, double tmax,
                        double rtol, double atol) {
  Launch P;
  const double w2 = p->omega_rf * p->omega_rf / 4.0;
  P.mr = p->m_atom / p->m_ion;
  P.nCa = (p->n * p->Cn) / p->m_atom;
  P.mCa = (p->m * p->Cm) / p->m_atom;
  P.pot_n = p->n;
  P.pot_m = p->m;
  for (int k = 0; k < 3; ++k) {
    P.ka[k] = p->a[k] * w2;
    P.kq[k] = 2.0 * p->q[k] * w2;
  }
  P.omega = p->omega_rf;
  P.r_exit2 = p->r_exit * p->r_exit;
  P.r_bounce2 = p->r_bounce * p->r_bounce;
  P.half_mi = 0.5 * p->m_ion;
  P.m_atom = p->m_atom;
  P.t0 = t0;
  P.tf = tmax;
  P.hmax = p->hmax > 0.0 ? p->hmax : 0.1 * (tmax - t0);
  P.rtol = rtol;
  P.inv_rtol = 1.0 / rtol;
  P.thr = atol / rtol;
  P.vbound = (rtol / atol) * (1.0 + 0x1p-20);
  P.hinit_den = 0.8 * std::pow(rtol, 0.2);
  P.max_steps = (int)p->max_steps;
  P.n = n;
  P.ld = ld;
  P.first_dynamic = 0;
  P.wide = 0;
  P.wide_waves = 0;
  P.exit_on = p->r_exit > 0.0;
  // single-precision stages: waves integrate in double within 100 R_e of the
  // ion, R_e = (m Cm / (n Cn))^(1/(m-n)) the minimum of V (10 a0 for Li +
  // Yb+); the potential's length scale is unknown otherwise, so double
  // throughout, unless there is no interaction at all
  if (p->Cn > 0.0 && p->Cm > 0.0) {
    const double re = std::pow(p->m * p->Cm / (p->n * p->Cn), 1.0 / (p->m - p->n));
    P.near2 = (100.0 * re) * (100.0 * re);
  } else {
    P.near2 = (p->Cn == 0.0 && p->Cm == 0.0) ? 0.0 : INFINITY;
  }
  P.refill_min = 1;
  P.y0 = nullptr;
  P.yf = nullptr;
  P.obs = nullptr;
  P.order = nullptr;
  P.key = nullptr;
  P.queue = nullptr;
  return P;
}

// AI_TIME_KERNEL: per thread, a ring of start/stop event pairs recorded around
// the integration kernels of its last AI_TIMER_RING calls with the flag.
constexpr int AI_TIMER_RING = 64;
struct KernelTimer {
  int device = -1;
  hipEvent_t start[AI_TIMER_RING] = {}, stop[AI_TIMER_RING] = {};
  int next = 0;        // slot of the next call
  long long count = 0; // calls recorded
};
thread_local KernelTimer g_timer;

hipError_t timer_events(KernelTimer& T) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (T.device != dev) {
    for (int i = 0; i < AI_TIMER_RING; ++i) {
      if (T.start[i]) (void)hipEventDestroy(T.start[i]);
      if (T.stop[i]) (void)hipEventDestroy(T.stop[i]);
      T.start[i] = T.stop[i] = nullptr;
    }
    T.next = 0;
    T.count = 0;
    T.device = -1;
    for (int i = 0; i < AI_TIMER_RING; ++i) {
      if ((e = hipEventCreate(&T.start[i])) != hipSuccess) return e;
      if ((e = hipEventCreate(&T.stop[i])) != hipSuccess) return e;
    }
    T.device = dev;
  }
  return hipSuccess;
}

// Record the start (or stop) event of the integration kernel on s if asked.
int time_mark(int32_t kernel, bool start, hipStream_t s) {
  if (!(kernel & AI_TIME_KERNEL)) return AI_OK;
  hipError_t e = timer_events(g_timer);
  if (e == hipSuccess)
    e = hipEventRecord(start ? g_timer.start[g_timer.next] : g_timer.stop[g_timer.next], s);
  if (e != hipSuccess) return hip_fail(e, "kernel timing event");
  if (!start) {
    g_timer.next = (g_timer.next + 1) % AI_TIMER_RING;
    g_timer.count += 1;
  }
  return AI_OK;
}

ai_order_model order_model(const ai_params* p, double t0, double tmax, double rtol, bool sampled) {
  return ai_make_order_model(p->a, p->q, p->omega_rf, p->r_exit, t0, tmax, rtol, sampled);
}

int launch_finalize(const Launch& P, double* final_state, double* obs, hipStream_t s) {
  const long long blocks = (P.n + 255) / 256;
  hipLaunchKernelGGL(ai_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, final_state,
                     obs);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AI_OK : hip_fail(e, "launch(finalize)");
}

// Pinned host staging for the launch tables that batched calls copy to the
// device with hipMemcpyAsync.  A copy from pageable memory would have to be
// staged by the runtime before the call returns; from pinned memory it runs
// asynchronously, so a block is handed out again only after the event
// recorded behind its copy on the caller's stream has completed.  Blocks are
// kept per device and reused; their number grows only with the number of
// copies in flight at once.
struct PinnedBlock {
  int device = -1;
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t copied = nullptr;  // recorded after the block's last copy
  // free; reserved by a call that is filling it (its event not yet
  // recorded); or in flight (free once `copied` has completed)
  enum { FREE, RESERVED, IN_FLIGHT } state = FREE;
};

std::mutex g_pinned_mutex;
std::vector<PinnedBlock*> g_pinned;

// A free pinned block of at least `bytes` on device `dev` (nullptr: out of
// memory, g_error set).
PinnedBlock* pinned_acquire(int dev, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_pinned_mutex);
  PinnedBlock* best = nullptr;
  for (PinnedBlock* b : g_pinned) {
    if (b->device != dev || b->state == PinnedBlock::RESERVED) continue;
    if (b->state == PinnedBlock::IN_FLIGHT) {
      const hipError_t q = hipEventQuery(b->copied);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) (void)hipGetLastError();
      b->state = PinnedBlock::FREE;
    }
    if (b->cap >= bytes && (!best || b->cap < best->cap)) best = b;
  }
  if (!best) {
    best = new (std::nothrow) PinnedBlock;
    if (!best) {
      fail(AI_ENOMEM, "pinned staging block");
      return nullptr;
    }
    best->device = dev;
    best->cap = bytes < 65536 ? 65536 : bytes;
    hipError_t e = hipHostMalloc((void**)&best->host, best->cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&best->copied, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (best->host) (void)hipHostFree(best->host);
      delete best;
      fail(AI_ENOMEM, "pinned staging block: %s", hipGetErrorString(e));
      return nullptr;
    }
    g_pinned.push_back(best);
  }
  best->state = PinnedBlock::RESERVED;  // until released
  return best;
}

// Mark the block's copy as enqueued on s (or give the block back unused).
hipError_t pinned_release(PinnedBlock* b, hipStream_t s, bool copied) {
  std::lock_guard<std::mutex> lock(g_pinned_mutex);
  if (!copied) {
    b->state = PinnedBlock::FREE;
    return hipSuccess;
  }
  const hipError_t e = hipEventRecord(b->copied, s);
  if (e != hipSuccess) {
    // the copy's completion cannot be tracked: wait for it before reuse
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    b->state = PinnedBlock::FREE;
    return e;
  }
  b->state = PinnedBlock::IN_FLIGHT;
  return e;
}

// The plain kernels over P (P.order set or not): with a schedule, the
// longest predicted trajectories run four lanes each.  Kernel timing events
// around the launch if asked.
int launch_plain(Launch& P, const ai_params* p, int32_t kernel, hipStream_t s) {
  const long long n = P.n;
  if (P.order && !(kernel & AI_FP32_STAGES)) {
    const long long width = wide_trajectories(kernel);
    P.wide = n < width ? n : width;
    P.wide_waves = (int)((P.wide + WAVE / 4 - 1) / (WAVE / 4));
  }
  const long long blocks = P.wide_waves + (n - P.wide + BLOCK - 1) / BLOCK;
  if (blocks > 0x7fffffffLL) return fail(AI_EINVAL, "n too large for one launch");
  int rc = time_mark(kernel, true, s);
  if (rc != AI_OK) return rc;
  if (kernel & AI_FP32_STAGES)
    hipLaunchKernelGGL(ai_plain32_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P);
  else if (p->n != 4 || p->m != 8)
    hipLaunchKernelGGL(ai_plain_nm_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P);
  else
    hipLaunchKernelGGL(ai_plain_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch(plain)");
  return time_mark(kernel, false, s);
}

}  // namespace

int ai_fail(int rc, const char* msg) { return fail(rc, "%s", msg); }

int ai_check_request(const ai_batch_item* item, int32_t kernel, bool host_ok) {
  g_error.clear();
  if (!item) return fail(AI_EINVAL, "item is NULL");
  if ((kernel & ~AI_FP32_STAGES) != AI_KERNEL_PLAIN)
    return fail(AI_EUNSUPPORTED, "a request runs the plain kernel (kernel 0x%x)",
                (unsigned)kernel);
  const int rc = validate(&item->params, item->y0, item->n, item->ld, item->t0, item->tmax,
                          item->rtol, item->atol, item->final_state, item->obs, kernel, host_ok);
  if (rc != AI_OK) return rc;
  return item->rtol < 100.0 * 2.220446049250313e-16 ? AI_WRTOL : AI_OK;
}

void ai_resident_describe(const ai_batch_item* it, int32_t kernel, double* y0s, double* fins,
                          double* obss, int64_t ld, uint64_t seq, uint64_t done_target,
                          const unsigned* order, ai_resident_desc* out) {
  std::memset(out, 0, sizeof *out);
  ResidentDesc d;
  std::memset(&d, 0, sizeof d);
  const double rtol = it->rtol < 100.0 * 2.220446049250313e-16 ? 100.0 * 2.220446049250313e-16
                                                                : it->rtol;
  d.P = launch_constants(&it->params, it->n, ld, it->t0, it->tmax, rtol, it->atol);
  d.P.y0 = y0s;
  d.P.yf = fins;
  d.P.obs = obss;
  d.P.order = order;
  d.seq = (long long)seq;
  d.target = (long long)done_target;
  d.fp32 = (kernel & AI_FP32_STAGES) ? 1 : 0;
  std::memcpy(out, &d, sizeof d);
}

int ai_resident_order(const ai_batch_item* it, const double* y0, int64_t ld, hipStream_t s,
                      const unsigned** order, void** ws) {
  *order = nullptr;
  *ws = nullptr;
  const double rtol = it->rtol < 100.0 * 2.220446049250313e-16 ? 100.0 * 2.220446049250313e-16
                                                                : it->rtol;
  unsigned* o = nullptr;
  unsigned* key = nullptr;
  const hipError_t e = ai_longest_first_order(
      y0, it->n, ld, order_model(&it->params, it->t0, it->tmax, rtol, false), &o, &key, ws, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? fail(AI_ENOMEM, "request order: %s", hipGetErrorString(e))
                                    : hip_fail(e, "request order");
  }
  *order = o;
  return AI_OK;
}

int ai_resident_launch(const ai_resident_args* a, hipStream_t s, int64_t* waves) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  static std::mutex mu;
  static int per_cu[64] = {};
  int cus = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute");
  {
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) return fail(AI_EHIP, "device ordinal %d out of range", dev);
    if (per_cu[dev] == 0) {
      int b = 0;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, ai_resident_kernel, BLOCK, 0)) !=
          hipSuccess)
        return hip_fail(e, "occupancy(resident)");
      per_cu[dev] = b > 0 ? b : 1;
    }
  }
  const long long grid = (long long)cus * per_cu[dev];
  hipLaunchKernelGGL(ai_resident_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, s, *a);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch(resident)");
  if (waves) *waves = grid;
  return AI_OK;
}

namespace {

// A batch's four-lane waves (with its longest-first order) and grid size.
void batch_layout(BatchLaunch& B, int32_t kernel) {
  B.wide = 0;
  B.wide_waves = 0;
  if (B.order) {
    const long long width = wide_trajectories(kernel);
    B.wide = B.total < width ? B.total : width;
    B.wide_waves = (int)((B.wide + WAVE / 4 - 1) / (WAVE / 4));
  }
}
unsigned batch_blocks(const BatchLaunch& B) {
  return (unsigned)(B.wide_waves + (B.total - B.wide + BLOCK - 1) / BLOCK);
}

// The host side of a batched call: validated items, the launch table's
// entries and the schedule's per-item models.
struct BatchPrep {
  std::vector<BatchEntry> entries;
  std::vector<ai_order_item> keys;
  long long total = 0;
  double cost_max = 0.0;
};

// Validate a batch and fill prep; `extra` are the kernel flags allowed besides
// the schedule.  Returns AI_OK, AI_WRTOL or a negative ai_rc (g_error set).
int prepare_batch(const ai_batch_item* items, int32_t count, int32_t kernel, int32_t extra,
                  BatchPrep& prep) {
  if (count < 0) return fail(AI_EINVAL, "count = %d < 0", count);
  if (count > 0 && !items) return fail(AI_EINVAL, "items is NULL");
  if ((kernel & ~(AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(3) | extra)) != AI_KERNEL_PLAIN)
    return fail(AI_EUNSUPPORTED, "a batch runs the plain double kernel (kernel 0x%x)",
                (unsigned)kernel);
  int warn = AI_OK;
  for (int32_t b = 0; b < count; ++b) {
    const ai_batch_item& it = items[b];
    int rc = validate(&it.params, it.y0, it.n, it.ld, it.t0, it.tmax, it.rtol, it.atol,
                      it.final_state, it.obs, AI_KERNEL_PLAIN);
    if (rc != AI_OK) {
      const std::string why = g_error;
      return fail(rc, "item %d: %s", b, why.c_str());
    }
    if (it.params.n != 4 || it.params.m != 8)
      return fail(AI_EUNSUPPORTED, "item %d: a batch integrates n=4, m=8 potentials", b);
    if (it.n == 0) continue;
    double rtol = it.rtol;
    if (rtol < 100.0 * 2.220446049250313e-16) {
      rtol = 100.0 * 2.220446049250313e-16;
      warn = AI_WRTOL;
    }
    BatchEntry E;
    E.P = launch_constants(&it.params, it.n, it.ld, it.t0, it.tmax, rtol, it.atol);
    E.P.y0 = it.y0;
    E.P.yf = it.final_state;
    E.P.obs = it.obs;
    E.offset = prep.total;
    prep.entries.push_back(E);
    ai_order_item K;
    K.y0 = it.y0;
    K.ld = it.ld;
    K.offset = prep.total;
    K.n = it.n;
    K.model = order_model(&it.params, it.t0, it.tmax, rtol, true);
    prep.cost_max = std::fmax(prep.cost_max, (double)K.model.horizon * K.model.rate);
    prep.keys.push_back(K);
    prep.total += it.n;
  }
  if ((prep.total + BLOCK - 1) / BLOCK > 0x7fffffffLL)
    return fail(AI_EINVAL, "%lld trajectories are too many for one launch", prep.total);
  return warn;
}

}  // namespace

extern "C" {

int ai_version(void) { return 1; }
int ai_nobs(void) { return AI_NOBS; }
const char* ai_last_error(void) { return g_error.c_str(); }

int ai_get_kernel_info(int32_t kernel, ai_kernel_info* info) {
  if (!info) return fail(AI_EINVAL, "info is NULL");
  const bool fp32 = (kernel & AI_FP32_STAGES) != 0;
  kernel &= 0xf;
  if (kernel != AI_KERNEL_PLAIN && kernel != AI_KERNEL_PERSISTENT)
    return fail(AI_EINVAL, "unknown kernel %d", kernel);
  if (fp32 && kernel != AI_KERNEL_PLAIN)
    return fail(AI_EUNSUPPORTED, "single-precision stages run in the plain kernel only");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  DeviceFacts* f = nullptr;
  int rc = device_facts(dev, &f);
  if (rc != AI_OK) return rc;
  const hipFuncAttributes& a = kernel == AI_KERNEL_PERSISTENT ? f->persistent_attr
                               : fp32                            ? f->plain32_attr
                                                                 : f->plain_attr;
  const int bpc = kernel == AI_KERNEL_PERSISTENT ? f->persistent_blocks_per_cu
                  : fp32                         ? f->plain32_blocks_per_cu
                                                 : f->plain_blocks_per_cu;
  info->block_threads = BLOCK;
  info->vgprs = a.numRegs;
  info->spill_bytes = (int32_t)a.localSizeBytes;
  info->blocks_per_cu = bpc;
  info->waves_per_simd = bpc * (BLOCK / WAVE) / 4;
  info->compute_units = f->cus;
  info->persistent_blocks = (int64_t)f->cus * f->persistent_blocks_per_cu;
  return AI_OK;
}

}  // extern "C"

namespace {

// ai_integrate_async's work.  scratch: NULL, or the library's static device
// scratch of this device (AI_STATIC_SCRATCH_BYTES), from which the schedule's
// workspace and the persistent kernel's queue counter are taken instead of the
// stream-ordered allocator; the caller has validated the arguments and checked
// what needs checking against the scratch's capacity.
int integrate_async(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
                    double tmax, double rtol, double atol, double* final_state, double* obs,
                    int32_t kernel, void* stream, char* scratch_ptr) {
  int rc = AI_OK;
  int warn = AI_OK;
  if (rtol < 100.0 * 2.220446049250313e-16) {
    rtol = 100.0 * 2.220446049250313e-16;
    warn = AI_WRTOL;
  }
  if (n == 0) return warn;

  hipStream_t s = (hipStream_t)stream;
  Launch P = launch_constants(p, n, ld, t0, tmax, rtol, atol);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  DeviceFacts* f = nullptr;
  rc = device_facts(dev, &f);
  if (rc != AI_OK) return rc;

  P.y0 = y0;
  P.yf = final_state;
  P.obs = obs;

  // optional schedule: longest predicted trajectories first
  unsigned* order = nullptr;
  unsigned* key = nullptr;
  void* order_ws = nullptr;
  if ((kernel & AI_SCHEDULE_LONGEST_FIRST) && n <= 0xffffffffLL) {
    e = ai_longest_first_order(y0, n, ld, order_model(p, t0, tmax, rtol, false), &order, &key,
                               &order_ws, s, scratch_ptr ? scratch_ptr + AI_STATIC_QUEUE_BYTES
                                                         : nullptr,
                               scratch_ptr ? AI_STATIC_SCRATCH_BYTES - AI_STATIC_QUEUE_BYTES : 0);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e == hipErrorOutOfMemory ? fail(AI_ENOMEM, "schedule workspace: %s",
                                             hipGetErrorString(e))
                                      : hip_fail(e, "schedule");
    }
  }
  P.order = order;
  P.key = key;
  auto release = [&]() -> int {
    if (order_ws) {
      hipError_t fe = hipFreeAsync(order_ws, s);
      if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync(schedule)");
    }
    return AI_OK;
  };
  auto conclude = [&]() -> int {
    const int frc = launch_finalize(P, final_state, obs, s);
    const int rrc = release();
    if (frc != AI_OK) return frc;
    return rrc != AI_OK ? rrc : warn;
  };

  if ((kernel & 0xf) == AI_KERNEL_PLAIN) {
    if ((rc = launch_plain(P, p, kernel, s)) != AI_OK) {
      release();
      return rc;
    }
    // the plain kernels store the derived observables themselves
    const int rrc = release();
    return rrc != AI_OK ? rrc : warn;
  }

  const int refill_min = (kernel >> 8) & 0x7f;
  P.refill_min = refill_min > 0 ? refill_min : 1;
  // with the schedule, the leading positions run four lanes each in waves of
  // their own (as in the plain kernel); the other waves start a wave's worth
  // of the following positions each and draw the rest from the queue
  if (P.order) {
    const long long width = wide_trajectories(kernel);
    P.wide = n < width ? n : width;
    P.wide_waves = (int)((P.wide + WAVE / 4 - 1) / (WAVE / 4));
  }
  long long blocks = (long long)f->cus * f->persistent_blocks_per_cu;
  const long long need = P.wide_waves + (n - P.wide + BLOCK - 1) / BLOCK;
  if (blocks > need) blocks = need;
  if (blocks < P.wide_waves) blocks = P.wide_waves;
  P.first_dynamic = P.wide + (blocks - P.wide_waves) * BLOCK;
  unsigned long long* queue = (unsigned long long*)scratch_ptr;
  // the queue counter: from the static scratch, else stream-ordered (released
  // by free_queue)
  auto free_queue = [&]() -> hipError_t {
    return scratch_ptr ? hipSuccess : hipFreeAsync(queue, s);
  };
  if (!queue && (e = hipMallocAsync((void**)&queue, sizeof(unsigned long long), s)) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(AI_ENOMEM, "hipMallocAsync(queue): %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(ai_queue_reset_kernel, dim3(1), dim3(1), 0, s, queue);
  if ((e = hipGetLastError()) != hipSuccess) {
    (void)free_queue();
    release();
    return hip_fail(e, "launch(queue reset)");
  }
  P.queue = queue;
  if ((rc = time_mark(kernel, true, s)) != AI_OK) {
    (void)free_queue();
    release();
    return rc;
  }
  hipLaunchKernelGGL(ai_persistent_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P);
  if ((e = hipGetLastError()) != hipSuccess) {
    (void)free_queue();
    release();
    return hip_fail(e, "launch(persistent)");
  }
  if ((rc = time_mark(kernel, false, s)) != AI_OK) {
    (void)free_queue();
    release();
    return rc;
  }
  if ((e = free_queue()) != hipSuccess) {
    release();
    return hip_fail(e, "hipFreeAsync(queue)");
  }
  return conclude();
}

}  // namespace

extern "C" {

int ai_integrate_async(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
                       double tmax, double rtol, double atol, double* final_state, double* obs,
                       int32_t kernel, void* stream) {
  g_error.clear();
  const int rc = validate(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel);
  if (rc != AI_OK) return rc;
  return integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel, stream,
                         nullptr);
}

int ai_integrate_static_async(const ai_params* p, const double* y0, int64_t n, int64_t ld,
                              double t0, double tmax, double rtol, double atol,
                              double* final_state, double* obs, int32_t kernel, void* stream) {
  g_error.clear();
  const int rc = validate(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel);
  if (rc != AI_OK) return rc;
  if (kernel & AI_TIME_KERNEL)
    return fail(AI_EINVAL, "AI_TIME_KERNEL needs events of its own: not in the static variant");
  if ((kernel & AI_SCHEDULE_LONGEST_FIRST) && n > AI_STATIC_MAX_SCHEDULED)
    return fail(AI_EINVAL, "n = %lld: a scheduled call takes at most %d trajectories here",
                (long long)n, AI_STATIC_MAX_SCHEDULED);
  if (n == 0) return integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs,
                                     kernel, stream, nullptr);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  char* scratch_ptr = nullptr;
  int frc = static_scratch(dev, &scratch_ptr);
  if (frc != AI_OK) return frc;
  if (kernel & AI_SCHEDULE_LONGEST_FIRST) {
    const size_t need = ai_order_workspace_bytes(n, (hipStream_t)stream);
    if (need == 0 || need > AI_STATIC_SCRATCH_BYTES - AI_STATIC_QUEUE_BYTES)
      return fail(AI_EINVAL, "the schedule of %lld trajectories needs %zu bytes of scratch; %zu held",
                  (long long)n, need, (size_t)(AI_STATIC_SCRATCH_BYTES - AI_STATIC_QUEUE_BYTES));
  }
  return integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel, stream,
                         scratch_ptr);
}

int ai_trace(const ai_params* p, const double* y0, double t0, double tmax, double rtol,
             double atol, int32_t refine, int64_t capacity, double* t_out, double* y_out,
             double* final_state, double* obs, int64_t* points) {
  g_error.clear();
  if (!points) return fail(AI_EINVAL, "points is NULL");
  *points = 0;
  if (refine < 1 || refine > 1024) return fail(AI_EINVAL, "refine = %d not in 1 .. 1024", refine);
  if (capacity < 0) return fail(AI_EINVAL, "capacity = %lld < 0", (long long)capacity);
  if (capacity > 0 && (!t_out || !y_out)) return fail(AI_EINVAL, "NULL point buffer");
  if (capacity > (int64_t)(INT64_MAX / 8 / 16)) return fail(AI_EINVAL, "capacity too large");
  int rc = validate(p, y0, 1, 1, t0, tmax, rtol, atol, final_state, obs, AI_KERNEL_PLAIN);
  if (rc != AI_OK) return rc;
  if (capacity > 0) {
    // the point buffers are disjoint from each other and from the others
    const char* lo[5] = {(const char*)y0, (const char*)final_state, (const char*)obs,
                         (const char*)t_out, (const char*)y_out};
    const int64_t ext[5] = {12 * 8, 12 * 8, AI_NOBS * 8, capacity * 8, 12 * capacity * 8};
    for (int i = 3; i < 5; ++i)
      for (int j = 0; j < i; ++j)
        if (lo[i] < lo[j] + ext[j] && lo[j] < lo[i] + ext[i])
          return fail(AI_EINVAL, "point buffers overlap");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (!on_current_device(t_out, dev) || !on_current_device(y_out, dev))
      return fail(AI_EINVAL, "t_out and y_out must be device memory of the current device");
  }
  int warn = AI_OK;
  if (rtol < 100.0 * 2.220446049250313e-16) {
    rtol = 100.0 * 2.220446049250313e-16;
    warn = AI_WRTOL;
  }
  Launch P = launch_constants(p, 1, 1, t0, tmax, rtol, atol);
  P.y0 = y0;
  P.yf = final_state;
  P.obs = obs;
  if (p->n != 4 || p->m != 8)
    hipLaunchKernelGGL(ai_trace_nm_kernel, dim3(1), dim3(BLOCK), 0, nullptr, P, (int)refine,
                       (long long)capacity, t_out, y_out);
  else
    hipLaunchKernelGGL(ai_trace_kernel, dim3(1), dim3(BLOCK), 0, nullptr, P, (int)refine,
                       (long long)capacity, t_out, y_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch(trace)");
  rc = launch_finalize(P, final_state, obs, nullptr);
  if (rc != AI_OK) return rc;
  double nsteps = 0.0;
  e = hipMemcpy(&nsteps, obs + AI_OBS_NSTEPS, sizeof nsteps, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(nsteps)");
  *points = (int64_t)nsteps * refine + 1;
  return warn;
}

int ai_kernel_time(int32_t back, float* ms) {
  g_error.clear();
  if (!ms) return fail(AI_EINVAL, "ms is NULL");
  *ms = 0.0f;
  if (back < 0 || back >= AI_TIMER_RING || back >= g_timer.count)
    return fail(AI_EINVAL, "no timed call %d back on this thread (%lld recorded, at most %d kept)",
                back, g_timer.count, AI_TIMER_RING);
  const int slot = ((g_timer.next - 1 - back) % AI_TIMER_RING + AI_TIMER_RING) % AI_TIMER_RING;
  const hipError_t e = hipEventElapsedTime(ms, g_timer.start[slot], g_timer.stop[slot]);
  if (e == hipErrorNotReady) return AI_EAGAIN;
  return e == hipSuccess ? AI_OK : hip_fail(e, "hipEventElapsedTime");
}

int ai_tune(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
            double tmax, double rtol, double atol, double* final_state, double* obs,
            int32_t* best_kernel, float* best_ms) {
  g_error.clear();
  if (!best_kernel || !best_ms) return fail(AI_EINVAL, "best_kernel or best_ms is NULL");
  *best_kernel = AI_KERNEL_PLAIN;
  *best_ms = 0.0f;
  if (final_state == y0 && n > 0)
    return fail(AI_EINVAL, "tuning runs the ensemble several times: final_state must not be y0");
  const bool general = p && (p->n != 4 || p->m != 8);
  const int32_t candidates[] = {
      AI_KERNEL_PLAIN,
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST,
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(1),
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(2),
      AI_KERNEL_PERSISTENT | AI_SCHEDULE_LONGEST_FIRST | AI_REFILL_MIN(1),
      AI_KERNEL_PERSISTENT | AI_SCHEDULE_LONGEST_FIRST | AI_REFILL_MIN(16),
      AI_KERNEL_PERSISTENT | AI_SCHEDULE_LONGEST_FIRST | AI_REFILL_MIN(64)};
  constexpr int NC = sizeof(candidates) / sizeof(candidates[0]);
  // one pair of events per candidate; a round enqueues every candidate
  // back-to-back on the null stream, each timed run right after an untimed run
  // of the same configuration, so each is timed as in a sequence of its own
  // calls (not from idle, and not after another configuration's different
  // load, e.g. the long, sparse tail of the unscheduled plain launch), and is
  // read after the round
  hipEvent_t ev[2 * NC] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 * NC && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  int rc = e == hipSuccess ? AI_OK : hip_fail(e, "hipEventCreate");
  int warn = AI_OK;
  float best = -1.0f;
  for (int round = 0; round < 2 && rc >= 0; ++round) {
    bool ran[NC] = {};
    for (int i = 0; i < NC; ++i) {
      const int32_t k = candidates[i];
      if (general && (k & 0xf) != AI_KERNEL_PLAIN) continue;  // other exponents: plain only
      rc = ai_integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, k, nullptr);
      if (rc < 0) break;
      (void)hipEventRecord(ev[2 * i], nullptr);
      rc = ai_integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, k, nullptr);
      if (rc < 0) break;
      warn = rc;
      (void)hipEventRecord(ev[2 * i + 1], nullptr);
      ran[i] = true;
    }
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) {
      if (rc >= 0) rc = hip_fail(e, "hipStreamSynchronize");
      break;
    }
    if (rc < 0) break;
    for (int i = 0; i < NC; ++i) {
      if (!ran[i]) continue;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
      if (best < 0.0f || ms < best) {
        best = ms;
        *best_kernel = candidates[i];
      }
    }
  }
  for (int i = 0; i < 2 * NC; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  if (rc < 0) return rc;
  *best_ms = best < 0.0f ? 0.0f : best;
  return warn;
}

int ai_tune_batch(const ai_batch_item* items, int32_t count, int32_t* best_kernel,
                  float* best_ms) {
  g_error.clear();
  if (!best_kernel || !best_ms) return fail(AI_EINVAL, "best_kernel or best_ms is NULL");
  *best_kernel = AI_KERNEL_PLAIN;
  *best_ms = 0.0f;
  for (int32_t b = 0; b < count && items; ++b)
    if (items[b].n > 0 && items[b].final_state == items[b].y0)
      return fail(AI_EINVAL, "item %d: tuning runs the batch several times: final_state must "
                  "not be y0", b);
  const int32_t candidates[] = {
      AI_KERNEL_PLAIN,
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(1),
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST,
      AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(2)};
  constexpr int NC = sizeof(candidates) / sizeof(candidates[0]);
  // as in ai_tune: two rounds, each candidate timed right after an untimed run
  // of itself on the null stream
  hipEvent_t ev[2 * NC] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 * NC && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  int rc = e == hipSuccess ? AI_OK : hip_fail(e, "hipEventCreate");
  int warn = AI_OK;
  float best = -1.0f;
  for (int round = 0; round < 2 && rc >= 0; ++round) {
    bool ran[NC] = {};
    for (int i = 0; i < NC; ++i) {
      rc = ai_integrate_batch_async(items, count, candidates[i], nullptr);
      if (rc < 0) break;
      (void)hipEventRecord(ev[2 * i], nullptr);
      rc = ai_integrate_batch_async(items, count, candidates[i], nullptr);
      if (rc < 0) break;
      warn = rc;
      (void)hipEventRecord(ev[2 * i + 1], nullptr);
      ran[i] = true;
    }
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) {
      if (rc >= 0) rc = hip_fail(e, "hipStreamSynchronize");
      break;
    }
    if (rc < 0) break;
    for (int i = 0; i < NC; ++i) {
      if (!ran[i]) continue;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
      if (best < 0.0f || ms < best) {
        best = ms;
        *best_kernel = candidates[i];
      }
    }
  }
  for (int i = 0; i < 2 * NC; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  if (rc < 0) return rc;
  *best_ms = best < 0.0f ? 0.0f : best;
  return warn;
}

int ai_integrate(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
                 double tmax, double rtol, double atol, double* final_state, double* obs,
                 int32_t kernel) {
  int rc = ai_integrate_async(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel,
                              nullptr);
  if (rc < 0) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return rc;
}

int ai_integrate_batch_async(const ai_batch_item* items, int32_t count, int32_t kernel,
                             void* stream) {
  g_error.clear();
  BatchPrep prep;
  int warn = prepare_batch(items, count, kernel, AI_TIME_KERNEL, prep);
  if (warn < 0) return warn;
  std::vector<BatchEntry>& entries = prep.entries;
  std::vector<ai_order_item>& keys = prep.keys;
  const long long total = prep.total;
  const double cost_max = prep.cost_max;
  if (total == 0) return warn;

  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  // the launch table: entries, then the schedule's items, in one allocation,
  // copied from a pinned staging block that stays reserved until the copy on
  // s has completed
  const int E = (int)entries.size();
  const size_t ebytes = (sizeof(BatchEntry) * E + 255) & ~size_t(255);
  const size_t kbytes = sizeof(ai_order_item) * E;
  const size_t tbytes = ebytes + kbytes;
  PinnedBlock* stage = pinned_acquire(dev, tbytes);
  if (!stage) return AI_ENOMEM;
  std::memcpy(stage->host, entries.data(), sizeof(BatchEntry) * E);
  std::memcpy(stage->host + ebytes, keys.data(), kbytes);
  char* table = nullptr;
  if ((e = hipMallocAsync((void**)&table, tbytes, s)) != hipSuccess) {
    (void)hipGetLastError();
    (void)pinned_release(stage, s, false);  // nothing was copied: cannot fail
    return fail(AI_ENOMEM, "hipMallocAsync(batch table): %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpyAsync(table, stage->host, tbytes, hipMemcpyHostToDevice, s)) !=
      hipSuccess) {
    (void)hipGetLastError();
    (void)pinned_release(stage, s, false);  // nothing was copied: cannot fail
    (void)hipFreeAsync(table, s);
    return hip_fail(e, "hipMemcpyAsync(batch table)");
  }
  if ((e = pinned_release(stage, s, true)) != hipSuccess) {
    (void)hipFreeAsync(table, s);
    return hip_fail(e, "hipEventRecord(batch table)");
  }
  BatchLaunch B;
  B.entries = (const BatchEntry*)table;
  B.count = E;
  B.total = total;
  B.order = nullptr;
  B.key = nullptr;
  B.wide = 0;
  B.wide_waves = 0;
  void* order_ws = nullptr;
  auto release = [&]() -> int {
    hipError_t fe = hipFreeAsync(table, s);
    if (order_ws && fe == hipSuccess) fe = hipFreeAsync(order_ws, s);
    return fe == hipSuccess ? AI_OK : hip_fail(fe, "hipFreeAsync(batch)");
  };
  if ((kernel & AI_SCHEDULE_LONGEST_FIRST) && total <= 0xffffffffLL) {
    unsigned* order = nullptr;
    unsigned* key = nullptr;
    e = ai_longest_first_order_batch((const ai_order_item*)(table + ebytes), E, total, cost_max,
                                     &order, &key, &order_ws, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release();
      return e == hipErrorOutOfMemory ? fail(AI_ENOMEM, "schedule workspace: %s",
                                             hipGetErrorString(e))
                                      : hip_fail(e, "schedule(batch)");
    }
    B.order = order;
    B.key = key;
  }
  batch_layout(B, kernel);
  int trc = time_mark(kernel, true, s);
  if (trc != AI_OK) {
    release();
    return trc;
  }
  hipLaunchKernelGGL(ai_plain_batch_kernel, dim3(batch_blocks(B)), dim3(BLOCK), 0, s, B);
  if ((e = hipGetLastError()) != hipSuccess) {
    release();
    return hip_fail(e, "launch(batch)");
  }
  if ((trc = time_mark(kernel, false, s)) != AI_OK) {
    release();
    return trc;
  }
  const int rc = release();
  return rc != AI_OK ? rc : warn;
}

int ai_integrate_batch(const ai_batch_item* items, int32_t count, int32_t kernel) {
  int rc = ai_integrate_batch_async(items, count, kernel, nullptr);
  if (rc < 0) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return rc;
}

// A batch prepared once: its launch table and (with the schedule) its order in
// device memory, so that each launch enqueues the integration and the
// observables kernels and nothing else.
struct ai_batch_plan {
  int device = 0;
  char* table = nullptr;  // BatchEntry[count] (hipMalloc)
  void* order_ws = nullptr;  // the schedule's stream-ordered workspace
  BatchLaunch launch{};
  int warn = AI_OK;
};

static void plan_release(ai_batch_plan* pl) {
  if (pl->order_ws) {
    (void)hipFreeAsync(pl->order_ws, nullptr);
    (void)hipStreamSynchronize(nullptr);
  }
  if (pl->table) (void)hipFree(pl->table);
  delete pl;
}

int ai_batch_plan_create(const ai_batch_item* items, int32_t count, int32_t kernel,
                         ai_batch_plan** out) {
  g_error.clear();
  if (!out) return fail(AI_EINVAL, "out is NULL");
  *out = nullptr;
  BatchPrep prep;
  const int warn = prepare_batch(items, count, kernel, 0, prep);
  if (warn < 0) return warn;
  ai_batch_plan* pl = new (std::nothrow) ai_batch_plan;
  if (!pl) return fail(AI_ENOMEM, "plan");
  pl->warn = warn;
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    plan_release(pl);
    return hip_fail(e, "hipGetDevice");
  }
  const int E = (int)prep.entries.size();
  BatchLaunch& B = pl->launch;
  B.count = E;
  B.total = prep.total;
  B.order = nullptr;
  B.key = nullptr;
  B.entries = nullptr;
  B.wide = 0;
  B.wide_waves = 0;
  if (prep.total > 0) {
    const size_t ebytes = (sizeof(BatchEntry) * E + 255) & ~size_t(255);
    const size_t kbytes = sizeof(ai_order_item) * E;
    std::vector<char> host(ebytes + kbytes);
    std::memcpy(host.data(), prep.entries.data(), sizeof(BatchEntry) * E);
    std::memcpy(host.data() + ebytes, prep.keys.data(), kbytes);
    if ((e = hipMalloc((void**)&pl->table, host.size())) != hipSuccess) {
      (void)hipGetLastError();
      plan_release(pl);
      return fail(AI_ENOMEM, "hipMalloc(plan table): %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(pl->table, host.data(), host.size(), hipMemcpyHostToDevice)) !=
        hipSuccess) {
      plan_release(pl);
      return hip_fail(e, "hipMemcpy(plan table)");
    }
    B.entries = (const BatchEntry*)pl->table;
    if ((kernel & AI_SCHEDULE_LONGEST_FIRST) && prep.total <= 0xffffffffLL) {
      unsigned* order = nullptr;
      unsigned* key = nullptr;
      e = ai_longest_first_order_batch((const ai_order_item*)(pl->table + ebytes), E,
                                       prep.total, prep.cost_max, &order, &key, &pl->order_ws,
                                       nullptr);
      if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        plan_release(pl);
        return e == hipErrorOutOfMemory
                   ? fail(AI_ENOMEM, "schedule workspace: %s", hipGetErrorString(e))
                   : hip_fail(e, "schedule(plan)");
      }
      B.order = order;
      B.key = key;
    }
    batch_layout(B, kernel);
  }
  *out = pl;
  return warn;
}

int ai_batch_plan_launch(const ai_batch_plan* pl, void* stream) {
  g_error.clear();
  if (!pl) return fail(AI_EINVAL, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
    return fail(AI_EINVAL, "launch a plan on the device it was created on");
  const BatchLaunch& B = pl->launch;
  if (B.total == 0) return pl->warn;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(ai_plain_batch_kernel, dim3(batch_blocks(B)), dim3(BLOCK), 0, s, B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch(plan)");
  return pl->warn;
}

int ai_batch_plan_destroy(ai_batch_plan* pl) {
  g_error.clear();
  if (!pl) return fail(AI_EINVAL, "plan is NULL");
  plan_release(pl);
  return AI_OK;
}

}  // extern "C"
