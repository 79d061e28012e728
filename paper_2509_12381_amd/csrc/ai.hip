// ai.hip -- HIP kernels and C ABI of libai.so (declared in include/ai.h).
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

#include "ai.h"

namespace {

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) coefficients (Dormand and Prince 1980; the pair ode45
// uses, Sec. 1 and Fig. 2 caption).  Row 7 of a equals the fifth-order
// weights b, so stage 7 is f at the new solution (first same as last); the
// error weights are e = b - bhat.
constexpr double C2 = 1.0 / 5.0, C3 = 3.0 / 10.0, C4 = 4.0 / 5.0, C5 = 8.0 / 9.0;
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                 A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                 A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
constexpr double A71 = 35.0 / 384.0, A73 = 500.0 / 1113.0, A74 = 125.0 / 192.0,
                 A75 = -2187.0 / 6784.0, A76 = 11.0 / 84.0;
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                 E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

constexpr int WAVE = 64;
constexpr int BLOCK = 64;  // one wave per workgroup: a finished wave frees its slot at once

// Launch constants: the system constants folded into the forms the force and
// the controller use, computed once per call on the host.  Passed by value, so
// they sit in scalar registers, uniform across the wave.
struct Launch {
  double inv_mi, inv_ma;     // 1/m_ion, 1/m_atom
  double nCn, mCm;           // 4 C4 and 8 C8: (dV/dr)/r = s^3 (4 C4 - 8 C8 s^2), s = 1/r^2
  double ka[3], kq[3];       // trap: kappa_k(t) = ka_k + kq_k cos(omega t) = (a_k + 2 q_k cos) omega^2/4
  double omega;
  double r_exit2, r_bounce2;
  double half_mi, m_atom;    // for the observables
  double t0, tf, hmax, rtol, thr;
  double hinit_den;          // 0.8 rtol^(1/5)
  long long max_steps;
  long long n, ld;
  long long first_dynamic;   // persistent kernel: first index handed out by the queue
  int exit_on;               // r_exit > 0
};

// Per-lane integration state.
struct Lane {
  double y[12];
  double k1[12];
  double t, h, absh, hmin;
  double va0[3];
  double w_prev, t_first, t_last, position, rmin2, r2;
  long long nsteps, nfailed, bounces;
  int status;
  bool done, nofailed, fresh, approached;
};

// Distance from |t| to the next larger double (MATLAB's eps(t)); exact.
__device__ __forceinline__ double spacing(double t) {
  const double at = fabs(t);
  return __longlong_as_double(__double_as_longlong(at) + 1) - at;
}

// f(t, y) of Sec. 2.1 for V(r) = -C4/r^4 + C8/r^8.  cosrf = cos(omega t).
// Returns r^2 of the input state.
__device__ __forceinline__ double force(const Launch& P, double cosrf, const double* y,
                                        double* f) {
  const double dx = y[0] - y[6], dy = y[1] - y[7], dz = y[2] - y[8];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double s = 1.0 / r2;
  const double s2 = s * s;
  const double g = s2 * s * (P.nCn - P.mCm * s2);  // (dV/dr) / r
  const double gi = g * P.inv_mi, ga = g * P.inv_ma;
  f[0] = y[3];
  f[1] = y[4];
  f[2] = y[5];
  f[3] = -gi * dx - (P.ka[0] + P.kq[0] * cosrf) * y[0];
  f[4] = -gi * dy - (P.ka[1] + P.kq[1] * cosrf) * y[1];
  f[5] = -gi * dz - (P.ka[2] + P.kq[2] * cosrf) * y[2];
  f[6] = y[9];
  f[7] = y[10];
  f[8] = y[11];
  f[9] = ga * dx;
  f[10] = ga * dy;
  f[11] = ga * dz;
  return r2;
}

// Start of trajectory idx: load its y0 column, f(t0, y0), ode45's initial
// step and the observables' initial values.
__device__ __forceinline__ void start(const Launch& P, const double* __restrict__ y0,
                                      long long idx, Lane& L) {
#pragma unroll
  for (int c = 0; c < 12; ++c) L.y[c] = y0[c * P.ld + idx];
  L.t = P.t0;
  L.r2 = force(P, cos(P.omega * P.t0), L.y, L.k1);
  L.nsteps = L.nfailed = L.bounces = 0;
  L.status = 0;
  L.fresh = true;
  L.done = false;
  L.nofailed = true;
  L.h = 0.0;
  L.hmin = 0.0;

  bool finite = true;
  double rh = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    finite = finite && isfinite(L.y[c]) && isfinite(L.k1[c]);
    rh = fmax(rh, fabs(L.k1[c]) / fmax(fabs(L.y[c]), P.thr));
  }
  rh = rh / P.hinit_den;
  double absh = fmin(P.hmax, P.tf - P.t0);
  if (absh * rh > 1.0) absh = 1.0 / rh;
  L.absh = fmax(absh, 16.0 * spacing(P.t0));
  if (!finite) L.status = AI_ST_NONFINITE;

  const double dx = L.y[0] - L.y[6], dy = L.y[1] - L.y[7], dz = L.y[2] - L.y[8];
  const double w = dx * (L.y[3] - L.y[9]) + dy * (L.y[4] - L.y[10]) + dz * (L.y[5] - L.y[11]);
  L.va0[0] = L.y[9];
  L.va0[1] = L.y[10];
  L.va0[2] = L.y[11];
  L.approached = (w >= 0.0);
  L.w_prev = w;
  L.t_first = L.t_last = L.position = 0.0;
  L.rmin2 = L.r2;
}

// Step set-up of ode45: floor and cap the step, stretch it onto tf when within
// 10% of the remaining span.
__device__ __forceinline__ void begin_step(const Launch& P, Lane& L) {
  L.hmin = 16.0 * spacing(L.t);
  L.absh = fmin(P.hmax, fmax(L.hmin, L.absh));
  L.h = L.absh;
  L.done = false;
  if (1.1 * L.absh >= P.tf - L.t) {
    L.h = P.tf - L.t;
    L.absh = L.h;
    L.done = true;
  }
  L.nofailed = true;
}

// One Dormand-Prince attempt of size L.h from (L.t, L.y) followed by the error
// test and the controller; on acceptance the state advances and the
// observables and exits are updated.
__device__ __forceinline__ void attempt(const Launch& P, Lane& L) {
  const double t = L.t, h = L.h;
  const double tnew = L.done ? P.tf : t + h;
  const double* y = L.y;
  const double* k1 = L.k1;
  double ys[12], k2[12], k3[12], k4[12], k5[12], k6[12], k7[12], yn[12];

  const double h21 = h * A21;
#pragma unroll
  for (int c = 0; c < 12; ++c) ys[c] = y[c] + h21 * k1[c];
  force(P, cos(P.omega * (t + C2 * h)), ys, k2);

  const double h31 = h * A31, h32 = h * A32;
#pragma unroll
  for (int c = 0; c < 12; ++c) ys[c] = y[c] + (h31 * k1[c] + h32 * k2[c]);
  force(P, cos(P.omega * (t + C3 * h)), ys, k3);

  const double h41 = h * A41, h42 = h * A42, h43 = h * A43;
#pragma unroll
  for (int c = 0; c < 12; ++c) ys[c] = y[c] + (h41 * k1[c] + h42 * k2[c] + h43 * k3[c]);
  force(P, cos(P.omega * (t + C4 * h)), ys, k4);

  const double h51 = h * A51, h52 = h * A52, h53 = h * A53, h54 = h * A54;
#pragma unroll
  for (int c = 0; c < 12; ++c)
    ys[c] = y[c] + (h51 * k1[c] + h52 * k2[c] + h53 * k3[c] + h54 * k4[c]);
  force(P, cos(P.omega * (t + C5 * h)), ys, k5);

  const double h61 = h * A61, h62 = h * A62, h63 = h * A63, h64 = h * A64, h65 = h * A65;
#pragma unroll
  for (int c = 0; c < 12; ++c)
    ys[c] = y[c] + (h61 * k1[c] + h62 * k2[c] + h63 * k3[c] + h64 * k4[c] + h65 * k5[c]);
  force(P, cos(P.omega * (t + h)), ys, k6);

  const double h71 = h * A71, h73 = h * A73, h74 = h * A74, h75 = h * A75, h76 = h * A76;
#pragma unroll
  for (int c = 0; c < 12; ++c)
    yn[c] = y[c] + (h71 * k1[c] + h73 * k3[c] + h74 * k4[c] + h75 * k5[c] + h76 * k6[c]);
  const double r2n = force(P, cos(P.omega * tnew), yn, k7);

  // err = |h| max_c |sum_j e_j k_j| / max(|y|, |ynew|, AbsTol/RelTol)
  double ratio = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double e = E1 * k1[c] + E3 * k3[c] + E4 * k4[c] + E5 * k5[c] + E6 * k6[c] + E7 * k7[c];
    const double sc = fmax(fmax(fabs(y[c]), fabs(yn[c])), P.thr);
    const double v = fabs(e) / sc;
    ratio = (v > ratio || v != v) ? v : ratio;
  }
  const double err = L.absh * ratio;

  if (!isfinite(err)) {
    L.status = AI_ST_NONFINITE;
    return;
  }
  if (err > P.rtol) {
    L.nfailed += 1;
    if (L.absh <= L.hmin) {
      L.status = AI_ST_HMIN;
      return;
    }
    if (L.nofailed)
      L.absh = fmax(L.hmin, L.absh * fmax(0.1, 0.8 * pow(P.rtol / err, 0.2)));
    else
      L.absh = fmax(L.hmin, 0.5 * L.absh);
    L.nofailed = false;
    L.h = L.absh;
    L.done = false;
    L.fresh = false;
    return;
  }

  // accepted
  L.nsteps += 1;
  L.t = tnew;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    L.y[c] = yn[c];
    L.k1[c] = k7[c];
  }
  if (L.nofailed) {
    const double temp = 1.25 * pow(err / P.rtol, 0.2);
    L.absh = (temp > 0.2) ? L.absh / temp : 5.0 * L.absh;
  }
  L.fresh = true;

  // observables: closest approach = sign change of r r' from - to +
  const double dx = yn[0] - yn[6], dy = yn[1] - yn[7], dz = yn[2] - yn[8];
  const double w = dx * (yn[3] - yn[9]) + dy * (yn[4] - yn[10]) + dz * (yn[5] - yn[11]);
  if (L.w_prev < 0.0 && w >= 0.0) {
    L.approached = true;
    if (r2n < P.r_bounce2) {
      L.bounces += 1;
      if (L.bounces == 1) {
        L.t_first = tnew;
        L.position = sqrt(yn[0] * yn[0] + yn[1] * yn[1] + yn[2] * yn[2]);
      }
      L.t_last = tnew;
    }
  }
  L.w_prev = w;
  L.rmin2 = fmin(L.rmin2, r2n);
  L.r2 = r2n;

  if (L.approached && P.exit_on && r2n > P.r_exit2)
    L.status = AI_ST_ESCAPED;
  else if (L.done)
    L.status = AI_ST_TMAX;
  else if (L.nsteps >= P.max_steps)
    L.status = AI_ST_MAXSTEPS;
}

// Final state and observables of trajectory idx.
__device__ __forceinline__ void finish(const Launch& P, const Lane& L, long long idx,
                                       double* __restrict__ yf, double* __restrict__ obs) {
  const double* y = L.y;
#pragma unroll
  for (int c = 0; c < 12; ++c) yf[c * P.ld + idx] = y[c];
  const double cx = L.va0[1] * y[11] - L.va0[2] * y[10];
  const double cy = L.va0[2] * y[9] - L.va0[0] * y[11];
  const double cz = L.va0[0] * y[10] - L.va0[1] * y[9];
  const double dot = L.va0[0] * y[9] + L.va0[1] * y[10] + L.va0[2] * y[11];
  const double dvx = y[9] - L.va0[0], dvy = y[10] - L.va0[1], dvz = y[11] - L.va0[2];
  const double dx = y[0] - y[6], dy = y[1] - y[7], dz = y[2] - y[8];
  double o[AI_NOBS];
  o[AI_OBS_TEND] = L.t;
  o[AI_OBS_STATUS] = (double)L.status;
  o[AI_OBS_NSTEPS] = (double)L.nsteps;
  o[AI_OBS_NFAILED] = (double)L.nfailed;
  o[AI_OBS_BOUNCES] = (double)L.bounces;
  o[AI_OBS_LIFETIME] = L.bounces >= 2 ? L.t_last - L.t_first : 0.0;
  o[AI_OBS_ANGLE] = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
  o[AI_OBS_TRANSFER] = P.m_atom * sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
  o[AI_OBS_POSITION] = L.position;
  o[AI_OBS_DIST] = sqrt(dx * dx + dy * dy + dz * dz);
  o[AI_OBS_KE] = P.half_mi * (y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
  o[AI_OBS_RMIN] = sqrt(L.rmin2);
  o[AI_OBS_HNEXT] = L.absh;
#pragma unroll
  for (int c = 0; c < AI_NOBS; ++c) obs[c * P.ld + idx] = o[c];
}

// One trajectory per lane; the grid covers n.
__global__ __launch_bounds__(BLOCK) void ai_plain_kernel(Launch P, const double* __restrict__ y0,
                                                         double* __restrict__ yf,
                                                         double* __restrict__ obs) {
  const long long idx = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= P.n) return;
  Lane L;
  start(P, y0, idx, L);
  while (L.status == 0) {
    if (L.fresh) begin_step(P, L);
    attempt(P, L);
  }
  finish(P, L, idx, yf, obs);
}

__global__ void ai_queue_reset_kernel(unsigned long long* queue) { *queue = 0ull; }

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Resident waves; lanes whose trajectory has ended take new indices from the
// device queue.  Indices below P.first_dynamic are assigned statically (lane
// i of the grid starts trajectory i), the rest in order of request.
__global__ __launch_bounds__(BLOCK) void ai_persistent_kernel(Launch P,
                                                              const double* __restrict__ y0,
                                                              double* __restrict__ yf,
                                                              double* __restrict__ obs,
                                                              unsigned long long* queue) {
  long long idx = (long long)blockIdx.x * BLOCK + threadIdx.x;
  Lane L;
  bool busy = false;
  if (idx < P.n) {
    start(P, y0, idx, L);
    busy = (L.status == 0);
    if (!busy) finish(P, L, idx, yf, obs);
  }
  bool exhausted = P.first_dynamic >= P.n;  // wave-uniform

  for (;;) {
    if (!exhausted) {
      const unsigned long long idle = __ballot(!busy);
      if (idle) {
        // one atomic per wave hands out as many indices as the wave has idle lanes
        const int cnt = __popcll(idle);
        const int leader = __ffsll((unsigned long long)idle) - 1;
        unsigned long long base = 0;
        if ((int)(threadIdx.x % WAVE) == leader) base = atomicAdd(queue, (unsigned long long)cnt);
        base = __shfl(base, leader, WAVE);
        const long long first = P.first_dynamic + (long long)base;
        if (!busy) {
          const long long mine = first + lanes_below(idle);
          if (mine < P.n) {
            idx = mine;
            start(P, y0, idx, L);
            busy = (L.status == 0);
            if (!busy) finish(P, L, idx, yf, obs);
          }
        }
        if (first + cnt >= P.n) exhausted = true;
      }
    }
    if (__ballot(busy) == 0ull) {
      if (exhausted) break;
      continue;
    }
    if (busy) {
      if (L.fresh) begin_step(P, L);
      attempt(P, L);
      if (L.status != 0) {
        finish(P, L, idx, yf, obs);
        busy = false;
      }
    }
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
  int persistent_blocks_per_cu = 0;
  hipFuncAttributes plain_attr{};
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
    if ((e = hipFuncGetAttributes(&f.persistent_attr, (const void*)ai_persistent_kernel)) != hipSuccess)
      return hip_fail(e, "hipFuncGetAttributes(persistent)");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.plain_blocks_per_cu,
                                                          ai_plain_kernel, BLOCK, 0)) != hipSuccess)
      return hip_fail(e, "occupancy(plain)");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.persistent_blocks_per_cu,
                                                          ai_persistent_kernel, BLOCK, 0)) != hipSuccess)
      return hip_fail(e, "occupancy(persistent)");
    if (f.persistent_blocks_per_cu < 1) f.persistent_blocks_per_cu = 1;
    f.ready = true;
  }
  *out = &f;
  return AI_OK;
}

int validate(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
             double tmax, double rtol, double atol, const double* yf, const double* obs,
             int32_t kernel) {
  if (!p) return fail(AI_EINVAL, "params is NULL");
  if (n < 0) return fail(AI_EINVAL, "n = %lld < 0", (long long)n);
  if (ld < n) return fail(AI_EINVAL, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (kernel != AI_KERNEL_PLAIN && kernel != AI_KERNEL_PERSISTENT)
    return fail(AI_EINVAL, "unknown kernel %d", kernel);
  if (!finite_params(p)) return fail(AI_EINVAL, "non-finite system constant");
  if (!(p->m_ion > 0.0) || !(p->m_atom > 0.0)) return fail(AI_EINVAL, "masses must be > 0");
  if (p->n < 1 || p->n >= p->m) return fail(AI_EINVAL, "need 1 <= n < m");
  if (p->hmax < 0.0 || p->r_exit < 0.0 || p->r_bounce < 0.0)
    return fail(AI_EINVAL, "hmax, r_exit and r_bounce must be >= 0");
  if (p->max_steps < 1) return fail(AI_EINVAL, "max_steps must be >= 1");
  if (!std::isfinite(t0) || !std::isfinite(tmax) || !(tmax > t0))
    return fail(AI_EINVAL, "need finite t0 < tmax");
  if (!std::isfinite(rtol) || !(rtol > 0.0) || !std::isfinite(atol) || !(atol > 0.0))
    return fail(AI_EINVAL, "rtol and atol must be finite and > 0");
  if (p->n != 4 || p->m != 8)
    return fail(AI_EUNSUPPORTED, "exponents n=%d, m=%d: this build integrates n=4, m=8",
                p->n, p->m);
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
  if (!on_current_device(y0, dev) || !on_current_device(yf, dev) || !on_current_device(obs, dev))
    return fail(AI_EINVAL, "y0, final_state and obs must be device memory of the current device");
  return AI_OK;
}

Launch launch_constants(const ai_params* p, int64_t n, int64_t ld, double t0, double tmax,
                        double rtol, double atol) {
  Launch P;
  const double w2 = p->omega_rf * p->omega_rf / 4.0;
  P.inv_mi = 1.0 / p->m_ion;
  P.inv_ma = 1.0 / p->m_atom;
  P.nCn = p->n * p->Cn;
  P.mCm = p->m * p->Cm;
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
  P.thr = atol / rtol;
  P.hinit_den = 0.8 * std::pow(rtol, 0.2);
  P.max_steps = p->max_steps;
  P.n = n;
  P.ld = ld;
  P.first_dynamic = 0;
  P.exit_on = p->r_exit > 0.0;
  return P;
}

}  // namespace

extern "C" {

int ai_version(void) { return 1; }
int ai_nobs(void) { return AI_NOBS; }
const char* ai_last_error(void) { return g_error.c_str(); }

int ai_get_kernel_info(int32_t kernel, ai_kernel_info* info) {
  if (!info) return fail(AI_EINVAL, "info is NULL");
  if (kernel != AI_KERNEL_PLAIN && kernel != AI_KERNEL_PERSISTENT)
    return fail(AI_EINVAL, "unknown kernel %d", kernel);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  DeviceFacts* f = nullptr;
  int rc = device_facts(dev, &f);
  if (rc != AI_OK) return rc;
  const hipFuncAttributes& a = kernel == AI_KERNEL_PLAIN ? f->plain_attr : f->persistent_attr;
  const int bpc = kernel == AI_KERNEL_PLAIN ? f->plain_blocks_per_cu : f->persistent_blocks_per_cu;
  info->block_threads = BLOCK;
  info->vgprs = a.numRegs;
  info->spill_bytes = (int32_t)a.localSizeBytes;
  info->blocks_per_cu = bpc;
  info->waves_per_simd = bpc * (BLOCK / WAVE) / 4;
  info->compute_units = f->cus;
  info->persistent_blocks = (int64_t)f->cus * f->persistent_blocks_per_cu;
  return AI_OK;
}

int ai_integrate_async(const ai_params* p, const double* y0, int64_t n, int64_t ld, double t0,
                       double tmax, double rtol, double atol, double* final_state, double* obs,
                       int32_t kernel, void* stream) {
  g_error.clear();
  int rc = validate(p, y0, n, ld, t0, tmax, rtol, atol, final_state, obs, kernel);
  if (rc != AI_OK) return rc;
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

  if (kernel == AI_KERNEL_PLAIN) {
    const long long blocks = (n + BLOCK - 1) / BLOCK;
    if (blocks > 0x7fffffffLL) return fail(AI_EINVAL, "n too large for one launch");
    hipLaunchKernelGGL(ai_plain_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P, y0,
                       final_state, obs);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch(plain)");
    return warn;
  }

  long long blocks = (long long)f->cus * f->persistent_blocks_per_cu;
  const long long need = (n + BLOCK - 1) / BLOCK;
  if (blocks > need) blocks = need;
  P.first_dynamic = blocks * BLOCK;
  unsigned long long* queue = nullptr;
  if ((e = hipMallocAsync((void**)&queue, sizeof(unsigned long long), s)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(AI_ENOMEM, "hipMallocAsync(queue): %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(ai_queue_reset_kernel, dim3(1), dim3(1), 0, s, queue);
  if ((e = hipGetLastError()) != hipSuccess) {
    (void)hipFreeAsync(queue, s);
    return hip_fail(e, "launch(queue reset)");
  }
  hipLaunchKernelGGL(ai_persistent_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, P, y0,
                     final_state, obs, queue);
  if ((e = hipGetLastError()) != hipSuccess) {
    (void)hipFreeAsync(queue, s);
    return hip_fail(e, "launch(persistent)");
  }
  if ((e = hipFreeAsync(queue, s)) != hipSuccess) return hip_fail(e, "hipFreeAsync(queue)");
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

}  // extern "C"
