// schedule.h -- ordering of an ensemble for the integration kernels (internal
// to libai.so; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Samples per RF period of the cost prediction's exit search.
constexpr int AI_ORDER_SAMPLES = 8;
// Longest span the exit search covers, in RF periods; a trajectory that has
// not ended by then is predicted from its straight-line exit time.
constexpr int AI_ORDER_MAX_PERIODS = 256;
// Resolution of the sort key: costs are ordered on 2^AI_ORDER_CODE_BITS
// levels between 0 and the largest possible cost (the horizon's), 1/4096 of
// the integration span, which is far finer than the predictions are good for.
constexpr int AI_ORDER_CODE_BITS = 12;
constexpr unsigned AI_ORDER_CODES = 1u << AI_ORDER_CODE_BITS;

// What the cost prediction knows of an ensemble's system.  Two predictions
// of a trajectory's duration:
//  - analytic: the time at which the atom, on a straight line at its initial
//    velocity, is r_exit away from the ion on its secular orbit (Newton steps
//    from the straight-line exit from the sphere about the trap centre), plus
//    the span a close pass costs (below);
//  - sampled: the exit rule itself, evaluated on AI_ORDER_SAMPLES samples per
//    RF period of a model in which only the trap acts: the atom flies in a
//    straight line and the ion follows the trap's linear equation of motion
//    exactly, through the matrices that map its (x, v) at the start of an RF
//    period to the samples inside the period and to the start of the next.
//    It also predicts the trajectories that end at once (the ion's motion
//    carries the pair apart across r_exit right after t0), which the analytic
//    prediction misses, and Mathieu-unstable traps.
// Within one ensemble the launch time is set by its longest trajectories,
// which both predict alike; the analytic one is cheaper.  Across ensembles
// of different systems the packing of lanes dominates and needs the sampled
// one.
// A close pass costs the integrator extra attempts at short range that its
// duration does not show: over the 2^20-trajectory thermal Li + Yb+ ensemble,
// trajectories whose atom passes within 500 a0 of the ion's secular orbit
// took up to ~250 attempts (8 RF periods' worth) more than their duration
// predicts, fading to none beyond 2000 a0.  The analytic prediction adds that
// span for a close pass, tapered linearly between the two radii (a generous
// estimate: starting such a trajectory early costs little, starting it late
// can end the launch late).  The sampled prediction adds it too.
constexpr double AI_ORDER_CLOSE_R_IN = 500.0;    // a0
constexpr double AI_ORDER_CLOSE_R_OUT = 2000.0;  // a0
constexpr double AI_ORDER_CLOSE_PERIODS = 8.0;   // RF periods

struct ai_order_model {
  float horizon;   // tmax - t0
  float close_span;  // AI_ORDER_CLOSE_PERIODS RF periods (0 for a static trap)
  float r_exit2;   // sampled: r_exit^2 (1 + 2^-12)
  float dt;        // sampled: sample spacing, one RF period / AI_ORDER_SAMPLES
  int periods;     // sampled: periods searched, min(ceil(horizon / period), AI_ORDER_MAX_PERIODS)
  float rate;      // relative attempts per unit time (orders keys across ensembles)
  int sampled;     // 1: sampled prediction, 0: analytic
  double r_exit;   // 0: every trajectory lasts `horizon`
  double secular_omega[3];            // analytic: (Omega/2) sqrt(a_k + q_k^2 / 2), 0 if imaginary
  float phi[3][AI_ORDER_SAMPLES][2];  // sampled, per axis: x at sample j + 1 = phi[j][0] x + phi[j][1] v
  float mono[3][4];                   // sampled, per axis: (x, v) one period on = [[0] [1]; [2] [3]] (x, v)
};

// The model of a system with trap parameters a, q (paper form, per axis),
// angular RF frequency omega_rf, exit radius r_exit, span t0 .. tmax and
// relative tolerance rtol, for the sampled or the analytic prediction (host
// code).
ai_order_model ai_make_order_model(const double a[3], const double q[3], double omega_rf,
                                   double r_exit, double t0, double tmax, double rtol,
                                   bool sampled);

// Enqueue on `stream` the construction of a permutation of 0 .. n-1 that
// lists trajectories by decreasing predicted cost, rate x duration (capped at
// the horizon).  The sampled duration is the first sample at which the
// atom-ion distance has passed a local minimum (or was growing at t0) and
// exceeds r_exit: the exit rule of the integration, with a margin.  A
// distance that only grazes r_exit between two samples may not do so at any
// of the integrator's steps, and predicting such a trajectory to end at once,
// when it then runs a full collision, starts its longest work last; the
// margin makes grazing cases long instead, which costs little.  The
// permutation (n unsigned ints, device memory) is returned in *order and the
// predicted costs in the same (decreasing) order in *key; both live inside
// *workspace, which the caller releases with hipFreeAsync on the same stream
// once the consumer has been enqueued.  The keys are the costs' codes
// (AI_ORDER_CODES levels up to horizon x rate), equal codes in no fixed order.
// Needs n < 2^32.  With ext (device memory of ext_bytes, at least
// ai_order_workspace_bytes(n), 256-byte aligned) the work uses that buffer
// instead, allocates nothing and leaves *workspace NULL; the buffer must stay
// untouched until the consumer of *order and *key has run.
hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld,
                                  const ai_order_model& model, unsigned** order, unsigned** key,
                                  void** workspace, hipStream_t stream, void* ext = nullptr,
                                  size_t ext_bytes = 0);

// Bytes of the workspace ai_longest_first_order needs for n trajectories (0
// if n is out of range).
size_t ai_order_workspace_bytes(int64_t n, hipStream_t stream);

// One ensemble of a batched ordering: its initial states and what the
// prediction needs; its trajectories hold the global indices
// offset .. offset + n - 1 (offsets increasing with the item).
struct ai_order_item {
  const double* y0;
  long long ld, offset, n;
  ai_order_model model;
};

// As ai_longest_first_order over the concatenation of `count` ensembles
// (items: device memory, read by the enqueued work; total = sum of n), with
// codes up to cost_max (the largest horizon x rate of the items); the
// permutation lists global indices.
hipError_t ai_longest_first_order_batch(const ai_order_item* items, int count, int64_t total,
                                        double cost_max, unsigned** order, unsigned** key,
                                        void** workspace, hipStream_t stream);
