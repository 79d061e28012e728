// schedule.h -- ordering of an ensemble for the integration kernels (internal
// to libai.so; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Enqueue on `stream` the construction of a permutation of 0 .. n-1 that
// lists trajectories by decreasing predicted duration: the time at which the
// atom, moving in a straight line at its initial velocity, is r_exit away
// from the ion following its secular motion in the trap (angular frequency
// secular_omega[k] per axis, zero for a free ion), capped at `horizon`;
// with r_exit = 0 every trajectory is predicted to last `horizon`.  The
// permutation (n unsigned ints, device memory) is returned in *order and the
// predicted durations in the same (decreasing) order in *key; both live
// inside *workspace, which the caller releases with hipFreeAsync on the same
// stream once the consumer has been enqueued.  Needs n < 2^32.
hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld, double horizon,
                                  double r_exit, const double secular_omega[3],
                                  unsigned** order, float** key,
                                  void** workspace, hipStream_t stream);

// One ensemble of a batched ordering: its initial states and what the
// prediction needs; its trajectories hold the global indices
// offset .. offset + n - 1 (offsets increasing with the item).
struct ai_order_item {
  const double* y0;
  long long ld, offset, n;
  double horizon, r_exit;
  double secular_omega[3];
};

// As ai_longest_first_order over the concatenation of `count` ensembles
// (items: device memory, read by the enqueued work; total = sum of n); the
// permutation lists global indices.
hipError_t ai_longest_first_order_batch(const ai_order_item* items, int count, int64_t total,
                                        unsigned** order, float** key, void** workspace,
                                        hipStream_t stream);
