// schedule.h -- ordering of an ensemble for the integration kernels (internal
// to libai.so; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Enqueue on `stream` the construction of a permutation of 0 .. n-1 that
// lists trajectories by decreasing predicted duration: the time the atom
// needs, at its initial speed, to cross a sphere whose radius is its initial
// distance from the ion (2 r / |v_atom|), capped at `horizon`; with
// by_speed = false every trajectory is predicted to last `horizon`.  The
// permutation (n unsigned ints, device memory) is returned in *order and the
// predicted durations in the same (decreasing) order in *key; both live
// inside *workspace, which the caller releases with hipFreeAsync on the same
// stream once the consumer has been enqueued.  Needs n < 2^32.
hipError_t ai_longest_first_order(const double* y0, int64_t n, int64_t ld, double horizon,
                                  bool by_speed, unsigned** order, float** key,
                                  void** workspace, hipStream_t stream);
