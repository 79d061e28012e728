// internal.h -- declarations shared by the library's sources (not part of the
// C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "ai.h"

// Validate one request as ai_integrate validates its arguments: AI_OK,
// AI_WRTOL (rtol below 100 eps will be raised) or a negative ai_rc with the
// text in ai_last_error().  host_ok: the buffers may also be host memory.
int ai_check_request(const ai_batch_item* item, int32_t kernel, bool host_ok = false);

// Set the calling thread's ai_last_error() text and return rc.
int ai_fail(int rc, const char* msg);

// ---- Resident serving kernel (ai.hip) and its host runtime (server.hip) ----
//
// The host publishes requests by copies on one stream, in order: a request's
// initial states into the server's device slab, its descriptor into a ring of
// descriptors in device memory, then the new request count into a device
// word; the kernel's resident waves claim trajectories of the oldest published
// request that has work left, integrate them from the slab into it, and
// signal a request's completion by writing its number + 1 into done_seq[slot]
// (host-coherent memory, the only host memory the kernel touches).  Device
// memory also holds the current-request word and, per ring slot, a claim
// counter (request << 32 | claimed, set by the publication) and the
// cumulative count of finished trajectories.

#include <stdint.h>

constexpr int AI_RESIDENT_DESC_WORDS = 64;  // 512-byte descriptors
struct ai_resident_desc {
  uint64_t w[AI_RESIDENT_DESC_WORDS];       // filled by ai_resident_describe
};

struct ai_resident_args {
  const ai_resident_desc* desc;  // device: ring of `ring` descriptors
  const uint64_t* pub;           // device: requests published so far
  const uint64_t* stop;          // device: nonzero: waves exit once idle
  uint64_t* done_seq;            // host-coherent: per slot, last completed request + 1
  uint64_t* cur;                 // device: oldest request that may have work left (zero at first)
  uint64_t* claimed;             // device: per slot, request << 32 | trajectories claimed
  uint64_t* done_cnt;            // device: per slot, finished trajectories (cumulative)
  int32_t ring;                  // descriptor slots
  int32_t refill_min;            // free lanes a busy wave gathers before refilling
  int64_t idle_ticks;            // idle time (100 MHz clock) after which a wave exits
};

// Fill *out for request number seq of the ring: the item's launch constants
// with y0, final state and observables in the slab at y0s, fins, obss (planes
// of ld >= n doubles), and the done count of its slot on completion.  kernel:
// AI_KERNEL_PLAIN, optionally | AI_FP32_STAGES.
void ai_resident_describe(const ai_batch_item* item, int32_t kernel, double* y0s, double* fins,
                          double* obss, int64_t ld, uint64_t seq, uint64_t done_target,
                          const unsigned* order, ai_resident_desc* out);

// Requests of at least this many trajectories, published while the resident
// kernel is not running, are taken longest predicted first (the order of the
// single-ensemble schedule); others in index order.
constexpr int64_t AI_RESIDENT_ORDER_MIN = 4096;

// Enqueue on s the longest-first order of the item's trajectories, whose
// initial states are at y0 (planes of ld): *order receives the permutation
// (device memory, valid once the work on s has run) and *ws the allocation
// that holds it, to be released with hipFreeAsync once the request has
// completed.  AI_OK or a negative ai_rc.
int ai_resident_order(const ai_batch_item* item, const double* y0, int64_t ld, hipStream_t s,
                      const unsigned** order, void** ws);

// Launch the resident kernel on s with one wave per resident slot of the
// device; *waves receives the grid size.  AI_OK or a negative ai_rc.
int ai_resident_launch(const ai_resident_args* a, hipStream_t s, int64_t* waves);
