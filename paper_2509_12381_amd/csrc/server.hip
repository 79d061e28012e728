// server.hip -- a stream of integration requests (the ai_server_* entry
// points of ai.h; host code only).
//
// Resident mode (continuous batching): one dispatcher thread admits requests
// in arrival order by footprint against the server's device slab, copies the
// initial states of requests whose buffers are host memory into the slab on a
// stream of its own (device buffers are integrated in place), publishes each
// request to the resident kernel (ai.hip) by copying its descriptor from a
// pinned staging ring into a ring of descriptors in device memory and then the
// new request count into a device word, keeps the kernel running (relaunching
// it after it has exited for lack of work), watches the completion words the
// kernel writes into host-coherent memory, copies staged results out on a
// second stream and frees the slab space.
//
// Launch mode: each of the server's workers owns a stream and a thread.  A
// worker whose previous launch has completed takes every queued request, in
// arrival order, up to max_batch trajectories, into one
// ai_integrate_batch_async call on its stream.  Requests that arrive while
// launches run therefore share the next one, a launch never waits for more
// requests to arrive, and with several workers a new launch fills the SIMDs
// that the tail of an earlier one (its longest trajectories) leaves idle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ai.h"
#include "internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  ai_batch_item item;
  int32_t kernel = 0;
  int base_rc = AI_OK;  // AI_OK or AI_WRTOL from validation
  ai_request_info info{};
  bool done = false;
  // resident mode
  size_t slab_off = 0, slab_len = 0;
  bool staged = false;  // buffers in host memory: integrated from and into the slab
  uint64_t seq = 0;
  hipEvent_t copied_in = nullptr, copied_out = nullptr;
  void* order_ws = nullptr;  // the request's longest-first order (stream-ordered allocation)
};

// Footprint of a request of n trajectories: initial states, final states and
// observables, each plane rounded up to 256 bytes.  Every admitted request
// holds that much of the server's budget; one whose buffers are in host
// memory is integrated from and into that region of the slab, one whose
// buffers are device memory of the server's device in place.
size_t plane_bytes(int64_t n) { return ((size_t)n * 8 + 255) & ~size_t(255); }
size_t footprint(int64_t n) { return (12 + 12 + AI_NOBS) * plane_bytes(n); }

// First-fit allocator over [0, size) of the slab.
struct SlabSpace {
  std::map<size_t, size_t> free;  // offset -> length
  void reset(size_t size) {
    free.clear();
    if (size) free[0] = size;
  }
  bool take(size_t len, size_t& off) {
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second < len) continue;
      off = it->first;
      const size_t rest = it->second - len;
      free.erase(it);
      if (rest) free[off + len] = rest;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t len) {
    auto next = free.lower_bound(off);
    if (next != free.end() && off + len == next->first) {
      len += next->second;
      next = free.erase(next);
    }
    if (next != free.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free[off] = len;
  }
};

// Whether a buffer is device memory of the current device (else host memory).
bool on_device(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  int dev = -1;
  return attr.type == hipMemoryTypeDevice && hipGetDevice(&dev) == hipSuccess &&
         attr.device == dev;
}

using RequestPtr = std::shared_ptr<Request>;

}  // namespace

struct ai_server {
  int device = 0;
  int32_t mode = AI_SERVE_LAUNCHES;
  int64_t max_batch = 0;
  int32_t schedule = 0;
  std::vector<hipStream_t> streams;  // launches: one per worker; resident: kernel, in, out
  std::vector<std::thread> workers;  // launches: workers; resident: the dispatcher

  // resident mode
  int32_t ring = 0;
  int32_t refill_min = 8;
  double idle_ms = 20.0;
  size_t slab_bytes = 0;
  char* slab = nullptr;                 // device
  // host-coherent: [8, 8 + ring) completion words done_seq[slot] (the kernel
  // writes them), [8 + ring, 8 + 2 ring) the request count and
  // [8 + 2 ring, 8 + 3 ring) the claim counter each publication copies to the
  // device, [1] the stop word's source
  uint64_t* ctl = nullptr;
  ai_resident_desc* desc = nullptr;     // pinned: descriptors, copied to dev_ring
  uint64_t* dev_ctl = nullptr;          // ctl as the device addresses it
  ai_resident_desc* dev_ring = nullptr; // device: ring of descriptors
  uint64_t* dev_words = nullptr;        // device: cur, pub, stop, done_cnt[ring] from word 8,
                                        // claimed[ring] after it
  bool broken = false;                  // dispatcher: a publication failed; refuse the rest
  hipEvent_t kernel_done = nullptr;
  bool kernel_running = false;
  int64_t launches = 0;
  SlabSpace space;                      // guarded by mu
  std::vector<uint64_t> slot_total;     // dispatcher: cumulative done target per slot
  std::vector<char> slot_busy;          // guarded by mu
  uint64_t next_seq = 0;                // guarded by mu

  std::mutex mu;
  std::condition_variable work;  // a request was queued, or stop
  std::condition_variable done;  // a launch completed
  std::deque<RequestPtr> queue;
  std::unordered_map<uint64_t, RequestPtr> held;  // submitted and not yet waited for
  uint64_t next_ticket = 1;
  int64_t next_batch = 0;
  bool stopping = false;

  void run(hipStream_t stream);
  void serve(std::vector<RequestPtr>& batch, hipStream_t stream);
  void dispatch();
  int start_resident(const ai_server_config& c);
  void release_resident();
  void finish(const RequestPtr& r, int rc, const std::string& error);
  void stop();
};

namespace {

// A request the batched kernel does not run: single-precision stages, or a
// potential with exponents other than n = 4, m = 8.
bool runs_alone(const Request& r) {
  return (r.kernel & AI_FP32_STAGES) || r.item.params.n != 4 || r.item.params.m != 8;
}

// Take the next launch's requests from the front of the queue (lock held): a
// request that runs alone, else batchable requests in order while they fit.
std::vector<RequestPtr> take_batch(std::deque<RequestPtr>& queue, int64_t max_batch) {
  std::vector<RequestPtr> batch;
  if (queue.empty()) return batch;
  if (runs_alone(*queue.front())) {
    batch.push_back(queue.front());
    queue.pop_front();
    return batch;
  }
  int64_t total = 0;
  while (!queue.empty()) {
    const RequestPtr& r = queue.front();
    if (runs_alone(*r)) break;
    if (!batch.empty() && total + r->item.n > max_batch) break;
    total += r->item.n;
    batch.push_back(r);
    queue.pop_front();
  }
  return batch;
}

}  // namespace

void ai_server::serve(std::vector<RequestPtr>& batch, hipStream_t stream) {
  const double start = now_s();
  int64_t trajectories = 0;
  for (const RequestPtr& r : batch) trajectories += r->item.n;
  int rc;
  if (batch.size() == 1 && runs_alone(*batch[0])) {
    const ai_batch_item& it = batch[0]->item;
    rc = ai_integrate_async(&it.params, it.y0, it.n, it.ld, it.t0, it.tmax, it.rtol, it.atol,
                            it.final_state, it.obs, batch[0]->kernel | schedule, stream);
  } else {
    std::vector<ai_batch_item> items;
    items.reserve(batch.size());
    for (const RequestPtr& r : batch) items.push_back(r->item);
    rc = ai_integrate_batch_async(items.data(), (int32_t)items.size(), schedule, stream);
  }
  std::string error;
  if (rc >= 0) {
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      rc = AI_EHIP;
      error = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    }
  } else {
    error = ai_last_error();
  }
  const double end = now_s();
  std::lock_guard<std::mutex> lock(mu);
  const int64_t id = next_batch++;
  for (const RequestPtr& r : batch) {
    ai_request_info& in = r->info;
    in.rc = rc < 0 ? rc : r->base_rc;
    in.batch_size = (int32_t)batch.size();
    in.batch_id = id;
    in.batch_trajectories = trajectories;
    in.start_s = start;
    in.end_s = end;
    std::strncpy(in.error, error.c_str(), sizeof in.error - 1);
    in.error[sizeof in.error - 1] = '\0';
    r->done = true;
  }
  done.notify_all();
}

void ai_server::run(hipStream_t stream) {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<RequestPtr> batch;
    {
      std::unique_lock<std::mutex> lock(mu);
      work.wait(lock, [&] { return stopping || !queue.empty(); });
      if (queue.empty()) return;  // stopping, and everything queued has been taken
      batch = take_batch(queue, max_batch);
    }
    serve(batch, stream);
  }
}

// Complete a resident request (any thread but the caller's lock-holders).
void ai_server::finish(const RequestPtr& r, int rc, const std::string& error) {
  if (r->copied_in) (void)hipEventDestroy(r->copied_in);
  if (r->copied_out) (void)hipEventDestroy(r->copied_out);
  r->copied_in = r->copied_out = nullptr;
  // the kernel reads a request's order only before its last trajectory is
  // counted done, so it is released once the completion has been seen
  if (r->order_ws) (void)hipFreeAsync(r->order_ws, streams[2]);
  r->order_ws = nullptr;
  const double end = now_s();
  std::lock_guard<std::mutex> lock(mu);
  if (r->slab_len) {
    space.give(r->slab_off, r->slab_len);
    slot_busy[r->seq % ring] = 0;
    r->slab_len = 0;
  }
  ai_request_info& in = r->info;
  in.rc = rc < 0 ? rc : r->base_rc;
  in.end_s = end;
  std::strncpy(in.error, error.c_str(), sizeof in.error - 1);
  in.error[sizeof in.error - 1] = '\0';
  r->done = true;
  done.notify_all();
}

// The resident mode's dispatcher: admission by footprint, copy-in,
// publication, kernel (re)launch, completion, copy-out.
void ai_server::dispatch() {
  (void)hipSetDevice(device);
  hipStream_t kstream = streams[0], in_stream = streams[1], out_stream = streams[2];
  uint64_t* stop_src = ctl + 1;
  uint64_t* done_seq = ctl + 8;
  uint64_t* pub_src = ctl + 8 + ring;
  uint64_t* claim_src = ctl + 8 + 2 * (size_t)ring;
  std::deque<RequestPtr> staging, running, draining;
  ai_resident_args args{};
  args.desc = dev_ring;
  args.pub = dev_words + 1;
  args.stop = dev_words + 2;
  args.done_seq = dev_ctl + 8;
  args.cur = dev_words;
  args.done_cnt = dev_words + 8;
  args.claimed = dev_words + 8 + ring;
  args.ring = ring;
  args.refill_min = refill_min;
  args.idle_ticks = (int64_t)(idle_ms * 1e5);  // 100 MHz clock
  int64_t in_flight_traj = 0;
  // a burst of submissions is published whole before a launch: the kernel is
  // launched once no request has been admitted for LAUNCH_QUIET_S, once the
  // first published request has waited LAUNCH_WAIT_S, or at once when queued
  // requests cannot be admitted (the budget or the ring is full)
  constexpr double LAUNCH_QUIET_S = 1e-3, LAUNCH_WAIT_S = 0.05;
  double last_admit_s = 0.0, waiting_since_s = -1.0;
  bool admission_blocked = false;

  auto hip_error = [](hipError_t e, const char* what) {
    (void)hipGetLastError();
    return std::string(what) + ": " + hipGetErrorString(e);
  };

  for (;;) {
    bool progress = false;
    // admit queued requests, in order, while their footprint fits and a ring
    // slot is free
    std::vector<RequestPtr> admit;
    {
      std::lock_guard<std::mutex> lock(mu);
      while (!queue.empty()) {
        const RequestPtr& r = queue.front();
        if (slot_busy[next_seq % ring]) break;
        size_t off = 0;
        const size_t len = footprint(r->item.n);
        if (!space.take(len, off)) break;
        r->slab_off = off;
        r->slab_len = len;
        r->seq = next_seq++;
        slot_busy[r->seq % ring] = 1;
        admit.push_back(r);
        queue.pop_front();
      }
      admission_blocked = !queue.empty();
      if (admit.empty() && queue.empty() && staging.empty() && running.empty() &&
          draining.empty() && stopping)
        break;
    }
    if (!admit.empty()) last_admit_s = now_s();
    // publication, in request order on the copy stream: the initial states
    // into the slab (host-memory requests), the descriptor into the device
    // ring, the slot's claim counter (request << 32), then the new
    // request count into the device word the kernel reads; the kernel sees a
    // request only once all of it is in device memory and never reads host
    // memory for it
    // the order's kernels, like the copies, wait for compute units while the
    // kernel's waves live: a request published to a running kernel is taken
    // in index order, one published while it is down longest first
    const bool kernel_alive = kernel_running && hipEventQuery(kernel_done) == hipErrorNotReady;
    for (const RequestPtr& r : admit) {
      const ai_batch_item& it = r->item;
      const size_t pb = plane_bytes(it.n);
      double* y0s = (double*)(slab + r->slab_off);
      const uint32_t slot = (uint32_t)(r->seq % ring);
      if (broken) {
        finish(r, AI_EHIP, "an earlier publication failed");
        continue;
      }
      slot_total[slot] += (uint64_t)it.n;
      pub_src[slot] = r->seq + 1;
      claim_src[slot] = r->seq << 32;
      hipError_t e = hipEventCreateWithFlags(&r->copied_in, hipEventDisableTiming);
      if (e == hipSuccess && r->staged)
        e = hipMemcpy2DAsync(y0s, pb, it.y0, (size_t)it.ld * 8, (size_t)it.n * 8, 12,
                             hipMemcpyDefault, in_stream);
      // a large request's trajectories are taken longest predicted first: its
      // order is computed on the copy stream from the initial states the
      // kernel will read, before the descriptor that points to it
      const double* y0_dev = r->staged ? y0s : it.y0;
      const int64_t ld_dev = r->staged ? (int64_t)(pb / 8) : it.ld;
      const unsigned* order = nullptr;
      if (e == hipSuccess && it.n >= AI_RESIDENT_ORDER_MIN && !kernel_alive &&
          ai_resident_order(&it, y0_dev, ld_dev, in_stream, &order, &r->order_ws) != AI_OK) {
        broken = true;
        (void)hipStreamSynchronize(in_stream);
        finish(r, AI_EHIP, ai_last_error());
        continue;
      }
      if (r->staged)
        ai_resident_describe(&it, r->kernel, y0s, y0s + 12 * pb / 8, y0s + 24 * pb / 8,
                             (int64_t)(pb / 8), r->seq, slot_total[slot], order, &desc[slot]);
      else
        ai_resident_describe(&it, r->kernel, const_cast<double*>(it.y0), it.final_state, it.obs,
                             it.ld, r->seq, slot_total[slot], order, &desc[slot]);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dev_ring + slot, desc + slot, sizeof(ai_resident_desc),
                           hipMemcpyHostToDevice, in_stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dev_words + 8 + ring + slot, claim_src + slot, sizeof(uint64_t),
                           hipMemcpyHostToDevice, in_stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dev_words + 1, pub_src + slot, sizeof(uint64_t),
                           hipMemcpyHostToDevice, in_stream);
      if (e == hipSuccess) e = hipEventRecord(r->copied_in, in_stream);
      if (e != hipSuccess) {
        // a request count that never arrives would stall every later request:
        // the server refuses the rest
        broken = true;
        (void)hipStreamSynchronize(in_stream);
        finish(r, AI_EHIP, hip_error(e, "publish"));
        continue;
      }
      staging.push_back(r);
      progress = true;
    }
    // published requests (their copies have completed), in order
    std::vector<RequestPtr> fresh;
    while (!staging.empty()) {
      const RequestPtr r = staging.front();
      const hipError_t q = hipEventQuery(r->copied_in);
      if (q == hipErrorNotReady) break;
      staging.pop_front();
      progress = true;
      if (q != hipSuccess) {
        broken = true;
        finish(r, AI_EHIP, hip_error(q, "publish"));
        continue;
      }
      const ai_batch_item& it = r->item;
      in_flight_traj += it.n;
      r->info.start_s = now_s();
      r->info.batch_size = (int32_t)(running.size() + 1);
      r->info.batch_trajectories = in_flight_traj;
      running.push_back(r);
      fresh.push_back(r);
    }
    // the kernel runs while published requests are unfinished.  Its waves
    // hold every compute unit while they live, and the runtime runs the
    // publication copies as kernels, so a launch waits until every
    // publication enqueued so far has completed: it then starts with all of
    // them in view instead of holding the rest back until its waves leave
    if (kernel_running && hipEventQuery(kernel_done) != hipErrorNotReady) kernel_running = false;
    bool launch_now = false;
    if (!running.empty() && !kernel_running && staging.empty()) {
      const double t = now_s();
      if (waiting_since_s < 0.0) waiting_since_s = t;
      launch_now = admission_blocked || t - last_admit_s >= LAUNCH_QUIET_S ||
                   t - waiting_since_s >= LAUNCH_WAIT_S;
    }
    if (launch_now) {
      waiting_since_s = -1.0;
      int64_t waves = 0;
      const int lrc = ai_resident_launch(&args, kstream, &waves);
      const hipError_t e = lrc == AI_OK ? hipEventRecord(kernel_done, kstream) : hipSuccess;
      if (lrc != AI_OK || e != hipSuccess) {
        const std::string why = lrc != AI_OK ? std::string(ai_last_error())
                                             : hip_error(e, "hipEventRecord");
        for (const RequestPtr& x : running) finish(x, AI_EHIP, why);
        running.clear();
        fresh.clear();
        in_flight_traj = 0;
      } else {
        kernel_running = true;
        launches += 1;
        progress = true;
      }
    }
    // the launch that serves them: the running one, else the next
    for (const RequestPtr& r : fresh) r->info.batch_id = kernel_running ? launches - 1 : launches;
    // completed requests: results out to the caller's buffers
    for (auto it = running.begin(); it != running.end();) {
      const RequestPtr r = *it;
      const uint32_t slot = (uint32_t)(r->seq % ring);
      if (__atomic_load_n(done_seq + slot, __ATOMIC_ACQUIRE) != r->seq + 1) {
        ++it;
        continue;
      }
      it = running.erase(it);
      progress = true;
      in_flight_traj -= r->item.n;
      if (!r->staged) {  // the results are in the caller's buffers
        finish(r, AI_OK, "");
        continue;
      }
      const ai_batch_item& itm = r->item;
      const size_t pb = plane_bytes(itm.n);
      const char* base = slab + r->slab_off;
      hipError_t e = hipEventCreateWithFlags(&r->copied_out, hipEventDisableTiming);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(itm.final_state, (size_t)itm.ld * 8, base + 12 * pb, pb,
                             (size_t)itm.n * 8, 12, hipMemcpyDefault, out_stream);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(itm.obs, (size_t)itm.ld * 8, base + 24 * pb, pb, (size_t)itm.n * 8,
                             AI_NOBS, hipMemcpyDefault, out_stream);
      if (e == hipSuccess) e = hipEventRecord(r->copied_out, out_stream);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(out_stream);  // the slab space is not reused under a copy
        finish(r, AI_EHIP, hip_error(e, "copy out"));
        continue;
      }
      draining.push_back(r);
    }
    // copied out: complete
    for (auto it = draining.begin(); it != draining.end();) {
      const hipError_t q = hipEventQuery((*it)->copied_out);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      const RequestPtr r = *it;
      it = draining.erase(it);
      progress = true;
      finish(r, q == hipSuccess ? AI_OK : AI_EHIP, q == hipSuccess ? "" : hip_error(q, "copy out"));
    }
    if (!progress) {
      std::unique_lock<std::mutex> lock(mu);
      work.wait_for(lock, std::chrono::microseconds(100));
    }
  }
  // everything is served: the waves exit once idle (at the latest after
  // idle_ms, should the stop word not arrive)
  *stop_src = 1;
  if (hipMemcpyAsync(dev_words + 2, stop_src, sizeof(uint64_t), hipMemcpyHostToDevice,
                     in_stream) == hipSuccess)
    (void)hipStreamSynchronize(in_stream);
  if (kernel_running) (void)hipEventSynchronize(kernel_done);
  kernel_running = false;
}

int ai_server::start_resident(const ai_server_config& c) {
  ring = c.ring > 0 ? c.ring : 1024;
  refill_min = c.refill_min > 0 ? c.refill_min : 8;
  idle_ms = c.idle_ms > 0.0 ? c.idle_ms : 20.0;
  slab_bytes = c.slab_bytes > 0 ? (size_t)c.slab_bytes : ((size_t)4 << 30);
  slot_total.assign(ring, 0);
  slot_busy.assign(ring, 0);
  space.reset(slab_bytes);
  hipError_t e;
  const size_t ctl_bytes = sizeof(uint64_t) * (8 + 3 * (size_t)ring);
  if ((e = hipHostMalloc((void**)&ctl, ctl_bytes, hipHostMallocCoherent | hipHostMallocMapped)) !=
          hipSuccess ||
      (e = hipHostMalloc((void**)&desc, sizeof(ai_resident_desc) * ring,
                         hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess) {
    (void)hipGetLastError();
    return ai_fail(AI_ENOMEM, "host-coherent request ring");
  }
  std::memset(ctl, 0, ctl_bytes);
  std::memset(desc, 0, sizeof(ai_resident_desc) * ring);
  if ((e = hipHostGetDevicePointer((void**)&dev_ctl, ctl, 0)) != hipSuccess)
    return ai_fail(AI_EHIP, hipGetErrorString(e));
  const size_t dev_bytes = sizeof(uint64_t) * (8 + 2 * (size_t)ring);
  if ((e = hipMalloc((void**)&dev_words, dev_bytes)) != hipSuccess ||
      (e = hipMalloc((void**)&dev_ring, sizeof(ai_resident_desc) * ring)) != hipSuccess ||
      (e = hipMalloc((void**)&slab, slab_bytes)) != hipSuccess) {
    (void)hipGetLastError();
    return ai_fail(AI_ENOMEM, "server slab");
  }
  if ((e = hipMemset(dev_words, 0, dev_bytes)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess ||
      (e = hipEventCreateWithFlags(&kernel_done, hipEventDisableTiming)) != hipSuccess)
    return ai_fail(AI_EHIP, hipGetErrorString(e));
  for (int k = 0; k < 3; ++k) {
    hipStream_t st = nullptr;  // default priority
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
      return ai_fail(AI_EHIP, hipGetErrorString(e));
    streams.push_back(st);
  }
  return AI_OK;
}

// After the dispatcher has stopped the kernel: release what start_resident took.
void ai_server::release_resident() {
  if (kernel_done) (void)hipEventDestroy(kernel_done);
  kernel_done = nullptr;
  if (slab) (void)hipFree(slab);
  if (dev_ring) (void)hipFree(dev_ring);
  if (dev_words) (void)hipFree(dev_words);
  if (desc) (void)hipHostFree(desc);
  if (ctl) (void)hipHostFree(ctl);
  slab = nullptr;
  dev_ring = nullptr;
  dev_words = nullptr;
  desc = nullptr;
  ctl = nullptr;
}

// Let the workers (or the dispatcher) finish what is queued, join them and
// release the streams.
void ai_server::stop() {
  {
    std::lock_guard<std::mutex> lock(mu);
    stopping = true;
  }
  work.notify_all();
  for (std::thread& t : workers)
    if (t.joinable()) t.join();
  if (mode == AI_SERVE_RESIDENT && kernel_running && kernel_done)
    (void)hipEventSynchronize(kernel_done);
  for (hipStream_t st : streams) (void)hipStreamDestroy(st);
  workers.clear();
  streams.clear();
  if (mode == AI_SERVE_RESIDENT) release_resident();
}

extern "C" {

int ai_server_create(const ai_server_config* cfg, ai_server** out) {
  if (!out) return ai_fail(AI_EINVAL, "out is NULL");
  *out = nullptr;
  ai_server_config c{};
  if (cfg) c = *cfg;
  if (c.max_batch < 0 || c.workers < 0 || c.workers > 16 ||
      (c.schedule != 0 && c.schedule != AI_SCHEDULE_LONGEST_FIRST))
    return ai_fail(AI_EINVAL, "config: max_batch >= 0, schedule 0 or AI_SCHEDULE_LONGEST_FIRST, "
                              "workers 0 .. 16");
  if ((c.mode != AI_SERVE_LAUNCHES && c.mode != AI_SERVE_RESIDENT) || c.ring < 0 ||
      c.ring > 65536 || c.slab_bytes < 0 || !(c.idle_ms >= 0.0) || c.idle_ms > 6e4 ||
      c.refill_min < 0 || c.refill_min > 64 || c.reserved != 0)
    return ai_fail(AI_EINVAL, "config: mode AI_SERVE_LAUNCHES or AI_SERVE_RESIDENT, ring 0 .. "
                              "65536, slab_bytes >= 0, idle_ms 0 .. 60000, refill_min 0 .. 64, "
                              "reserved 0");
  std::unique_ptr<ai_server> s(new (std::nothrow) ai_server);
  if (!s) return ai_fail(AI_ENOMEM, "server");
  s->mode = c.mode;
  s->max_batch = c.max_batch > 0 ? c.max_batch : (int64_t)1 << 22;
  s->schedule = c.schedule;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return ai_fail(AI_EHIP, hipGetErrorString(e));
  if (s->mode == AI_SERVE_RESIDENT) {
    const int rc = s->start_resident(c);
    if (rc != AI_OK) {
      const std::string why = ai_last_error();
      s->stop();
      return ai_fail(rc, why.c_str());
    }
    ai_server* raw = s.get();
    try {
      s->workers.emplace_back([raw] { raw->dispatch(); });
    } catch (...) {
      s->stop();
      return ai_fail(AI_ENOMEM, "dispatcher thread");
    }
    *out = s.release();
    return AI_OK;
  }
  const int workers = c.workers > 0 ? c.workers : 3;
  for (int w = 0; w < workers; ++w) {
    // default priority: the only stream priority these kernels are run with
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      s->stop();
      return ai_fail(AI_EHIP, hipGetErrorString(e));
    }
    s->streams.push_back(st);
    ai_server* raw = s.get();
    try {
      s->workers.emplace_back([raw, st] { raw->run(st); });
    } catch (...) {
      s->stop();
      return ai_fail(AI_ENOMEM, "worker thread");
    }
  }
  *out = s.release();
  return AI_OK;
}

int ai_server_submit(ai_server* srv, const ai_batch_item* item, int32_t kernel,
                     uint64_t* ticket) {
  if (!srv || !ticket) return ai_fail(AI_EINVAL, "server or ticket is NULL");
  *ticket = 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != srv->device)
    return ai_fail(AI_EINVAL, "submit from the server's device");
  const bool resident = srv->mode == AI_SERVE_RESIDENT;
  const int rc = ai_check_request(item, kernel, resident);
  if (rc < 0) return rc;
  if (resident) {
    if (item->params.n != 4 || item->params.m != 8)
      return ai_fail(AI_EUNSUPPORTED, "the resident kernel integrates n=4, m=8 potentials");
    if (item->n > 0xffffffffLL || footprint(item->n) > srv->slab_bytes)
      return ai_fail(AI_EINVAL, "the request does not fit in the server's slab");
  }
  auto r = std::make_shared<Request>();
  r->item = *item;
  r->kernel = kernel;
  r->staged = resident && item->n > 0 &&
              !(on_device(item->y0) && on_device(item->final_state) && on_device(item->obs));
  r->base_rc = rc;
  r->info.submit_s = now_s();
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->stopping) return ai_fail(AI_EINVAL, "server is stopping");
    *ticket = srv->next_ticket++;
    srv->held.emplace(*ticket, r);
    // an empty request needs no launch
    if (item->n == 0) {
      r->info.rc = rc;
      r->info.batch_id = -1;
      r->info.start_s = r->info.end_s = r->info.submit_s;
      r->done = true;
    } else {
      srv->queue.push_back(r);
    }
  }
  srv->work.notify_one();
  return rc;
}

int ai_server_wait(ai_server* srv, uint64_t ticket, double timeout_s, ai_request_info* info) {
  if (!srv || !info) return ai_fail(AI_EINVAL, "server or info is NULL");
  std::unique_lock<std::mutex> lock(srv->mu);
  auto it = srv->held.find(ticket);
  if (it == srv->held.end()) return ai_fail(AI_EINVAL, "unknown ticket");
  RequestPtr r = it->second;
  auto finished = [&] { return r->done; };
  if (timeout_s < 0.0) {
    srv->done.wait(lock, finished);
  } else if (!srv->done.wait_for(lock, std::chrono::duration<double>(timeout_s), finished)) {
    return AI_EAGAIN;
  }
  *info = r->info;
  srv->held.erase(ticket);
  return AI_OK;
}

int ai_server_destroy(ai_server* srv) {
  if (!srv) return ai_fail(AI_EINVAL, "server is NULL");
  srv->stop();
  delete srv;
  return AI_OK;
}

}  // extern "C"
