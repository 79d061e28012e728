// server.hip -- a stream of integration requests served by batched launches
// (the ai_server_* entry points of ai.h; host code only).
//
// Each of the server's workers owns a stream and a thread.  A worker whose
// previous launch has completed takes every queued request, in arrival order,
// up to max_batch trajectories, into one ai_integrate_batch_async call on its
// stream.  Requests that arrive while launches run therefore share the next
// one, a launch never waits for more requests to arrive, and with several
// workers a new launch fills the SIMDs that the tail of an earlier one (its
// longest trajectories) leaves idle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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
};

using RequestPtr = std::shared_ptr<Request>;

}  // namespace

struct ai_server {
  int device = 0;
  int64_t max_batch = 0;
  int32_t schedule = 0;
  std::vector<hipStream_t> streams;  // one per worker
  std::vector<std::thread> workers;

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

// Let the workers finish what is queued, join them and release the streams.
void ai_server::stop() {
  {
    std::lock_guard<std::mutex> lock(mu);
    stopping = true;
  }
  work.notify_all();
  for (std::thread& t : workers)
    if (t.joinable()) t.join();
  for (hipStream_t st : streams) (void)hipStreamDestroy(st);
  workers.clear();
  streams.clear();
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
  std::unique_ptr<ai_server> s(new (std::nothrow) ai_server);
  if (!s) return ai_fail(AI_ENOMEM, "server");
  s->max_batch = c.max_batch > 0 ? c.max_batch : (int64_t)1 << 22;
  s->schedule = c.schedule;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return ai_fail(AI_EHIP, hipGetErrorString(e));
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
  const int rc = ai_check_request(item, kernel);
  if (rc < 0) return rc;
  auto r = std::make_shared<Request>();
  r->item = *item;
  r->kernel = kernel;
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
