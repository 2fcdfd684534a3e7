// Request serving on one GPU behind the C ABI (gbs_server_* in gbs_mps.h).
//
// A request is one pure Gaussian state to convert (Sec. II) plus a number of
// photon-number samples to draw from its MPS.  Requests wait in a FIFO queue.
// `slots` worker threads, each owning one HIP stream, take the head of the
// queue as soon as they are free and the head's device-memory footprint fits
// the budget beside the requests already in service.  Admission is therefore
// continuous: a request does not wait for a batch to form or drain, and the
// kernels of up to `slots` requests (a latency-bound Gaussian SVD chain of one
// request next to the sampling GEMMs of another) share the GPU at once.
// Every temporary is a stream-ordered allocation on the worker's stream, so
// one request's frees never wait on another's kernels.  A request's results
// do not depend on what else is in service: the build is deterministic and
// the sampler's random numbers are keyed by (seed, shot, site).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gbs_internal.h"

namespace {

int sfail(int code, const std::string& msg) { return gbs_fail(code, msg); }

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  gbs_request r;
  int64_t id = 0;
  int64_t fp = 0;
  double t_submit = 0, t_start = 0, t_built = 0, t_done = 0;
  int status = GBS_OK;
  int max_bond = 0;
  double eps_max = 0;
  bool done = false;
  std::string err;
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest-rank definition
  size_t k = (size_t)std::max(1.0, std::ceil(q * (double)v.size()));
  return v[std::min(k, v.size()) - 1];
}

}  // namespace

struct gbs_server_s {
  int device = 0;
  int64_t budget = 0;
  int slots = 0;
  int max_queue = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<int64_t, Req*> recs;
  int64_t in_use = 0, peak = 0, next_id = 1;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<double> lat;
  int64_t submitted = 0, completed = 0, failed = 0;
  double t_first = -1.0, t_last = 0.0;

  void worker(int slot);
};

void gbs_server_s::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t st = streams[slot];
  for (;;) {
    Req* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        if (queue.empty()) return stop;
        return running == 0 || in_use + queue.front()->fp <= budget;
      });
      if (queue.empty()) return;  // stop requested and nothing left
      q = queue.front();
      queue.pop_front();
      in_use += q->fp;
      peak = std::max(peak, in_use);
      ++running;
    }
    q->t_start = wall_ms();
    gbs_mps h = nullptr;
    int rc = gbs_build_handle(q->r.gamma, q->r.M, &q->r.opt, st, true, &h, 0);
    q->t_built = wall_ms();
    if (rc == GBS_OK && q->r.shots > 0) rc = gbs_mps_sample(h, q->r.shots, q->r.seed, q->r.out, st);
    if (rc == GBS_OK && hipStreamSynchronize(st) != hipSuccess) {
      (void)hipGetLastError();
      rc = sfail(GBS_E_DEVICE, "HIP error while sampling");
    }
    q->t_done = wall_ms();
    if (rc != GBS_OK) q->err = gbs_last_error();
    if (h) {
      gbs_mps_info_t inf;
      if (gbs_mps_info(h, &inf, nullptr, nullptr, nullptr, nullptr) == GBS_OK) {
        q->max_bond = inf.max_bond;
        q->eps_max = inf.eps_max;
      }
      gbs_mps_free(h);  // stream-ordered release on `st`
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      in_use -= q->fp;
      --running;
      q->status = rc;
      q->done = true;
      if (rc == GBS_OK) {
        ++completed;
        lat.push_back(q->t_done - q->t_submit);
      } else {
        ++failed;
      }
      t_last = std::max(t_last, q->t_done);
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

int gbs_server_create(int32_t slots, int64_t budget_bytes, int32_t max_queue, gbs_server* out) {
  if (!out) return sfail(GBS_E_INVAL, "NULL output");
  *out = nullptr;
  if (slots < 1 || slots > 64) return sfail(GBS_E_INVAL, "slots must be in [1, 64]");
  if (budget_bytes <= 0) return sfail(GBS_E_INVAL, "budget_bytes must be > 0");
  if (max_queue < 1) return sfail(GBS_E_INVAL, "max_queue must be >= 1");
  gbs_server_s* s = new (std::nothrow) gbs_server_s();
  if (!s) return sfail(GBS_E_NOMEM, "host allocation failed");
  s->budget = budget_bytes;
  s->slots = slots;
  s->max_queue = max_queue;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return sfail(GBS_E_DEVICE, "hipGetDevice failed");
  }
  for (int i = 0; i < slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return sfail(GBS_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < slots; ++i) s->workers.emplace_back(&gbs_server_s::worker, s, i);
  *out = s;
  return GBS_OK;
}

int gbs_server_submit(gbs_server s, const gbs_request* req, int64_t* id) {
  if (!s || !req || !id) return sfail(GBS_E_INVAL, "NULL argument");
  if (!req->gamma || req->M < 1 || req->shots < 0 || (req->shots > 0 && !req->out))
    return sfail(GBS_E_INVAL, "invalid request (gamma, M, shots or out)");
  const int64_t fp = gbs_mps_footprint(req->M, &req->opt, req->shots);
  if (fp < 0) return sfail(GBS_E_INVAL, "invalid build options");
  if (fp > s->budget) return sfail(GBS_E_NOMEM, "request footprint exceeds the server's memory budget");
  Req* q = new (std::nothrow) Req();
  if (!q) return sfail(GBS_E_NOMEM, "host allocation failed");
  q->r = *req;
  q->fp = fp;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return sfail(GBS_E_INVAL, "server is shutting down");
    }
    if ((int)s->queue.size() >= s->max_queue) {
      delete q;
      return sfail(GBS_E_BUSY, "request queue is full");
    }
    q->id = s->next_id++;
    q->t_submit = wall_ms();
    if (s->t_first < 0) s->t_first = q->t_submit;
    s->recs[q->id] = q;
    s->queue.push_back(q);
    ++s->submitted;
    *id = q->id;
  }
  s->cv_work.notify_one();
  return GBS_OK;
}

int gbs_server_poll(gbs_server s, int64_t id, int32_t* done) {
  if (!s || !done) return sfail(GBS_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->recs.find(id);
  if (it == s->recs.end()) return sfail(GBS_E_INVAL, "unknown request id");
  *done = it->second->done ? 1 : 0;
  return GBS_OK;
}

int gbs_server_wait(gbs_server s, int64_t id, gbs_result* res) {
  if (!s) return sfail(GBS_E_INVAL, "NULL server");
  Req* q;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->recs.find(id);
    if (it == s->recs.end()) return sfail(GBS_E_INVAL, "unknown request id");
    q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    s->recs.erase(id);  // `it` may be stale: other submits can rehash the map meanwhile
  }
  int rc = q->status;
  if (res) {
    res->status = q->status;
    res->max_bond = q->max_bond;
    res->eps_max = q->eps_max;
    res->queue_ms = q->t_start - q->t_submit;
    res->build_ms = q->t_built - q->t_start;
    res->sample_ms = q->t_done - q->t_built;
    res->latency_ms = q->t_done - q->t_submit;
  }
  std::string err = q->err;
  delete q;
  return rc == GBS_OK ? GBS_OK : sfail(rc, err);
}

int gbs_server_stats(gbs_server s, gbs_server_stats_t* out) {
  if (!s || !out) return sfail(GBS_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->p50_ms = percentile(s->lat, 0.50);
  out->p99_ms = percentile(s->lat, 0.99);
  double sum = 0.0, mx = 0.0;
  for (double x : s->lat) {
    sum += x;
    mx = std::max(mx, x);
  }
  out->mean_ms = s->lat.empty() ? 0.0 : sum / (double)s->lat.size();
  out->max_ms = mx;
  out->wall_s = s->t_first >= 0 ? std::max(0.0, (s->t_last - s->t_first) / 1000.0) : 0.0;
  out->throughput_rps = out->wall_s > 0 ? (double)s->completed / out->wall_s : 0.0;
  out->peak_bytes = s->peak;
  return GBS_OK;
}

int gbs_server_reset_stats(gbs_server s) {
  if (!s) return sfail(GBS_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat.clear();
  s->submitted = s->completed = s->failed = 0;
  s->t_first = -1.0;
  s->t_last = 0.0;
  s->peak = s->in_use;
  return GBS_OK;
}

void gbs_server_destroy(gbs_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (auto& kv : s->recs) delete kv.second;
  delete s;
}

}  // extern "C"
