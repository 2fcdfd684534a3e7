// Request serving on one GPU behind the C ABI (gbs_server_* in gbs_mps.h).
//
// Requests convert pure Gaussian states (Sec. II) and draw photon-number
// samples from their MPS (the consumer of Sec. I).  Three kinds:
//   build + sample : build, draw the shots, free the MPS;
//   build          : build and keep the MPS resident (optionally drawing shots),
//                    the request's id naming the resident MPS;
//   sample         : draw shots from a resident MPS.
// Builds wait in a FIFO queue; `slots` worker threads, each with its own HIP
// stream, take its head as soon as they are free and the head's footprint
// fits the memory budget beside everything admitted (resident MPS included).
// Sampling has its own engine: one thread and one stream run a batched
// sweep in which every active request advances one site per step, all of
// them in the same launches (a descriptor per request: its site tensors,
// current site, buffers, seed and output).  Requests join the sweep at any
// step, as memory allows, and leave it after their last site, so sampling
// is batched continuously across requests while builds run beside it.  A
// request's samples are identical whether it runs alone or in a mix: the
// build is deterministic and every shot's arithmetic depends only on its own
// MPS, seed and shot number.
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

constexpr int kMaxActive = 256;  // requests in the batched sweep at once
// Site steps enqueued per round of the batched sweep: one host round trip
// (descriptor upload, launches, synchronisation, admission) per this many
// steps.  A step's launches wait behind the builds that share the device, so
// a synchronisation per site would cost a 144-site request 144 such waits.
constexpr int kStepsPerRound = 16;

int sfail(int code, const std::string& msg) { return gbs_fail(code, msg); }

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Resident {
  gbs_mps h = nullptr;
  int64_t bytes = 0;
  int refs = 0;          // sample requests admitted or queued on it
  bool release = false;  // free once refs reaches 0
};

struct Req {
  gbs_request r{};
  int64_t id = 0;
  int64_t fp = 0;        // bytes reserved while building
  int64_t sbytes = 0;    // bytes of its sampling buffers while in the sweep
  double t_submit = 0, t_start = 0, t_built = 0, t_done = 0;
  int status = GBS_OK;
  int max_bond = 0;
  double eps_max = 0;
  bool done = false;
  std::string err;
  gbs_mps h = nullptr;       // MPS to sample
  bool free_after = false;   // build + sample: free h after the shots
  int64_t resident = 0;      // id of the resident MPS it samples (0: none)
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest-rank definition
  size_t k = (size_t)std::max(1.0, std::ceil(q * (double)v.size()));
  return v[std::min(k, v.size()) - 1];
}

struct Job {  // one request in the batched sweep
  Req* q;
  SampleBatchDesc d;
  void* region;
};

}  // namespace

struct gbs_server_s {
  int device = 0;
  int64_t budget = 0;
  int slots = 0;
  int max_queue = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_sample;
  std::deque<Req*> queue;          // builds
  std::deque<Req*> squeue;         // samples waiting for the sweep
  std::unordered_map<int64_t, Req*> recs;
  std::unordered_map<int64_t, Resident> residents;
  int64_t in_use = 0, peak = 0, next_id = 1;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::thread engine;
  std::vector<hipStream_t> streams;
  hipStream_t sstream = nullptr;   // the sampling engine's stream
  SampleBatchDesc* desc_dev = nullptr;
  SampleBatchDesc* desc_host = nullptr;  // pinned
  std::vector<double> lat;
  int64_t submitted = 0, completed = 0, failed = 0;
  int64_t steps = 0, step_requests = 0, max_batch = 0;
  double t_first = -1.0, t_last = 0.0;

  void worker(int slot);
  void sampler();
  void finish(Req* q, int rc);       // with mu held
  void unref(Req* q);                // with mu held: drop the request's hold on its MPS
};

// With mu held: record the outcome and wake waiters.
void gbs_server_s::finish(Req* q, int rc) {
  q->t_done = wall_ms();
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

void gbs_server_s::unref(Req* q) {
  if (q->free_after && q->h) {
    in_use -= gbs_mps_device_bytes(q->h);
    gbs_mps_free(q->h);
    q->h = nullptr;
  }
  if (q->resident) {
    auto it = residents.find(q->resident);
    if (it != residents.end() && --it->second.refs == 0 && it->second.release) {
      in_use -= it->second.bytes;
      gbs_mps_free(it->second.h);
      residents.erase(it);
    }
  }
}

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
    // Served builds run the Gaussian SVD as the chain: builds of several
    // requests share the GPU, so total work counts rather than one build's
    // latency, and computing every site on its own does more work (a start
    // from Gamma per site) and, for the banded circuits of a typical mix
    // (bond modes with D - 1 near 1e-10), falls back to the chain anyway.
    int rc = gbs_build_handle(q->r.gamma, q->r.M, &q->r.opt, st, true, &h, 0);
    q->t_built = wall_ms();
    std::string err = rc != GBS_OK ? gbs_last_error() : std::string();
    if (h) {
      gbs_mps_info_t inf;
      if (gbs_mps_info(h, &inf, nullptr, nullptr, nullptr, nullptr) == GBS_OK) {
        q->max_bond = inf.max_bond;
        q->eps_max = inf.eps_max;
      }
    }
    // FP64 handles have no MFMA sampler operand: their shots are drawn here
    const bool direct = h && q->r.shots > 0 && !gbs_batch_supported(h, q->r.shots);
    if (rc == GBS_OK && direct) {
      rc = gbs_mps_sample(h, q->r.shots, q->r.seed, q->r.out, st);
      if (rc == GBS_OK && hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        rc = sfail(GBS_E_DEVICE, "HIP error while sampling");
      }
      if (rc != GBS_OK) err = gbs_last_error();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      --running;
      in_use -= q->fp;  // the build's reservation; the MPS now holds its own bytes
      q->err = err;
      if (rc != GBS_OK) {
        if (h) gbs_mps_free(h);
        finish(q, rc);
      } else {
        const int64_t hb = gbs_mps_device_bytes(h);
        in_use += hb;
        peak = std::max(peak, in_use);
        const bool keep = q->r.kind == GBS_REQ_BUILD;
        if (keep) residents[q->id] = Resident{h, hb, 0, false};
        if (q->r.shots > 0 && !direct) {
          q->h = h;
          q->free_after = !keep;
          if (keep) {
            q->resident = q->id;
            residents[q->id].refs++;
          }
          squeue.push_back(q);  // the sweep completes the request
        } else {
          if (!keep) {
            in_use -= hb;
            gbs_mps_free(h);
          }
          finish(q, GBS_OK);
        }
      }
    }
    cv_done.notify_all();
    cv_work.notify_all();
    cv_sample.notify_all();
  }
}

void gbs_server_s::sampler() {
  (void)hipSetDevice(device);
  hipStream_t st = sstream;
  std::vector<Job> active;
  for (;;) {
    std::vector<Req*> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_sample.wait(lk, [&] { return stop || !squeue.empty() || !active.empty(); });
      if (stop && squeue.empty() && active.empty() && queue.empty() && running == 0) return;
      // admit from the head while memory allows (always one when idle)
      while (!squeue.empty() && (int)(active.size() + admit.size()) < kMaxActive) {
        Req* q = squeue.front();
        const bool batch = gbs_batch_supported(q->h, q->r.shots);
        const int64_t b = batch ? gbs_batch_bytes(q->h, q->r.shots) : 0;
        if (!(active.empty() && admit.empty()) && in_use + b > budget) break;
        squeue.pop_front();
        q->sbytes = b;
        in_use += b;
        peak = std::max(peak, in_use);
        if (q->t_start == 0) q->t_start = wall_ms();
        admit.push_back(q);
      }
    }
    if (admit.empty() && active.empty()) {
      std::unique_lock<std::mutex> lk(mu);
      // woken with nothing to do (e.g. stop with builds still running)
      cv_sample.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    for (Req* q : admit) {
      int rc = GBS_OK;
      Job j{q, SampleBatchDesc{}, nullptr};
      if (gbs_batch_supported(q->h, q->r.shots)) {
        if (hipMallocAsync(&j.region, (size_t)q->sbytes, st) != hipSuccess) {
          (void)hipGetLastError();
          j.region = nullptr;
          rc = sfail(GBS_E_NOMEM, "device allocation of the sampling buffers failed");
        } else {
          rc = gbs_batch_prepare(q->h, q->r.shots, q->r.seed, q->r.out, st, j.region, (size_t)q->sbytes, &j.d);
        }
      } else {  // an FP64 resident MPS: the vector sweep, on its own
        rc = gbs_mps_sample(q->h, q->r.shots, q->r.seed, q->r.out, st);
        if (rc == GBS_OK && hipStreamSynchronize(st) != hipSuccess) {
          (void)hipGetLastError();
          rc = sfail(GBS_E_DEVICE, "HIP error while sampling");
        }
        if (rc == GBS_OK) {
          std::lock_guard<std::mutex> lk(mu);
          unref(q);
          finish(q, GBS_OK);
          cv_done.notify_all();
          cv_work.notify_all();
          continue;
        }
      }
      if (rc != GBS_OK) {
        const std::string err = gbs_last_error();
        if (j.region) (void)hipFreeAsync(j.region, st);
        std::lock_guard<std::mutex> lk(mu);
        in_use -= q->sbytes;
        q->err = err;
        unref(q);
        finish(q, rc);
        cv_done.notify_all();
        cv_work.notify_all();
        continue;
      }
      active.push_back(j);
    }
    if (active.empty()) continue;
    // up to kStepsPerRound site steps of every active request (a request
    // whose last site comes earlier takes part in the steps up to it)
    const int64_t spb = sampler_shots_per_block();
    int nsteps = 0;
    int nreq_k[kStepsPerRound], nt_k[kStepsPerRound];
    int64_t blocks_k[kStepsPerRound], shots_k[kStepsPerRound];
    for (int k = 0; k < kStepsPerRound; ++k) {
      int n = 0, nt = 8;
      int64_t mb = 0, ms = 0;
      for (Job& j : active) {
        const int site = j.d.site + k;
        if (site > j.d.M) continue;
        SampleBatchDesc& dk = desc_host[(size_t)k * kMaxActive + n++];
        dk = j.d;
        dk.site = site;
        nt = std::max(nt, gbs_batch_site_nt(j.q->h, site));
        mb = std::max(mb, (j.d.nshots + spb - 1) / spb + 1);
        ms = std::max(ms, j.d.nshots);
      }
      if (n == 0) break;
      nreq_k[k] = n;
      nt_k[k] = nt;
      blocks_k[k] = mb;
      shots_k[k] = ms;
      nsteps = k + 1;
    }
    hipError_t e = hipMemcpyAsync(desc_dev, desc_host, (size_t)nsteps * kMaxActive * sizeof(SampleBatchDesc),
                                  hipMemcpyHostToDevice, st);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
      SampleBatchDesc* dd = desc_dev + (size_t)k * kMaxActive;
      e = launch_sample_batch(st, dd, nreq_k[k], blocks_k[k], nt_k[k]);
      if (e == hipSuccess) e = launch_partition_batch(st, dd, nreq_k[k], shots_k[k]);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) (void)hipGetLastError();
    std::vector<Job> next;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int k = 0; k < nsteps; ++k) {
        ++steps;
        step_requests += nreq_k[k];
        max_batch = std::max<int64_t>(max_batch, nreq_k[k]);
      }
      for (Job& j : active) {
        const bool last = j.d.site + nsteps > j.d.M;
        if (e == hipSuccess && !last) {
          j.d.site += nsteps;
          next.push_back(j);
          continue;
        }
        (void)hipFreeAsync(j.region, st);
        in_use -= j.q->sbytes;
        if (e != hipSuccess) j.q->err = std::string("HIP error '") + hipGetErrorString(e) + "' in the batched sweep";
        unref(j.q);
        finish(j.q, e == hipSuccess ? GBS_OK : GBS_E_DEVICE);
      }
    }
    active.swap(next);
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
  auto undo = [&](const char* msg) {
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    if (s->sstream) (void)hipStreamDestroy(s->sstream);
    if (s->desc_dev) (void)hipFree(s->desc_dev);
    if (s->desc_host) (void)hipHostFree(s->desc_host);
    (void)hipGetLastError();
    delete s;
    return sfail(GBS_E_DEVICE, msg);
  };
  if (hipGetDevice(&s->device) != hipSuccess) return undo("hipGetDevice failed");
  for (int i = 0; i < slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return undo("hipStreamCreateWithFlags failed");
    s->streams.push_back(st);
  }
  if (hipStreamCreateWithFlags(&s->sstream, hipStreamNonBlocking) != hipSuccess)
    return undo("hipStreamCreateWithFlags failed");
  if (hipMalloc((void**)&s->desc_dev, (size_t)kStepsPerRound * kMaxActive * sizeof(SampleBatchDesc)) != hipSuccess)
    return undo("device allocation of the sweep descriptors failed");
  if (hipHostMalloc((void**)&s->desc_host, (size_t)kStepsPerRound * kMaxActive * sizeof(SampleBatchDesc),
                    hipHostMallocDefault) != hipSuccess)
    return undo("pinned host allocation of the sweep descriptors failed");
  for (int i = 0; i < slots; ++i) s->workers.emplace_back(&gbs_server_s::worker, s, i);
  s->engine = std::thread(&gbs_server_s::sampler, s);
  *out = s;
  return GBS_OK;
}

int gbs_server_submit(gbs_server s, const gbs_request* req, int64_t* id) {
  if (!s || !req || !id) return sfail(GBS_E_INVAL, "NULL argument");
  if (req->kind < GBS_REQ_BUILD_SAMPLE || req->kind > GBS_REQ_SAMPLE) return sfail(GBS_E_INVAL, "unknown request kind");
  if (req->shots < 0 || (req->shots > 0 && !req->out)) return sfail(GBS_E_INVAL, "invalid request (shots or out)");
  int64_t fp = 0;
  gbs_build_opts opt = req->opt;
  opt.flags |= GBS_CHAIN_GSVD;  // served builds run the chain (see the build worker)
  if (req->kind != GBS_REQ_SAMPLE) {
    if (!req->gamma || req->M < 1) return sfail(GBS_E_INVAL, "invalid request (gamma or M)");
    fp = gbs_mps_footprint(req->M, &opt, req->shots);
    if (fp < 0) return sfail(GBS_E_INVAL, "invalid build options");
    if (fp > s->budget) return sfail(GBS_E_NOMEM, "request footprint exceeds the server's memory budget");
    fp = gbs_mps_footprint(req->M, &opt, 0);  // the build's own reservation
  } else if (req->shots < 1) {
    return sfail(GBS_E_INVAL, "a sample request needs shots >= 1");
  }
  Req* q = new (std::nothrow) Req();
  if (!q) return sfail(GBS_E_NOMEM, "host allocation failed");
  q->r = *req;
  q->r.opt = opt;
  q->fp = fp;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return sfail(GBS_E_INVAL, "server is shutting down");
    }
    if (req->kind == GBS_REQ_SAMPLE) {
      auto it = s->residents.find(req->handle);
      if (it == s->residents.end() || it->second.release) {
        delete q;
        return sfail(GBS_E_INVAL, "no resident MPS with this id");
      }
      if ((int)s->squeue.size() >= s->max_queue) {
        delete q;
        return sfail(GBS_E_BUSY, "request queue is full");
      }
      it->second.refs++;
      q->h = it->second.h;
      q->resident = req->handle;
      q->id = s->next_id++;
      q->t_submit = wall_ms();
      if (s->t_first < 0) s->t_first = q->t_submit;
      s->recs[q->id] = q;
      s->squeue.push_back(q);
      ++s->submitted;
      *id = q->id;
    } else {
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
  }
  s->cv_work.notify_one();
  s->cv_sample.notify_one();
  return GBS_OK;
}

int gbs_server_release(gbs_server s, int64_t handle) {
  if (!s) return sfail(GBS_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->residents.find(handle);
  if (it == s->residents.end() || it->second.release) return sfail(GBS_E_INVAL, "no resident MPS with this id");
  it->second.release = true;
  if (it->second.refs == 0) {
    s->in_use -= it->second.bytes;
    gbs_mps_free(it->second.h);
    s->residents.erase(it);
  }
  s->cv_work.notify_all();
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
    const double t_start = q->t_start > 0 ? q->t_start : q->t_done;
    const double t_built = q->t_built > 0 ? q->t_built : t_start;
    res->queue_ms = t_start - q->t_submit;
    res->build_ms = t_built - t_start;
    res->sample_ms = q->t_done - t_built;
    res->latency_ms = q->t_done - q->t_submit;
    res->handle = q->r.kind == GBS_REQ_BUILD && rc == GBS_OK ? q->id : 0;
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
  out->resident = (int64_t)s->residents.size();
  out->sweep_steps = s->steps;
  out->mean_batch = s->steps > 0 ? (double)s->step_requests / (double)s->steps : 0.0;
  out->max_batch = s->max_batch;
  return GBS_OK;
}

int gbs_server_reset_stats(gbs_server s) {
  if (!s) return sfail(GBS_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat.clear();
  s->submitted = s->completed = s->failed = 0;
  s->steps = s->step_requests = s->max_batch = 0;
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
  {
    std::lock_guard<std::mutex> lk(s->mu);  // builds are done: wake the sweep to drain
  }
  s->cv_sample.notify_all();
  s->engine.join();
  for (auto& kv : s->residents) gbs_mps_free(kv.second.h);
  (void)hipStreamSynchronize(s->sstream);
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  (void)hipStreamDestroy(s->sstream);
  (void)hipFree(s->desc_dev);
  (void)hipHostFree(s->desc_host);
  for (auto& kv : s->recs) delete kv.second;
  delete s;
}

}  // extern "C"
