// Continuous-batching server over sift_extract_batch: requests of any size
// are admitted in arrival order into batches that fit a free range of a
// caller-owned device arena, and launched on a few streams of the server's
// own so consecutive batches overlap.  One host worker thread admits,
// launches and retires batches.  Batches are formed under the server mutex
// but their launch sequences are enqueued outside it, so submit, poll and
// wait never wait for a launch.  Each server stream has a handle of its own,
// so the sub-batch streams a large batch forks onto are never shared by two
// batches in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sift.h"
#include "sift_internal.h"
#include "sift_sched.h"

using namespace sift;

namespace sift {
void set_last_error(const std::string& msg);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  const float* image;
  int32_t h, w;
  int64_t pitch;
  sift_output out;
  int64_t region;   // workspace bytes of this image's region
};

struct Ticket {
  Clock::time_point submitted, finished;
  bool done = false;
};

struct Batch {
  int stream;
  hipEvent_t event = nullptr;
  int64_t offset, bytes;
  std::vector<uint64_t> tickets;
};

sift_status server_fail(sift_status st, const std::string& msg) {
  set_last_error(msg);
  return st;
}

}  // namespace

struct sift_server {
  std::vector<sift_handle*> handles;   // one per stream (each with its own sub-batch streams)
  char* arena = nullptr;
  int64_t arena_bytes = 0;
  int max_batch = 1, max_inflight = 1;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<bool> stream_busy;

  std::mutex mu;
  std::condition_variable cv;       // worker wake-up: submit, stop
  std::condition_variable done_cv;  // waiters: a batch retired
  std::deque<Request> pending;
  std::vector<Batch> inflight;
  int launching = 0;                // batches being enqueued outside the mutex
  std::unordered_map<uint64_t, Ticket> tickets;
  Arena alloc;
  int64_t arena_in_use = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string worker_error;
  sift_server_stats stats{};
  std::thread worker;

  void run();
  bool retire();
  void launch_ready(std::unique_lock<std::mutex>& lk);
  void end_batch(const Batch& b, Clock::time_point now);
};

// Marks a batch's tickets done and returns its arena range and stream.
// Caller holds mu.
void sift_server::end_batch(const Batch& b, Clock::time_point now) {
  for (uint64_t t : b.tickets) {
    auto it = tickets.find(t);
    if (it != tickets.end()) {
      it->second.done = true;
      it->second.finished = now;
    }
  }
  stats.completed += (int64_t)b.tickets.size();
  alloc.give(b.offset, b.bytes);
  arena_in_use -= b.bytes;
  stream_busy[b.stream] = false;
}

// Retires finished batches; returns true if any retired.  Caller holds mu.
bool sift_server::retire() {
  bool any = false;
  for (size_t i = 0; i < inflight.size();) {
    const hipError_t q = hipEventQuery(inflight[i].event);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (q != hipSuccess && worker_error.empty())
      worker_error = std::string("batch completion: ") + hipGetErrorString(q);
    end_batch(inflight[i], Clock::now());
    hipEventDestroy(inflight[i].event);
    inflight.erase(inflight.begin() + i);
    any = true;
  }
  return any;
}

// Forms batches while a stream is free and the head request fits, and
// enqueues each one's launch sequence with mu released.  Called and returns
// with mu held.
void sift_server::launch_ready(std::unique_lock<std::mutex>& lk) {
  while (!pending.empty() && (int)inflight.size() + launching < max_inflight) {
    int64_t bytes = 0;
    const int n = next_batch(pending, max_batch, alloc.largest(), &bytes);
    if (n == 0) break;   // the head waits for arena space
    const int64_t off = alloc.take(bytes);
    int si = 0;
    while (stream_busy[si]) ++si;
    std::vector<const float*> imgs(n);
    std::vector<int32_t> hs(n), ws(n);
    std::vector<int64_t> ps(n);
    std::vector<sift_output> outs(n);
    Batch b;
    b.stream = si;
    b.offset = off;
    b.bytes = bytes;
    for (int i = 0; i < n; ++i) {
      const Request& r = pending[i];
      imgs[i] = r.image;
      hs[i] = r.h;
      ws[i] = r.w;
      ps[i] = r.pitch;
      outs[i] = r.out;
      b.tickets.push_back(r.ticket);
    }
    pending.erase(pending.begin(), pending.begin() + n);
    stream_busy[si] = true;
    arena_in_use += bytes;
    stats.batches += 1;
    stats.largest_batch = std::max(stats.largest_batch, (int64_t)n);
    if (!inflight.empty() || launching > 0) stats.overlapped_batches += 1;
    stats.peak_arena = std::max(stats.peak_arena, arena_in_use);
    ++launching;

    lk.unlock();
    const sift_status st = sift_extract_batch(handles[si], n, imgs.data(), hs.data(), ws.data(),
                                              ps.data(), arena + off, (size_t)bytes, outs.data(),
                                              streams[si]);
    hipError_t e = hipSuccess;
    if (st == SIFT_OK) e = hipEventCreateWithFlags(&b.event, hipEventDisableTiming);
    if (st == SIFT_OK && e == hipSuccess) e = hipEventRecord(b.event, streams[si]);
    std::string err;
    if (st != SIFT_OK) err = std::string("batch launch: ") + sift_last_error();
    else if (e != hipSuccess) err = std::string("batch event: ") + hipGetErrorString(e);
    if (!err.empty() && st == SIFT_OK) {
      hipStreamSynchronize(streams[si]);   // the batch's kernels did launch
      if (b.event) hipEventDestroy(b.event);
      b.event = nullptr;
    }
    lk.lock();

    --launching;
    if (!err.empty()) {
      // nothing (more) is in flight for this batch: its requests end here
      if (worker_error.empty()) worker_error = err;
      end_batch(b, Clock::now());
      done_cv.notify_all();
      continue;
    }
    inflight.push_back(std::move(b));
    stats.peak_inflight = std::max(stats.peak_inflight, (int64_t)inflight.size());
  }
}

void sift_server::run() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    if (retire()) done_cv.notify_all();
    launch_ready(lk);
    if (stop && pending.empty() && inflight.empty()) break;
    if (inflight.empty()) {
      // idle: sleep until a submit (or stop) arrives
      cv.wait(lk, [&] { return stop || !pending.empty(); });
    } else {
      // batches in flight: check their events again shortly
      cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
  done_cv.notify_all();
}

extern "C" {

sift_status sift_server_batch_bytes(const sift_params* p, int32_t n, const int32_t* heights,
                                    const int32_t* widths, size_t* bytes) {
  if (!p || !heights || !widths || !bytes) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (n < 1) return server_fail(SIFT_ERR_INVALID_ARG, "batch size must be >= 1");
  sift_handle* h = nullptr;
  sift_status st = sift_create(p, &h);
  if (st != SIFT_OK) return server_fail(st, sift_last_error());
  const int64_t hdr1 = header_bytes(1);
  int64_t regions = 0;
  for (int i = 0; i < n && st == SIFT_OK; ++i) {
    size_t one = 0;
    st = sift_workspace_size(h, heights[i], widths[i], &one);
    regions += (int64_t)one - hdr1;
  }
  sift_destroy(h);
  if (st != SIFT_OK) return server_fail(st, sift_last_error());
  *bytes = (size_t)batch_bytes(n, regions);
  return SIFT_OK;
}

sift_status sift_server_create(const sift_params* p, void* d_arena, size_t arena_bytes,
                               int32_t max_batch, int32_t max_inflight, sift_server** out) {
  if (!p || !d_arena || !out) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (reinterpret_cast<uintptr_t>(d_arena) % kArenaAlign != 0)
    return server_fail(SIFT_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  if (max_batch < 1 || max_batch > 4096)
    return server_fail(SIFT_ERR_INVALID_ARG, "max_batch must be in 1..4096");
  if (max_inflight < 1 || max_inflight > 8)
    return server_fail(SIFT_ERR_INVALID_ARG, "max_inflight must be in 1..8");
  *out = nullptr;
  sift_server* s = new sift_server();
  sift_status st = SIFT_OK;
  for (int i = 0; i < max_inflight && st == SIFT_OK; ++i) {
    sift_handle* h = nullptr;
    st = sift_create(p, &h);
    if (st == SIFT_OK) s->handles.push_back(h);
  }
  if (st != SIFT_OK) {
    const std::string msg = sift_last_error();
    for (sift_handle* h : s->handles) sift_destroy(h);
    delete s;
    return server_fail(st, msg);
  }
  s->arena = static_cast<char*>(d_arena);
  s->arena_bytes = (int64_t)arena_bytes / kArenaAlign * kArenaAlign;
  s->max_batch = max_batch;
  s->max_inflight = max_inflight;
  s->alloc.reset(s->arena_bytes);
  hipError_t e = hipGetDevice(&s->device);
  for (int i = 0; i < max_inflight && e == hipSuccess; ++i) {
    hipStream_t q = nullptr;
    e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(q);
  }
  if (e != hipSuccess) {
    for (hipStream_t q : s->streams) hipStreamDestroy(q);
    for (sift_handle* h : s->handles) sift_destroy(h);
    delete s;
    return server_fail(SIFT_ERR_HIP, std::string("server streams: ") + hipGetErrorString(e));
  }
  s->stream_busy.assign(max_inflight, false);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SIFT_OK;
}

}  // extern "C"

namespace {

// Checks one request and fills *r (all but its ticket).
sift_status make_request(sift_server* s, const float* d_image, int32_t height, int32_t width,
                         int64_t pitch, const sift_output* out, Request* r) {
  if (!d_image || !out) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (pitch < width) return server_fail(SIFT_ERR_INVALID_ARG, "pitch < width");
  if (!out->keypoints || !out->descriptors || !out->count || out->capacity < 0)
    return server_fail(SIFT_ERR_INVALID_ARG, "bad output buffers");
  size_t one = 0;
  const sift_status st = sift_workspace_size(s->handles[0], height, width, &one);
  if (st != SIFT_OK) return server_fail(st, sift_last_error());
  if ((int64_t)one > s->arena_bytes)
    return server_fail(SIFT_ERR_TOO_LARGE, "request workspace exceeds the arena");
  r->image = d_image;
  r->h = height;
  r->w = width;
  r->pitch = pitch;
  r->out = *out;
  r->region = (int64_t)one - header_bytes(1);
  return SIFT_OK;
}

// Queues checked requests under one hold of the lock (the worker sees all of
// them at once) and assigns their tickets.
sift_status enqueue(sift_server* s, std::vector<Request>& reqs, Clock::time_point arrived,
                    uint64_t* tickets) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return server_fail(SIFT_ERR_INVALID_ARG, "server is shutting down");
    for (size_t i = 0; i < reqs.size(); ++i) {
      Request& r = reqs[i];
      r.ticket = s->next_ticket++;
      Ticket t;
      t.submitted = arrived;
      s->tickets.emplace(r.ticket, t);
      s->pending.push_back(r);
      s->stats.submitted += 1;
      tickets[i] = r.ticket;
    }
  }
  s->cv.notify_one();
  return SIFT_OK;
}

}  // namespace

extern "C" {

sift_status sift_server_submit(sift_server* s, const float* d_image, int32_t height, int32_t width,
                               int64_t pitch, const sift_output* out, uint64_t* ticket) {
  // the request's latency counts from here, before any validation or lock
  const Clock::time_point arrived = Clock::now();
  if (!s || !ticket) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::vector<Request> reqs(1);
  const sift_status st = make_request(s, d_image, height, width, pitch, out, &reqs[0]);
  if (st != SIFT_OK) return st;
  return enqueue(s, reqs, arrived, ticket);
}

sift_status sift_server_submit_n(sift_server* s, int32_t n, const float* const* d_images,
                                 const int32_t* heights, const int32_t* widths,
                                 const int64_t* pitches, const sift_output* outs,
                                 uint64_t* tickets) {
  const Clock::time_point arrived = Clock::now();
  if (!s || !d_images || !heights || !widths || !pitches || !outs || !tickets)
    return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (n < 1) return server_fail(SIFT_ERR_INVALID_ARG, "n must be >= 1");
  std::vector<Request> reqs(n);
  for (int i = 0; i < n; ++i) {
    const sift_status st = make_request(s, d_images[i], heights[i], widths[i], pitches[i],
                                        &outs[i], &reqs[i]);
    if (st != SIFT_OK) return st;
  }
  return enqueue(s, reqs, arrived, tickets);
}

namespace {

// Caller holds mu.  Reports and forgets a finished ticket.
sift_status report(sift_server* s, uint64_t ticket, int32_t* done, double* latency_ms) {
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return server_fail(SIFT_ERR_INVALID_ARG, "unknown ticket");
  if (!it->second.done) {
    if (done) *done = 0;
    return SIFT_OK;
  }
  if (done) *done = 1;
  if (latency_ms)
    *latency_ms =
        std::chrono::duration<double, std::milli>(it->second.finished - it->second.submitted)
            .count();
  s->tickets.erase(it);
  if (!s->worker_error.empty()) return server_fail(SIFT_ERR_HIP, s->worker_error);
  return SIFT_OK;
}

}  // namespace

sift_status sift_server_poll(sift_server* s, uint64_t ticket, int32_t* done, double* latency_ms) {
  if (!s || !done) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  return report(s, ticket, done, latency_ms);
}

sift_status sift_server_wait(sift_server* s, uint64_t ticket, double* latency_ms) {
  if (!s) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return server_fail(SIFT_ERR_INVALID_ARG, "unknown ticket");
  s->done_cv.wait(lk, [&] { return it->second.done; });
  int32_t done = 0;
  return report(s, ticket, &done, latency_ms);
}

sift_status sift_server_get_stats(sift_server* s, sift_server_stats* stats) {
  if (!s || !stats) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *stats = s->stats;
  return SIFT_OK;
}

sift_status sift_server_destroy(sift_server* s) {
  if (!s) return SIFT_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  const std::string err = s->worker_error;
  for (hipStream_t q : s->streams) hipStreamDestroy(q);
  for (sift_handle* h : s->handles) sift_destroy(h);
  delete s;
  if (!err.empty()) return server_fail(SIFT_ERR_HIP, err);
  return SIFT_OK;
}

}  // extern "C"
