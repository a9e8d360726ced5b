// Continuous-batching server over sift_extract_batch: requests of any size
// are admitted in arrival order into batches that fit a free range of a
// caller-owned device arena, and launched on a few streams of the server's
// own so consecutive batches overlap.  One host worker thread does the
// admitting, launching and retiring; submit, poll and wait only touch the
// shared queues under a mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sift.h"
#include "sift_internal.h"

using namespace sift;

namespace sift {
void set_last_error(const std::string& msg);
}

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kAlign = 256;
int64_t align_up256(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

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

// First-fit allocator over [0, size) in 256-byte units; free ranges coalesce.
class Arena {
 public:
  void reset(int64_t size) {
    free_.clear();
    if (size > 0) free_[0] = size;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  int64_t take(int64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void give(int64_t off, int64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<int64_t, int64_t> free_;
};

sift_status server_fail(sift_status st, const std::string& msg) {
  set_last_error(msg);
  return st;
}

int64_t header_bytes(int n) {
  Header hd;
  make_header(n, &hd);
  return hd.bytes;
}

// Workspace bytes that cover a batch of n requests whose regions sum to
// `regions`, however the batched call splits it: at most min(n, kMaxParts)
// sub-batches, each with a header no larger than the whole batch's.
int64_t batch_bytes(int n, int64_t regions) {
  return align_up256((int64_t)std::min(n, kMaxParts) * header_bytes(n) + regions);
}

}  // namespace

struct sift_server {
  sift_handle* handle = nullptr;
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
  bool admit();
};

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
    const Clock::time_point now = Clock::now();
    Batch& b = inflight[i];
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
    hipEventDestroy(b.event);
    inflight.erase(inflight.begin() + i);
    any = true;
  }
  return any;
}

// Forms and launches batches while a stream is free and the head request
// fits; returns true if any launched.  Caller holds mu.
bool sift_server::admit() {
  bool any = false;
  while (!pending.empty() && (int)inflight.size() < max_inflight) {
    const int64_t room = alloc.largest();
    int n = 0;
    int64_t regions = 0;
    while (n < (int)pending.size() && n < max_batch) {
      const int64_t need = batch_bytes(n + 1, regions + pending[n].region);
      if (need > room) break;
      regions += pending[n].region;
      ++n;
    }
    if (n == 0) break;   // the head waits for arena space
    const int64_t bytes = batch_bytes(n, regions);
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
    const sift_status st = sift_extract_batch(handle, n, imgs.data(), hs.data(), ws.data(),
                                              ps.data(), arena + off, (size_t)bytes, outs.data(),
                                              streams[si]);
    hipError_t e = hipSuccess;
    if (st == SIFT_OK) e = hipEventCreateWithFlags(&b.event, hipEventDisableTiming);
    if (st == SIFT_OK && e == hipSuccess) e = hipEventRecord(b.event, streams[si]);
    if (st != SIFT_OK || e != hipSuccess) {
      if (worker_error.empty())
        worker_error = st != SIFT_OK ? std::string("batch launch: ") + sift_last_error()
                                     : std::string("batch event: ") + hipGetErrorString(e);
      // nothing (more) was enqueued for this batch: the requests end here
      const Clock::time_point now = Clock::now();
      for (uint64_t t : b.tickets) {
        tickets[t].done = true;
        tickets[t].finished = now;
      }
      alloc.give(off, bytes);
      if (st == SIFT_OK) {
        hipStreamSynchronize(streams[si]);   // the batch's kernels did launch
        if (e != hipSuccess && b.event) hipEventDestroy(b.event);
      }
      done_cv.notify_all();
      continue;
    }
    stream_busy[si] = true;
    arena_in_use += bytes;
    stats.batches += 1;
    stats.peak_arena = std::max(stats.peak_arena, arena_in_use);
    inflight.push_back(std::move(b));
    stats.peak_inflight = std::max(stats.peak_inflight, (int64_t)inflight.size());
    any = true;
  }
  return any;
}

void sift_server::run() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    const bool retired = retire();
    if (retired) done_cv.notify_all();
    admit();
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

sift_status sift_server_create(const sift_params* p, void* d_arena, size_t arena_bytes,
                               int32_t max_batch, int32_t max_inflight, sift_server** out) {
  if (!p || !d_arena || !out) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (reinterpret_cast<uintptr_t>(d_arena) % kAlign != 0)
    return server_fail(SIFT_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  if (max_batch < 1 || max_batch > 4096)
    return server_fail(SIFT_ERR_INVALID_ARG, "max_batch must be in 1..4096");
  if (max_inflight < 1 || max_inflight > 8)
    return server_fail(SIFT_ERR_INVALID_ARG, "max_inflight must be in 1..8");
  *out = nullptr;
  sift_handle* h = nullptr;
  sift_status st = sift_create(p, &h);
  if (st != SIFT_OK) return server_fail(st, sift_last_error());
  sift_server* s = new sift_server();
  s->handle = h;
  s->arena = static_cast<char*>(d_arena);
  s->arena_bytes = (int64_t)arena_bytes / kAlign * kAlign;
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
    sift_destroy(h);
    delete s;
    return server_fail(SIFT_ERR_HIP, std::string("server streams: ") + hipGetErrorString(e));
  }
  s->stream_busy.assign(max_inflight, false);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SIFT_OK;
}

sift_status sift_server_submit(sift_server* s, const float* d_image, int32_t height, int32_t width,
                               int64_t pitch, const sift_output* out, uint64_t* ticket) {
  if (!s || !d_image || !out || !ticket) return server_fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (pitch < width) return server_fail(SIFT_ERR_INVALID_ARG, "pitch < width");
  if (!out->keypoints || !out->descriptors || !out->count || out->capacity < 0)
    return server_fail(SIFT_ERR_INVALID_ARG, "bad output buffers");
  size_t one = 0;
  const sift_status st = sift_workspace_size(s->handle, height, width, &one);
  if (st != SIFT_OK) return server_fail(st, sift_last_error());
  if ((int64_t)one > s->arena_bytes)
    return server_fail(SIFT_ERR_TOO_LARGE, "request workspace exceeds the arena");
  Request r;
  r.image = d_image;
  r.h = height;
  r.w = width;
  r.pitch = pitch;
  r.out = *out;
  r.region = (int64_t)one - header_bytes(1);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return server_fail(SIFT_ERR_INVALID_ARG, "server is shutting down");
    r.ticket = s->next_ticket++;
    Ticket t;
    t.submitted = Clock::now();
    s->tickets.emplace(r.ticket, t);
    s->pending.push_back(r);
    s->stats.submitted += 1;
    *ticket = r.ticket;
  }
  s->cv.notify_one();
  return SIFT_OK;
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
  sift_destroy(s->handle);
  delete s;
  if (!err.empty()) return server_fail(SIFT_ERR_HIP, err);
  return SIFT_OK;
}

}  // extern "C"
