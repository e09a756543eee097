// server.cpp -- continuous-batching request loop over the libhers C ABI.
//
// The server keeps encrypted galleries and the evaluation key resident (they
// live in the context and in caller memory) and serves queries as they
// arrive.  Each query runs the client and server halves of the search
// protocol (App. B, Alg. "HERS Search"): probe encryption, the batched
// encrypted search over its gallery, decryption of the scores.
//
// Admission is by memory: every request needs device memory for its probe
// search form, score ciphertexts and decrypted scores, carved from a
// caller-provided arena by a first-fit allocator; a request that does not fit
// waits in the queue (a deferral) until earlier results are collected.  A
// worker thread forms waves: the oldest queued request and the later queued
// requests on the same gallery, which share one pass over it
// (hers_search_batch).  Requests on other galleries would share nothing and
// would only wait for the wave's largest search, so they go in waves of their
// own.  Up to SRV_STREAMS waves are in flight, each on its own stream, so
// small searches run beside large ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hers.h"
#include "internal.h"

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Gallery {
  const uint32_t* ptr;
  uint64_t words;
  int64_t m;
  int32_t d;
};

struct Request {
  int64_t ticket;
  int32_t gid;
  std::vector<int32_t> query;
  uint64_t seed;
  double t_arrival = 0, t_start = 0, t_done = 0;
  size_t off = 0, bytes = 0;          // one arena range: probe | score cts | scores
  size_t o_probe = 0, o_ct = 0, o_out = 0;
  int state = 0;                      // 0 queued, 1 on the GPU, 2 done, 3 failed
  bool in_arena = false;              // holds its arena range [off, off + bytes)
  std::string error;
};

#define SRV_STREAMS 4
#define SRV_MAX_ROUND 256   // blocks per search round of a wave (halved while the arena is short)

// A wave carries copies of everything the unlocked launch reads: its
// requests' gallery records and the workspace sizes it was carved with
// (hers_server_add_gallery may grow both meanwhile).  A failure is recorded
// here and applied to the requests by the retire step, under the lock.
struct Wave {
  std::vector<Request*> reqs;
  std::vector<Gallery> gals;          // gallery of reqs[i]
  size_t enc_ws = 0, dec_ws = 0;
  size_t ws_off = 0, ws_bytes = 0;
  hipEvent_t ev = nullptr;
  int stream = 0;
  bool failed = false;
  std::string error;
};

}  // namespace

struct hers_server {
  hers_ctx* ctx;
  const uint8_t* sk;
  char* arena_base;
  Arena arena;
  int max_batch;
  hers_info info;
  int device = 0;
  std::vector<Gallery> galleries;
  std::deque<Request*> queue;
  std::map<int64_t, Request*> reqs;
  std::vector<Wave> inflight;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  int64_t next_ticket = 1;
  hipStream_t streams[SRV_STREAMS] = {};
  hipEvent_t events[SRV_STREAMS] = {};  // a wave's completion, on its stream (one wave per stream)
  bool stream_busy[SRV_STREAMS] = {};
  hipStream_t copy_stream = nullptr;
  hers_server_stats st;
  uint32_t bound = 0;                 // the context's feature bound
  size_t enc_ws = 0, dec_ws = 0;
  // bumped when arena memory is returned (results collected) and when a
  // request is queued: a worker whose admission failed sleeps until one changes
  uint64_t mem_gen = 0, queue_gen = 0;

  hers_server(hers_ctx* c, const uint8_t* s, char* base, size_t bytes, int mb)
      : ctx(c), sk(s), arena_base(base), arena(bytes), max_batch(mb) {
    std::memset(&st, 0, sizeof(st));
  }
};

namespace {

size_t request_bytes(const hers_server* s, const Gallery& g, size_t* op, size_t* oc, size_t* oo) {
  size_t off = 0;
  *op = off; off += align256(hers_probe_words(s->ctx, g.d) * 4);
  *oc = off; off += align256(hers_blocks(s->ctx, g.m) * hers_ct_words(s->ctx) * 8);
  *oo = off; off += align256((size_t)g.m * 4);
  return off;
}

// Workspace of one wave: probe encryption + batched search (rounds of cb
// blocks per request) + decryption.
size_t wave_ws_bytes(hers_server* s, size_t enc_ws, size_t dec_ws, size_t nreq, int64_t cb) {
  const size_t per = hers_workspace_bytes(s->ctx, 2, s->info.n, 1);
  return align256(enc_ws) + align256(dec_ws) + align256(per * (size_t)cb * nreq);
}

// Records a wave's failure (applied to its requests when it is retired).
// Work already enqueued may still use the wave's memory: wait for its stream
// before the memory can be handed out again.
void fail_wave(hers_server* s, Wave& w, const char* what) {
  w.failed = true;
  w.error = std::string(what) + ": " + hers_last_error();
  (void)hipStreamSynchronize(s->streams[w.stream]);
}

// Enqueues a wave; called with the lock released (the ctx belongs to the
// worker).  Reads only the wave and its requests' fixed fields.
void launch_wave(hers_server* s, Wave& w) {
  hipStream_t st = s->streams[w.stream];
  char* base = s->arena_base;
  char* ws = base + w.ws_off;
  void* ws_enc = ws;
  void* ws_dec = ws + align256(w.enc_ws);
  void* ws_srch = ws + align256(w.enc_ws) + align256(w.dec_ws);
  const size_t srch_bytes = w.ws_bytes - align256(w.enc_ws) - align256(w.dec_ws);
  const size_t nr = w.reqs.size();
  std::vector<const uint32_t*> gal(nr), prb(nr);
  std::vector<uint64_t> gw(nr), pw(nr);
  std::vector<int64_t> ms(nr);
  std::vector<int32_t> ds(nr);
  std::vector<uint64_t*> sc(nr);
  // algorithmic gallery bytes of the wave: groups of up to 16 requests per gallery stream it once
  {
    std::map<int32_t, std::pair<int64_t, Gallery>> per;
    for (size_t i = 0; i < nr; ++i) {
      auto& e = per[w.reqs[i]->gid];
      e.first += 1;
      e.second = w.gals[i];
    }
    uint64_t bytes = 0;
    for (auto& kv : per) {
      const Gallery& g = kv.second.second;
      bytes += (uint64_t)((kv.second.first + 15) / 16) * hers_gallery_words(s->ctx, g.m, g.d) * 4;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.gallery_bytes += bytes;
  }
  for (size_t i = 0; i < nr; ++i) {
    Request* r = w.reqs[i];
    const Gallery& g = w.gals[i];
    char* rb = base + r->off;
    // the query (host copy) was range checked at submission
    if (hers::encrypt_probe_prechecked(s->ctx, r->query.data(), g.d, r->seed, (uint32_t*)(rb + r->o_probe), ws_enc,
                                       w.enc_ws, st)) {
      fail_wave(s, w, "probe encryption");
      return;
    }
    gal[i] = g.ptr; gw[i] = g.words; ms[i] = g.m; ds[i] = g.d;
    pw[i] = hers_probe_words(s->ctx, g.d);
    prb[i] = (const uint32_t*)(rb + r->o_probe);
    sc[i] = (uint64_t*)(rb + r->o_ct);
  }
  if (hers_search_batch(s->ctx, (int32_t)nr, gal.data(), gw.data(), ms.data(), ds.data(), prb.data(), pw.data(),
                        sc.data(), ws_srch, srch_bytes, st)) { fail_wave(s, w, "hers_search_batch"); return; }
  for (size_t i = 0; i < nr; ++i) {
    Request* r = w.reqs[i];
    char* rb = base + r->off;
    if (hers_decrypt_scores(s->ctx, s->sk, sc[i], ms[i], (int32_t*)(rb + r->o_out), ws_dec, w.dec_ws, st)) {
      fail_wave(s, w, "hers_decrypt_scores");
      return;
    }
  }
  if (hipEventRecord(w.ev, st) != hipSuccess) fail_wave(s, w, "event");
}

// Applies a finished (or failed) wave to its requests and returns its
// workspace; called with the lock held.
void retire_wave(hers_server* s, Wave& w) {
  const double t = now_ms();
  for (Request* r : w.reqs) {
    r->t_done = t;
    if (w.failed) {
      r->state = 3;
      r->error = w.error;
    } else {
      r->state = 2;
    }
    s->st.completed += 1;
  }
  s->arena.release(w.ws_off, w.ws_bytes);
  s->stream_busy[w.stream] = false;
}

void worker_main(hers_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  // generations seen at the last failed admission (memory short): the worker
  // does not try again until results are collected or a request arrives
  bool blocked = false;
  uint64_t seen_mem = 0, seen_queue = 0;
  while (true) {
    // retire finished waves
    for (size_t i = 0; i < s->inflight.size();) {
      Wave& w = s->inflight[i];
      bool done = w.failed;
      if (!done) {
        const hipError_t q = hipEventQuery(w.ev);
        if (q == hipSuccess) {
          done = true;
        } else if (q != hipErrorNotReady) {
          w.failed = done = true;
          w.error = std::string("wave: ") + hipGetErrorString(q);
        }
      }
      if (done) {
        retire_wave(s, w);
        s->inflight.erase(s->inflight.begin() + i);
        s->cv_done.notify_all();
        blocked = false;                 // its workspace is free again
      } else {
        ++i;
      }
    }
    if (s->stop) {
      // no new waves once stopping: queued requests fail, in-flight ones finish
      for (Request* r : s->queue) {
        r->state = 3;
        r->error = "server stopped";
      }
      s->queue.clear();
      s->cv_done.notify_all();
      if (s->inflight.empty()) break;
    }
    if (blocked && (s->mem_gen != seen_mem || s->queue_gen != seen_queue)) blocked = false;
    // admit a wave: the oldest queued request and the later ones on its
    // gallery, in arrival order, while memory allows
    if (!blocked && (int)s->inflight.size() < SRV_STREAMS && !s->queue.empty()) {
      Wave w;
      const int32_t gid = s->queue.front()->gid;
      const Gallery gal = s->galleries[gid];
      w.enc_ws = s->enc_ws;
      w.dec_ws = s->dec_ws;
      bool short_of_memory = false;
      for (auto it = s->queue.begin(); it != s->queue.end() && (int)w.reqs.size() < s->max_batch;) {
        Request* r = *it;
        if (r->gid != gid) { ++it; continue; }
        size_t off;
        if (!s->arena.alloc(r->bytes, &off)) {
          short_of_memory = true;
          break;
        }
        r->off = off;
        r->in_arena = true;
        r->state = 1;
        r->t_start = now_ms();
        w.reqs.push_back(r);
        w.gals.push_back(gal);
        it = s->queue.erase(it);
      }
      // the wave's workspace: rounds of cb blocks, halved while it does not
      // fit; when it does not fit at one block, the newest request of the
      // wave goes back to the queue (in arrival order) and frees its range
      const int64_t cb_max = std::min<int64_t>((int64_t)hers_blocks(s->ctx, gal.m), SRV_MAX_ROUND);
      while (!w.reqs.empty()) {
        bool fits = false;
        for (int64_t cb = cb_max;; cb = (cb + 1) / 2) {
          w.ws_bytes = wave_ws_bytes(s, w.enc_ws, w.dec_ws, w.reqs.size(), cb);
          if (s->arena.alloc(w.ws_bytes, &w.ws_off)) { fits = true; break; }
          if (cb == 1) break;
        }
        if (fits) break;
        short_of_memory = true;
        Request* r = w.reqs.back();
        w.reqs.pop_back();
        w.gals.pop_back();
        r->state = 0;
        r->in_arena = false;
        s->arena.release(r->off, r->bytes);
        auto pos = s->queue.begin();
        while (pos != s->queue.end() && (*pos)->ticket < r->ticket) ++pos;
        s->queue.insert(pos, r);
      }
      if (short_of_memory) s->st.deferrals += 1;
      if (!w.reqs.empty()) {
        w.stream = 0;
        while (s->stream_busy[w.stream]) ++w.stream;     // fewer than SRV_STREAMS waves are in flight
        s->stream_busy[w.stream] = true;
        w.ev = s->events[w.stream];
        s->st.waves += 1;
        s->st.max_wave = std::max<int64_t>(s->st.max_wave, (int64_t)w.reqs.size());
        s->st.arena_peak = s->arena.peak();
        lk.unlock();
        launch_wave(s, w);
        lk.lock();
        s->inflight.push_back(std::move(w));
        continue;
      }
      if (short_of_memory) {
        blocked = true;
        seen_mem = s->mem_gen;
        seen_queue = s->queue_gen;
      }
    }
    if (s->inflight.empty()) {
      // nothing on the GPU: sleep until there is something to admit (the
      // predicate is false while admission is blocked, so the lock is released)
      s->cv_work.wait(lk, [&] {
        return s->stop || (!s->queue.empty() &&
                           (!blocked || s->mem_gen != seen_mem || s->queue_gen != seen_queue));
      });
    } else {
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

// Streams and events of a server (those created so far).
void release_device(hers_server* s) {
  for (int i = 0; i < SRV_STREAMS; ++i) {
    if (s->events[i]) (void)hipEventDestroy(s->events[i]);
    if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
  }
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
}

}  // namespace

extern "C" {

int hers_server_create(hers_ctx* ctx, const uint8_t* sk_dev, void* arena_dev, size_t arena_bytes, int32_t max_batch,
                       hers_server** out) {
  if (!ctx || !sk_dev || !arena_dev || !out || max_batch < 1) return HERS_EINVAL;
  *out = nullptr;
  hers_server* s = new hers_server(ctx, sk_dev, (char*)arena_dev, arena_bytes, max_batch);
  if (hers_ctx_info(ctx, &s->info)) { delete s; return HERS_EINVAL; }
  s->bound = s->info.feature_bound;
  (void)hipGetDevice(&s->device);
  bool ok = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < SRV_STREAMS; ++i)
    ok = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    release_device(s);
    delete s;
    return HERS_EDEVICE;
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return HERS_OK;
}

int hers_server_add_gallery(hers_server* s, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                            int32_t* gallery_id) {
  if (!s || !gallery_dev || m < 1 || d < 1 || !gallery_id) return HERS_EINVAL;
  const uint64_t blk = hers_gallery_words(s->ctx, s->info.n, d);
  if (!blk || gallery_words % blk || gallery_words < hers_gallery_words(s->ctx, m, d)) {
    hers::set_last_error("gallery buffer length is not whole blocks of d dimensions covering the m items");
    return HERS_EDIM;
  }
  std::lock_guard<std::mutex> g(s->mu);
  s->galleries.push_back({gallery_dev, gallery_words, m, d});
  *gallery_id = (int32_t)s->galleries.size() - 1;
  s->enc_ws = std::max<size_t>(s->enc_ws, hers_workspace_bytes(s->ctx, 1, 0, d));
  s->dec_ws = std::max<size_t>(s->dec_ws, hers_workspace_bytes(s->ctx, 3, std::min<int64_t>(m, 256 * (int64_t)s->info.n), 1));
  return HERS_OK;
}

int hers_server_submit(hers_server* s, int32_t gallery_id, const int32_t* query, uint64_t seed, int64_t* ticket) {
  if (!s || !query || !ticket) return HERS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (gallery_id < 0 || gallery_id >= (int32_t)s->galleries.size()) return HERS_EINVAL;
  const Gallery& gal = s->galleries[gallery_id];
  const int64_t bound = (int64_t)s->bound;
  for (int32_t i = 0; i < gal.d; ++i)
    if ((int64_t)query[i] > bound || (int64_t)query[i] < -bound) {
      hers::set_last_error("a query value lies outside [-feature_bound, feature_bound]");
      return HERS_ERANGE;
    }
  Request* r = new Request();
  r->ticket = s->next_ticket++;
  r->gid = gallery_id;
  r->query.assign(query, query + gal.d);
  r->seed = seed;
  r->t_arrival = now_ms();
  r->bytes = request_bytes(s, gal, &r->o_probe, &r->o_ct, &r->o_out);
  if (r->bytes + wave_ws_bytes(s, s->enc_ws, s->dec_ws, 1, 1) > s->arena.size()) { delete r; return HERS_ENOMEM; }
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  s->queue_gen += 1;
  s->st.submitted += 1;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return HERS_OK;
}

int hers_server_wait(hers_server* s, int64_t ticket, int32_t* scores_out, uint64_t* ct_out, double* latency_ms) {
  if (!s) return HERS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return HERS_EINVAL;
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->state >= 2; });
  // the request's wave is retired and only this caller holds the ticket now:
  // copy without the lock
  s->reqs.erase(it);
  const Gallery g = s->galleries[r->gid];
  lk.unlock();
  int rc = r->state == 2 ? HERS_OK : HERS_EDEVICE;
  if (rc != HERS_OK) hers::set_last_error(r->error);
  char* rb = s->arena_base + r->off;
  if (rc == HERS_OK && scores_out &&
      hipMemcpyAsync(scores_out, rb + r->o_out, (size_t)g.m * 4, hipMemcpyDeviceToHost, s->copy_stream) != hipSuccess)
    rc = HERS_EDEVICE;
  if (rc == HERS_OK && ct_out &&
      hipMemcpyAsync(ct_out, rb + r->o_ct, hers_blocks(s->ctx, g.m) * hers_ct_words(s->ctx) * 8,
                     hipMemcpyDeviceToHost, s->copy_stream) != hipSuccess)
    rc = HERS_EDEVICE;
  if ((scores_out || ct_out) && hipStreamSynchronize(s->copy_stream) != hipSuccess) rc = HERS_EDEVICE;
  if (latency_ms) *latency_ms = r->t_done - r->t_arrival;
  lk.lock();
  if (r->in_arena) {
    s->arena.release(r->off, r->bytes);
    s->mem_gen += 1;                   // a worker short of memory may admit again
  }
  delete r;
  s->cv_work.notify_one();
  return rc;
}

int hers_server_stats_get(hers_server* s, hers_server_stats* out) {
  if (!s || !out) return HERS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  out->arena_peak = s->arena.peak();
  out->queued = (int64_t)s->queue.size();
  out->in_flight = (int64_t)s->inflight.size();
  return HERS_OK;
}

void hers_server_destroy(hers_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->reqs) delete kv.second;
  release_device(s);
  delete s;
}

}  // extern "C"
