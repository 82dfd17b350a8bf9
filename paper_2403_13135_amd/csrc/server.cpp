// server.cpp -- continuous-batching request server over sil_label_batch
// (interface and model in include/sil_server.h).
//
// Host-side runtime: a FIFO admission queue gated by a first-fit HBM arena
// for outputs, an active list of admitted requests with chips left, and a
// window of in-flight batched launches retired through HIP events.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "sil.h"
#include "sil_server.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kCopyEvents = 256;  // host-scene copies whose launches are still to enqueue

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// Label rows start on 128-byte boundaries, so the labeller writes whole
// cache lines (rows of W bytes rounded up).
int64_t label_pitch_of(int32_t W) { return ((int64_t)W + 127) / 128 * 128; }

struct Req {
  sil_request r;
  int32_t nchips = 0, next_chip = 0;
  int32_t ncy = 0, ncx = 0;
  uint64_t off = 0, bytes = 0, hist_off = 0;
  uint64_t in_off = 0, in_bytes = 0;  // a host scene's bands in the arena
  hipEvent_t ready = nullptr;         // its copy, while launches remain to enqueue
  int32_t outstanding = 0, launches = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool admitted = false, done = false;
};

struct Launch {
  hipEvent_t ev;
  std::vector<uint64_t> tags;
};

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
 public:
  explicit Arena(uint64_t size) : size_(size) { free_[0] = size; }
  bool alloc(uint64_t n, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        uint64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
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
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  uint64_t size() const { return size_; }

 private:
  uint64_t size_, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct sil_server {
  sil_params p;
  sil_server_config cfg;
  char* base = nullptr;
  Arena* arena = nullptr;
  std::vector<hipStream_t> streams;
  hipStream_t copy_stream = nullptr;
  std::vector<hipEvent_t> event_pool;
  std::vector<hipEvent_t> copy_events;
  hipEvent_t epoch = nullptr;
  Clock::time_point epoch_host;
  std::deque<uint64_t> queue;
  std::deque<uint64_t> active;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<Launch> inflight;
  std::deque<uint64_t> completed;
  int next_stream = 0;
  sil_server_stats st{};

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - epoch_host).count();
  }

  uint64_t out_bytes(int32_t H, int32_t W, int32_t ncy, int32_t ncx) const {
    return align_up((uint64_t)H * (uint64_t)label_pitch_of(W)) +
           align_up((uint64_t)ncy * ncx * 3 * 4);
  }
  uint64_t esize() const { return p.dtype == SIL_U16 ? 2 : 1; }

  // Retire launches whose events have completed.
  int retire() {
    for (auto it = inflight.begin(); it != inflight.end();) {
      hipError_t q = hipEventQuery(it->ev);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (q != hipSuccess) return SIL_EDEVICE;
      float ms = 0;
      if (hipEventElapsedTime(&ms, epoch, it->ev) != hipSuccess) return SIL_EDEVICE;
      for (uint64_t tag : it->tags) {
        Req& rq = reqs.at(tag);
        rq.t_done = std::max(rq.t_done, (double)ms);
        if (--rq.outstanding == 0 && rq.next_chip == rq.nchips) {
          rq.done = true;
          completed.push_back(tag);
          ++st.completed;
        }
      }
      event_pool.push_back(it->ev);
      it = inflight.erase(it);
    }
    return SIL_OK;
  }

  // Admit from the head of the queue while its bytes fit; a host scene's
  // three bands are copied into the arena on the copy stream (returns
  // SIL_EDEVICE if a copy cannot be enqueued).
  int admit() {
    while (!queue.empty()) {
      Req& rq = reqs.at(queue.front());
      const bool host = rq.r.flags & SIL_REQ_HOST_SCENE;
      if (host && copy_events.empty()) break;
      uint64_t off;
      if (!arena->alloc(rq.bytes, &off)) break;
      rq.off = off;
      rq.hist_off = off + align_up((uint64_t)rq.r.H * (uint64_t)label_pitch_of(rq.r.W));
      if (host) {
        rq.in_off = rq.hist_off + align_up((uint64_t)rq.ncy * rq.ncx * 3 * 4);
        const uint64_t plane = (uint64_t)rq.r.H * (uint64_t)rq.r.pitch * esize();
        for (int b = 0; b < 3; ++b)
          if (hipMemcpyAsync(base + rq.in_off + b * plane,
                             (const char*)rq.r.scene + (uint64_t)rq.r.sel[b] * plane, plane,
                             hipMemcpyHostToDevice, copy_stream) != hipSuccess)
            return SIL_EDEVICE;
        rq.ready = copy_events.back();
        copy_events.pop_back();
        if (hipEventRecord(rq.ready, copy_stream) != hipSuccess) return SIL_EDEVICE;
      }
      rq.admitted = true;
      rq.t_admit = now_ms();
      active.push_back(queue.front());
      queue.pop_front();
      ++st.admitted;
    }
    return SIL_OK;
  }

  int launch_one() {
    sil_job jobs[SIL_BATCH_MAX_JOBS];
    uint64_t tags[SIL_BATCH_MAX_JOBS];
    int n = 0;
    int32_t budget = cfg.max_chips_per_launch;
    for (auto it = active.begin(); it != active.end() && n < SIL_BATCH_MAX_JOBS && budget > 0;
         ++it) {
      Req& rq = reqs.at(*it);
      int32_t cnt = std::min(rq.nchips - rq.next_chip, budget);
      if (cnt <= 0) continue;
      sil_job& j = jobs[n];
      if (rq.r.flags & SIL_REQ_HOST_SCENE) {  // the arena copy of its three bands
        j.scene = base + rq.in_off;
        j.nbands = 3;
        for (int b = 0; b < 3; ++b) j.sel[b] = b;
      } else {
        j.scene = rq.r.scene;
        j.nbands = rq.r.nbands;
        for (int b = 0; b < 3; ++b) j.sel[b] = rq.r.sel[b];
      }
      j.H = rq.r.H;
      j.W = rq.r.W;
      j.pitch = rq.r.pitch;
      j.labels = (uint8_t*)(base + rq.off);
      j.label_pitch = label_pitch_of(rq.r.W);
      j.hist = (uint32_t*)(base + rq.hist_off);
      j.chips = nullptr;
      j.chip_begin = rq.next_chip;
      j.chip_count = cnt;
      tags[n++] = *it;
      budget -= cnt;
    }
    if (n == 0) return SIL_OK;
    hipStream_t sm = streams[next_stream];
    next_stream = (next_stream + 1) % (int)streams.size();
    for (int i = 0; i < n; ++i) {
      const Req& rq = reqs.at(tags[i]);
      if (rq.ready && hipStreamWaitEvent(sm, rq.ready, 0) != hipSuccess) return SIL_EDEVICE;
    }
    int rc = sil_label_batch(jobs, n, &p, (void*)sm);
    if (rc != SIL_OK) return rc;
    if (event_pool.empty()) return SIL_EDEVICE;
    Launch L;
    L.ev = event_pool.back();
    event_pool.pop_back();
    if (hipEventRecord(L.ev, sm) != hipSuccess) return SIL_EDEVICE;
    int64_t chips = 0;
    for (int i = 0; i < n; ++i) {
      Req& rq = reqs.at(tags[i]);
      rq.next_chip += jobs[i].chip_count;
      chips += jobs[i].chip_count;
      ++rq.outstanding;
      ++rq.launches;
      L.tags.push_back(tags[i]);
      if (rq.ready && rq.next_chip == rq.nchips) {
        // every launch that reads the copy waits on it already; the event
        // may be recorded again for another request
        copy_events.push_back(rq.ready);
        rq.ready = nullptr;
      }
    }
    active.erase(std::remove_if(active.begin(), active.end(),
                                [&](uint64_t t) {
                                  const Req& rq = reqs.at(t);
                                  return rq.next_chip == rq.nchips;
                                }),
                 active.end());
    inflight.push_back(std::move(L));
    ++st.launches;
    st.chips += (uint64_t)chips;
    return SIL_OK;
  }
};

extern "C" {

void sil_server_config_default(sil_server_config* c) {
  if (!c) return;
  c->arena_bytes = 4ull << 30;
  c->max_chips_per_launch = 4096;
  c->max_inflight = 4;
  c->nstreams = 2;
  c->max_queue = 65536;
}

int sil_server_create(const sil_params* p, const sil_server_config* cfg, sil_server** out) {
  if (!p || !cfg || !out) return SIL_EINVAL;
  if (cfg->arena_bytes == 0 || cfg->max_chips_per_launch < 1 || cfg->max_inflight < 1 ||
      cfg->max_inflight > 64 || cfg->nstreams < 1 || cfg->nstreams > 8 || cfg->max_queue < 1)
    return SIL_EINVAL;
  // the batched labeller's parameter rules, checked on a 1x1 probe scene
  const int32_t sel[3] = {0, 1, 2};
  int rc = sil_validate(3, sel, 1, 1, 1, 1, p);
  if (rc != SIL_OK) return rc;
  if (p->filter != 1 || p->patch_h != p->chip || p->patch_w != p->chip) return SIL_EUNSUPPORTED;

  sil_server* s = new (std::nothrow) sil_server();
  if (!s) return SIL_EDEVICE;
  s->p = *p;
  s->cfg = *cfg;
  if (hipMalloc((void**)&s->base, cfg->arena_bytes) != hipSuccess) {
    delete s;
    return SIL_EDEVICE;
  }
  s->arena = new Arena(cfg->arena_bytes);
  bool ok = true;
  for (int i = 0; i < cfg->nstreams && ok; ++i) {
    hipStream_t sm;
    ok = hipStreamCreateWithFlags(&sm, hipStreamNonBlocking) == hipSuccess;
    if (ok) s->streams.push_back(sm);
  }
  for (int i = 0; i < cfg->max_inflight && ok; ++i) {
    hipEvent_t e;
    ok = hipEventCreate(&e) == hipSuccess;
    if (ok) s->event_pool.push_back(e);
  }
  ok = ok && hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < kCopyEvents && ok; ++i) {
    hipEvent_t e;
    ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (ok) s->copy_events.push_back(e);
  }
  ok = ok && hipEventCreate(&s->epoch) == hipSuccess;
  ok = ok && hipStreamSynchronize(s->streams[0]) == hipSuccess;
  ok = ok && hipEventRecord(s->epoch, s->streams[0]) == hipSuccess;
  ok = ok && hipEventSynchronize(s->epoch) == hipSuccess;
  s->epoch_host = Clock::now();
  if (!ok) {
    sil_server_destroy(s);
    return SIL_EDEVICE;
  }
  *out = s;
  return SIL_OK;
}

int sil_server_submit(sil_server* s, const sil_request* r) {
  if (!s || !r || !r->scene || (r->flags & ~SIL_REQ_HOST_SCENE)) return SIL_EINVAL;
  int rc = sil_validate(r->nbands, r->sel, r->H, r->W, r->pitch, r->W, &s->p);
  if (rc != SIL_OK) return rc;
  if (s->reqs.count(r->tag)) return SIL_EINVAL;
  if ((int64_t)s->queue.size() >= s->cfg.max_queue) return SIL_EUNSUPPORTED;
  Req rq;
  rq.r = *r;
  const int32_t C = (int32_t)s->p.chip;
  rq.ncy = (r->H + C - 1) / C;
  rq.ncx = (r->W + C - 1) / C;
  rq.nchips = rq.ncy * rq.ncx;
  rq.bytes = s->out_bytes(r->H, r->W, rq.ncy, rq.ncx);
  if (r->flags & SIL_REQ_HOST_SCENE) {
    rq.in_bytes = align_up(3 * (uint64_t)r->H * (uint64_t)r->pitch * s->esize());
    rq.bytes += rq.in_bytes;
  }
  if (rq.bytes > s->arena->size()) return SIL_EINVAL;
  rq.t_submit = s->now_ms();
  s->reqs.emplace(r->tag, rq);
  s->queue.push_back(r->tag);
  ++s->st.submitted;
  return SIL_OK;
}

int sil_server_pump(sil_server* s, int32_t* n_launched) {
  if (!s) return SIL_EINVAL;
  int32_t n = 0;
  int rc = s->retire();
  if (rc != SIL_OK) return rc;
  rc = s->admit();
  if (rc != SIL_OK) return rc;
  while ((int32_t)s->inflight.size() < s->cfg.max_inflight && !s->active.empty()) {
    rc = s->launch_one();
    if (rc != SIL_OK) return rc;
    ++n;
    rc = s->admit();
    if (rc != SIL_OK) return rc;
  }
  if (n_launched) *n_launched = n;
  return SIL_OK;
}

int sil_server_poll(sil_server* s, sil_completion* out, int32_t max, int32_t* n) {
  if (!s || !n || (max > 0 && !out)) return SIL_EINVAL;
  int rc = s->retire();
  if (rc != SIL_OK) return rc;
  int32_t k = 0;
  while (k < max && !s->completed.empty()) {
    const uint64_t tag = s->completed.front();
    s->completed.pop_front();
    const Req& rq = s->reqs.at(tag);
    sil_completion& c = out[k++];
    c.tag = tag;
    c.labels = (uint8_t*)(s->base + rq.off);
    c.hist = (uint32_t*)(s->base + rq.hist_off);
    c.H = rq.r.H;
    c.W = rq.r.W;
    c.launches = rq.launches;
    c.label_pitch = (int32_t)label_pitch_of(rq.r.W);
    c.t_submit_ms = rq.t_submit;
    c.t_admit_ms = rq.t_admit;
    c.t_done_ms = rq.t_done;
  }
  *n = k;
  return SIL_OK;
}

int sil_server_release(sil_server* s, uint64_t tag) {
  if (!s) return SIL_EINVAL;
  auto it = s->reqs.find(tag);
  if (it == s->reqs.end() || !it->second.done) return SIL_EINVAL;
  s->arena->release(it->second.off, it->second.bytes);
  s->reqs.erase(it);
  ++s->st.released;
  return SIL_OK;
}

int sil_server_cancel(sil_server* s, uint64_t tag) {
  if (!s) return SIL_EINVAL;
  auto it = s->reqs.find(tag);
  if (it == s->reqs.end()) return SIL_EINVAL;
  if (it->second.admitted) return SIL_EUNSUPPORTED;
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == tag) {
      s->queue.erase(q);
      break;
    }
  s->reqs.erase(it);
  ++s->st.cancelled;
  return SIL_OK;
}

int sil_server_expire(sil_server* s, double max_wait_ms, uint64_t* tags, int32_t max,
                      int32_t* n) {
  if (!s || !n || max_wait_ms < 0 || (max > 0 && !tags)) return SIL_EINVAL;
  const double now = s->now_ms();
  int32_t k = 0;
  // the queue is in submission order, so the requests that waited longest lead it
  while (k < max && !s->queue.empty()) {
    const uint64_t tag = s->queue.front();
    if (now - s->reqs.at(tag).t_submit <= max_wait_ms) break;
    s->queue.pop_front();
    s->reqs.erase(tag);
    ++s->st.cancelled;
    tags[k++] = tag;
  }
  *n = k;
  return SIL_OK;
}

int sil_server_drain(sil_server* s) {
  if (!s) return SIL_EINVAL;
  for (auto& L : s->inflight)
    if (hipEventSynchronize(L.ev) != hipSuccess) return SIL_EDEVICE;
  return s->retire();
}

int sil_server_get_stats(const sil_server* s, sil_server_stats* out) {
  if (!s || !out) return SIL_EINVAL;
  *out = s->st;
  out->arena_used = s->arena->used();
  out->arena_peak = s->arena->peak();
  out->queued = (int32_t)s->queue.size();
  out->active = (int32_t)s->active.size();
  out->inflight = (int32_t)s->inflight.size();
  return SIL_OK;
}

double sil_server_clock_ms(const sil_server* s) { return s ? s->now_ms() : 0.0; }

int sil_server_run(sil_server* s, const sil_request* reqs, const double* arrival_ms, int32_t n,
                   int32_t release, sil_completion* out, double* start_ms) {
  if (!s || !reqs || !arrival_ms || !out || n < 0) return SIL_EINVAL;
  std::unordered_map<uint64_t, int32_t> index;
  index.reserve((size_t)n * 2);
  for (int32_t i = 0; i < n; ++i) {
    if (i > 0 && arrival_ms[i] < arrival_ms[i - 1]) return SIL_EINVAL;
    if (!index.emplace(reqs[i].tag, i).second) return SIL_EINVAL;
  }
  const double t0 = s->now_ms();
  if (start_ms) *start_ms = t0;
  int32_t next = 0, done = 0;
  std::vector<sil_completion> buf(64);
  while (done < n) {
    const double now = s->now_ms() - t0;
    while (next < n && arrival_ms[next] <= now) {
      int rc = sil_server_submit(s, &reqs[next]);
      if (rc != SIL_OK) return rc;
      ++next;
    }
    int rc = sil_server_pump(s, nullptr);
    if (rc != SIL_OK) return rc;
    // kept outputs that fill the arena: nothing runs and the queue's head
    // can only be admitted once the caller releases
    if (!release && s->inflight.empty() && s->active.empty() && !s->queue.empty() &&
        s->completed.empty())
      return SIL_EUNSUPPORTED;
    int32_t got = 0;
    rc = sil_server_poll(s, buf.data(), (int32_t)buf.size(), &got);
    if (rc != SIL_OK) return rc;
    for (int32_t k = 0; k < got; ++k) {
      out[index.at(buf[k].tag)] = buf[k];
      if (release) {
        rc = sil_server_release(s, buf[k].tag);
        if (rc != SIL_OK) return rc;
      }
      ++done;
    }
  }
  return SIL_OK;
}

int sil_server_destroy(sil_server* s) {
  if (!s) return SIL_EINVAL;
  int rc = SIL_OK;
  for (auto& L : s->inflight)
    if (hipEventSynchronize(L.ev) != hipSuccess) rc = SIL_EDEVICE;
  for (auto& L : s->inflight) (void)hipEventDestroy(L.ev);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->copy_stream && hipStreamSynchronize(s->copy_stream) != hipSuccess) rc = SIL_EDEVICE;
  for (auto& kv : s->reqs)
    if (kv.second.ready) s->copy_events.push_back(kv.second.ready);
  for (hipEvent_t e : s->copy_events) (void)hipEventDestroy(e);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->epoch) (void)hipEventDestroy(s->epoch);
  for (hipStream_t sm : s->streams) (void)hipStreamDestroy(sm);
  if (s->base) (void)hipFree(s->base);
  delete s->arena;
  delete s;
  return rc;
}

}  // extern "C"
