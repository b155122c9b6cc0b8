// Continuous batching of gasket life solves, natively: a request queue,
// first-come first-served admission by HBM footprint, a device buffer pool
// recycled by level, and scheduling rounds that queue batched passes
// (sg_pass_run) over every resident request without waiting for the device
// until a request finishes or a horizon of queued cell updates is reached.
//
// Requests may also carry pinned host states: such a request is uploaded when
// it is admitted and its result read back when it finishes, each on a copy
// stream of its own, so transfers overlap the passes of other requests; the
// request takes part in passes between the two.  A cap on the requests in
// flight (1: one request at a time through the same loop) and a replay loop
// that submits requests at their arrival times complete the serving path.
//
// Host code only; the passes are the library's batched life kernel.  A server
// is used from one host thread.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "../../include/sg.h"
#include "sg_launch.h"

namespace {

constexpr int kMinLevel = 6;  // the batched pass's smallest tile is 64 cells a side

uint64_t pow3u(int e) {
  uint64_t v = 1;
  for (int i = 0; i < e; ++i) v *= 3;
  return v;
}

uint64_t footprint(int r) { return 2ull << (2 * r); }  // two n x n uint8 buffers

enum class Phase { Uploading, Active, Downloading };

struct Req {
  uint64_t tag;
  int r, steps, remaining;
  const uint8_t *init;  // device state, or pinned host state (host_io)
  uint8_t *out;         // caller's copy of the result (device, or pinned host), or NULL
  bool host_io;
  uint8_t *buf[2];
  int cur;              // buffer holding the current state
  Phase phase;
  hipEvent_t ev;        // end of the upload or download of a host request
};

}  // namespace

struct sg_server {
  sg_tune tune;
  uint64_t cap, horizon, budget, used = 0;
  uint64_t allocated = 0;      // device bytes of every buffer held (pool, resident, results)
  uint64_t max_allocated = 0;
  int max_requests;
  int max_active = 0;                             // requests in flight at most (0: any)
  int transfer_window = 1;                        // host transfers in flight at most (0: any)
  hipStream_t stream;
  hipStream_t up = nullptr, down = nullptr;       // copy streams of host requests
  sg_pass_ctx *ctx = nullptr;
  std::deque<Req> queue;                          // submitted, not yet admitted
  std::vector<Req> active;                        // in flight (any phase), in admission order
  std::vector<hipEvent_t> events;                 // idle events of host requests
  std::map<int, std::vector<uint8_t *>> pool;     // free buffers by level
  std::vector<std::pair<int, uint8_t *>> held;    // last round's results, freed next round
  std::vector<uint8_t *> owned;                   // every buffer allocated and not freed
  std::vector<sg_pass_item> items;
  sg_server_stats stats = {};
};

namespace {

uint64_t level_bytes(int r) { return 1ull << (2 * r); }

// Frees idle pooled buffers of levels other than `keep` until `need` more
// bytes fit under the cap.  Pooled buffers belong to requests retired by
// earlier rounds, each of which ended with a device wait, so no queued work
// uses them.
void make_room(sg_server *s, int keep, uint64_t need) {
  for (auto &kv : s->pool) {
    if (kv.first == keep) continue;
    auto &v = kv.second;
    while (!v.empty() && s->allocated + need > s->cap) {
      uint8_t *p = v.back();
      v.pop_back();
      (void)hipFree(p);
      s->owned.erase(std::find(s->owned.begin(), s->owned.end(), p));
      s->allocated -= level_bytes(kv.first);
    }
  }
}

// A fresh n x n buffer of level r, keeping the bytes held under the cap;
// cleared on the server's stream (so it holds 0 off the gasket; passes never
// write there) unless `whole` says the caller overwrites all of it (a host
// request's upload, on another stream: a clear queued on the server's stream
// would not be ordered with it).
int new_buffer(sg_server *s, int r, bool whole, uint8_t **out) {
  const uint64_t bytes = level_bytes(r);
  make_room(s, r, bytes);
  if (s->allocated + bytes > s->cap) return SG_ENOMEM;
  uint8_t *p = nullptr;
  if (hipMalloc((void **)&p, bytes) != hipSuccess) return SG_ENOMEM;
  s->owned.push_back(p);
  s->allocated += bytes;
  if (s->allocated > s->max_allocated) s->max_allocated = s->allocated;
  if (!whole && hipMemsetAsync(p, 0, bytes, s->stream) != hipSuccess) return SG_EHIP;
  *out = p;
  return SG_OK;
}

// A zeroed n x n buffer of level r: from the pool, or newly allocated.  The
// admission test keeps the footprints of resident requests under the cap,
// and buffers of other levels that sit idle in the pool are freed before an
// allocation would take the bytes held past it, so the device memory the
// server holds never exceeds the cap.
int take_buffer(sg_server *s, int r, bool whole, uint8_t **out) {
  auto &free = s->pool[r];
  if (!free.empty()) {
    *out = free.back();
    free.pop_back();
    return SG_OK;
  }
  return new_buffer(s, r, whole, out);
}

void release_held(sg_server *s) {
  for (auto &h : s->held) s->pool[h.first].push_back(h.second);
  s->held.clear();
}

int take_event(sg_server *s, hipEvent_t *ev) {
  if (!s->events.empty()) {
    *ev = s->events.back();
    s->events.pop_back();
    return SG_OK;
  }
  return hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess ? SG_OK : SG_EHIP;
}

// Requests holding buffers: uploading, in passes, or downloading.
int in_flight(const sg_server *s) { return (int)s->active.size(); }

// Host requests uploading or reading back.
int transfers(const sg_server *s) {
  int k = 0;
  for (const Req &q : s->active) k += q.phase != Phase::Active;
  return k;
}

}  // namespace


namespace {
// C entry points report an allocation failure inside them as SG_ENOMEM
// rather than letting the exception cross the C ABI.
template <class F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return SG_ENOMEM;
  }
}
}  // namespace

extern "C" {

SG_API int sg_server_create(const sg_tune *tune, uint64_t cap_bytes, int max_requests,
                            uint64_t horizon_cells, uint64_t budget_cells, void *stream,
                            sg_server **out) {
  return guarded([&]() -> int {
    if (!out || !tune || max_requests < 1 || max_requests > (1 << 20) || cap_bytes == 0)
      return SG_EINVAL;
    *out = nullptr;
    if (!sg::life_tb_supported(tune->rho) || tune->steps_per_pass < 1 ||
        tune->steps_per_pass > sg::kMaxStepsPerPass || tune->groups_per_cu < 0 ||
        tune->groups_per_cu > 64 || (tune->threads != 256 && tune->threads != 512))
      return SG_EINVAL;
    std::unique_ptr<sg_server> s(new sg_server());
    s->tune = *tune;
    s->cap = cap_bytes;
    s->horizon = horizon_cells;
    s->budget = budget_cells;
    s->max_requests = max_requests;
    s->stream = (hipStream_t)stream;
    s->items.reserve(max_requests);
    const int st = sg_pass_ctx_create(max_requests, &s->ctx);
    if (st != SG_OK) return st;
    // copy streams at the default priority
    if (hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->down, hipStreamNonBlocking) != hipSuccess) {
      sg_server_destroy(s.release());
      return SG_EHIP;
    }
    *out = s.release();
    return SG_OK;
  });
}

SG_API int sg_server_reserve(sg_server *s, const int32_t *levels, int count) {
  return guarded([&]() -> int {
    if (!s || count < 0 || (count > 0 && !levels)) return SG_EINVAL;
    for (int i = 0; i < count; ++i)
      if (levels[i] < kMinLevel || levels[i] > SG_MAX_R) return SG_EINVAL;
    for (int i = 0; i < count; ++i) {
      if (s->allocated + footprint(levels[i]) > s->cap) break;
      for (int b = 0; b < 2; ++b) {
        const uint64_t bytes = level_bytes(levels[i]);
        uint8_t *p = nullptr;
        if (hipMalloc((void **)&p, bytes) != hipSuccess) return SG_ENOMEM;
        s->owned.push_back(p);
        s->allocated += bytes;
        if (s->allocated > s->max_allocated) s->max_allocated = s->allocated;
        if (hipMemsetAsync(p, 0, bytes, s->stream) != hipSuccess) return SG_EHIP;
        s->pool[levels[i]].push_back(p);
      }
    }
    return hipStreamSynchronize(s->stream) == hipSuccess ? SG_OK : SG_EHIP;
  });
}

SG_API int sg_server_submit(sg_server *s, int r, int steps, const uint8_t *d_init,
                            uint8_t *d_out, uint64_t tag) {
  return guarded([&]() -> int {
    if (!s || r < kMinLevel || r > SG_MAX_R || steps < 0 || !d_init || ((uintptr_t)d_init & 15u) ||
        ((uintptr_t)d_out & 15u))
      return SG_EINVAL;
    if ((int)(s->queue.size() + s->active.size()) >= s->max_requests) return SG_ENOMEM;
    s->queue.push_back(Req{tag, r, steps, steps, d_init, d_out, false, {nullptr, nullptr}, 0,
                           Phase::Active, nullptr});
    return SG_OK;
  });
}

SG_API int sg_server_submit_host(sg_server *s, int r, int steps, const uint8_t *h_init,
                                 uint8_t *h_out, uint64_t tag) {
  return guarded([&]() -> int {
    if (!s || r < kMinLevel || r > SG_MAX_R || steps < 0 || !h_init) return SG_EINVAL;
    if ((int)(s->queue.size() + s->active.size()) >= s->max_requests) return SG_ENOMEM;
    s->queue.push_back(Req{tag, r, steps, steps, h_init, h_out, true, {nullptr, nullptr}, 0,
                           Phase::Uploading, nullptr});
    return SG_OK;
  });
}

SG_API int sg_server_set_max_active(sg_server *s, int max_active) {
  if (!s || max_active < 0) return SG_EINVAL;
  s->max_active = max_active;
  return SG_OK;
}

SG_API int sg_server_set_transfer_window(sg_server *s, int window) {
  if (!s || window < 0) return SG_EINVAL;
  s->transfer_window = window;
  return SG_OK;
}

SG_API int sg_server_step(sg_server *s, sg_server_done *done, int max_done, int *n_done) {
  return guarded([&]() -> int {
    if (!s || !n_done || max_done < 0 || (max_done > 0 && !done)) return SG_EINVAL;
    *n_done = 0;
    release_held(s);
    if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
    // host requests whose upload or download has ended
    {
      std::vector<Req> still;
      still.reserve(s->active.size());
      for (Req &q : s->active) {
        if (q.phase != Phase::Active) {
          const hipError_t e = hipEventQuery(q.ev);
          if (e != hipSuccess && e != hipErrorNotReady) return SG_EHIP;
          if (e == hipSuccess && (q.phase == Phase::Uploading || *n_done < max_done)) {
            s->events.push_back(q.ev);
            q.ev = nullptr;
            if (q.phase == Phase::Uploading) {
              q.phase = Phase::Active;  // joins this round's passes
            } else {                    // read back: the request is done
              done[(*n_done)++] = sg_server_done{q.tag, q.out, 0};
              s->pool[q.r].push_back(q.buf[0]);
              s->pool[q.r].push_back(q.buf[1]);
              s->used -= footprint(q.r);
              ++s->stats.completed;
              s->stats.cell_steps += pow3u(q.r) * (uint64_t)q.steps;
              continue;
            }
          }
        }
        still.push_back(q);
      }
      s->active.swap(still);
    }
    // admission, first come first served while the footprint fits (and the
    // number of requests in flight stays within max_active, if set)
    bool queued_work = false;  // work queued on the server's stream this round
    while (!s->queue.empty()) {
      if (s->max_active && in_flight(s) >= s->max_active) break;
      Req q = s->queue.front();
      // a host request's upload waits while the transfer window is full:
      // host-device copies in both directions share one link, and uploads
      // of later requests interleaved with earlier requests' read-backs
      // would delay those
      if (q.host_io && s->transfer_window && transfers(s) >= s->transfer_window) break;
      const uint64_t fp = footprint(q.r);
      if (fp > s->cap) {  // can never fit
        if (*n_done >= max_done) break;
        s->queue.pop_front();
        done[(*n_done)++] = sg_server_done{q.tag, nullptr, 1};
        ++s->stats.rejected;
        continue;
      }
      if (s->used + fp > s->cap) break;
      int st = take_buffer(s, q.r, q.host_io, &q.buf[0]);
      if (st != SG_OK) return st;
      st = take_buffer(s, q.r, false, &q.buf[1]);
      if (st != SG_OK) {
        s->pool[q.r].push_back(q.buf[0]);  // stays owned, back in the pool
        return st;
      }
      const size_t bytes = (size_t)1 << (2 * q.r);
      if (q.host_io) {
        st = take_event(s, &q.ev);
        if (st == SG_OK && (hipMemcpyAsync(q.buf[0], q.init, bytes, hipMemcpyHostToDevice,
                                           s->up) != hipSuccess ||
                            hipEventRecord(q.ev, s->up) != hipSuccess))
          st = SG_EHIP;
        if (st != SG_OK) {
          s->pool[q.r].push_back(q.buf[0]);
          s->pool[q.r].push_back(q.buf[1]);
          return st;
        }
        q.phase = Phase::Uploading;
      } else {
        if (hipMemcpyAsync(q.buf[0], q.init, bytes, hipMemcpyDeviceToDevice, s->stream) !=
            hipSuccess)
          return SG_EHIP;
        q.phase = Phase::Active;
        queued_work = true;
      }
      s->queue.pop_front();
      s->used += fp;
      s->active.push_back(q);
    }
    if (s->used > s->stats.max_resident_bytes) s->stats.max_resident_bytes = s->used;
    if (s->active.size() > s->stats.max_active) s->stats.max_active = s->active.size();
    // passes over the requests in passes, queued back to back until one
    // finishes or the horizon
    const int T = s->tune.steps_per_pass;
    bool finished = false, any = false;
    for (const Req &q : s->active)
      if (q.phase == Phase::Active) {
        any = true;
        finished |= q.remaining == 0;
      }
    if (!any) return SG_OK;
    uint64_t queued = 0;
    std::vector<int> idx;  // active requests in this round's passes
    idx.reserve(s->active.size());
    for (int i = 0; i < (int)s->active.size(); ++i)
      if (s->active[i].phase == Phase::Active) idx.push_back(i);
    while (!finished) {
      s->items.clear();
      uint64_t spent = 0;
      for (int i : idx) {
        Req &q = s->active[i];
        int k = q.remaining < T ? q.remaining : T;
        const uint64_t cost = pow3u(q.r) * (uint64_t)k;
        if (spent > 0 && s->budget && spent + cost > s->budget) k = 0;  // the first always runs
        if (k > 0) spent += cost;
        s->items.push_back(sg_pass_item{q.buf[q.cur], q.buf[1 - q.cur], q.r, k});
      }
      if (spent > 0) {
        const int st =
            sg_pass_run(s->ctx, s->items.data(), (int)s->items.size(), &s->tune, s->stream);
        if (st != SG_OK) return st;
        ++s->stats.passes;
        queued_work = true;
      }
      for (size_t j = 0; j < idx.size(); ++j) {
        Req &q = s->active[idx[j]];
        const int k = s->items[j].steps;
        if (k > 0) {
          q.remaining -= k;
          q.cur = 1 - q.cur;
        }
        finished |= q.remaining == 0;
      }
      queued += spent;
      if (!s->horizon || queued >= s->horizon) break;
    }
    // the callers' device copies of finished results, ordered after the passes
    for (int i : idx) {
      const Req &q = s->active[i];
      if (q.remaining == 0 && !q.host_io && q.out) {
        if (hipMemcpyAsync(q.out, q.buf[q.cur], (size_t)1 << (2 * q.r),
                           hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
          return SG_EHIP;
        queued_work = true;
      }
    }
    if (queued_work) {
      if (hipStreamSynchronize(s->stream) != hipSuccess) return SG_EHIP;
      ++s->stats.rounds;
    }
    // retire finished device requests (their result buffers stay valid until
    // the next step); start the read-back of finished host requests
    std::vector<Req> still;
    still.reserve(s->active.size());
    for (Req &q : s->active) {
      if (q.phase != Phase::Active || q.remaining > 0) {
        still.push_back(q);
        continue;
      }
      if (q.host_io && q.out) {
        int st = take_event(s, &q.ev);
        if (st == SG_OK && (hipMemcpyAsync(q.out, q.buf[q.cur], (size_t)1 << (2 * q.r),
                                           hipMemcpyDeviceToHost, s->down) != hipSuccess ||
                            hipEventRecord(q.ev, s->down) != hipSuccess))
          st = SG_EHIP;
        if (st != SG_OK) return st;
        q.phase = Phase::Downloading;
        still.push_back(q);
        continue;
      }
      if (*n_done >= max_done) {
        still.push_back(q);
        continue;
      }
      done[(*n_done)++] = sg_server_done{q.tag, q.host_io ? nullptr : q.buf[q.cur], 0};
      s->held.push_back({q.r, q.buf[0]});
      s->held.push_back({q.r, q.buf[1]});
      s->used -= footprint(q.r);
      ++s->stats.completed;
      s->stats.cell_steps += pow3u(q.r) * (uint64_t)q.steps;
    }
    s->active.swap(still);
    return SG_OK;
  });
}

// Seconds since `t0` on the steady clock.
static double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

SG_API int sg_server_replay(sg_server *s, const sg_server_request *reqs, int count,
                            double *finish_s, int32_t *rejected) {
  return guarded([&]() -> int {
    if (!s || count < 0 || (count > 0 && (!reqs || !finish_s || !rejected))) return SG_EINVAL;
    for (int i = 0; i < count; ++i) {
      if (!(reqs[i].arrival_s >= 0.0) || (i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s))
        return SG_EINVAL;  // arrivals in order, from 0
      finish_s[i] = -1.0;
      rejected[i] = 0;
    }
    if (!s->queue.empty() || !s->active.empty()) return SG_EINVAL;  // an idle server
    std::vector<sg_server_done> done((size_t)s->max_requests);
    const auto t0 = std::chrono::steady_clock::now();
    int next = 0, open = 0;
    while (next < count || open > 0) {
      const double now = seconds_since(t0);
      while (next < count && reqs[next].arrival_s <= now) {
        const sg_server_request &q = reqs[next];
        const int st = q.host ? sg_server_submit_host(s, q.r, q.steps, q.init, q.out,
                                                      (uint64_t)next)
                              : sg_server_submit(s, q.r, q.steps, q.init, q.out, (uint64_t)next);
        if (st != SG_OK) return st;
        ++next;
        ++open;
      }
      if (open == 0) continue;  // idle until the next arrival
      int n = 0;
      const int st = sg_server_step(s, done.data(), (int)done.size(), &n);
      if (st != SG_OK) return st;
      const double t = seconds_since(t0);
      for (int k = 0; k < n; ++k) {
        const int i = (int)done[k].tag;
        finish_s[i] = t;
        rejected[i] = done[k].rejected;
        --open;
      }
    }
    return SG_OK;
  });
}

SG_API int sg_server_get_stats(const sg_server *s, sg_server_stats *out) {
  if (!s || !out) return SG_EINVAL;
  *out = s->stats;
  out->queued = s->queue.size();
  out->active = s->active.size();
  out->resident_bytes = s->used;
  out->allocated_bytes = s->allocated;
  out->max_allocated_bytes = s->max_allocated;
  out->transferring = (uint64_t)transfers(s);
  return SG_OK;
}

SG_API void sg_server_destroy(sg_server *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->up) (void)hipStreamSynchronize(s->up);
  if (s->down) (void)hipStreamSynchronize(s->down);
  sg_pass_ctx_destroy(s->ctx);
  for (uint8_t *p : s->owned) (void)hipFree(p);
  for (const Req &q : s->active)
    if (q.ev) (void)hipEventDestroy(q.ev);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->up) (void)hipStreamDestroy(s->up);
  if (s->down) (void)hipStreamDestroy(s->down);
  delete s;
}

}  // extern "C"
