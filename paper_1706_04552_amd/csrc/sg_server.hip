// Continuous batching of gasket life solves, natively: a request queue,
// first-come first-served admission by HBM footprint, a device buffer pool
// recycled by level, and scheduling rounds that queue batched passes
// (sg_pass_run) over every resident request without waiting for the device
// until a request finishes or a horizon of queued cell updates is reached.
//
// Host code only; the passes are the library's batched life kernel.  A server
// is used from one host thread.
#include <string.h>

#include <algorithm>
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

struct Req {
  uint64_t tag;
  int r, steps, remaining;
  const uint8_t *init;
  uint8_t *out;  // caller's copy of the result, or NULL
  uint8_t *buf[2];
  int cur;  // buffer holding the current state
};

}  // namespace

struct sg_server {
  sg_tune tune;
  uint64_t cap, horizon, budget, used = 0;
  uint64_t allocated = 0;      // device bytes of every buffer held (pool, resident, results)
  uint64_t max_allocated = 0;
  int max_requests;
  hipStream_t stream;
  sg_pass_ctx *ctx = nullptr;
  std::deque<Req> queue;                          // submitted, not yet admitted
  std::vector<Req> active;                        // resident, in admission order
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

// A fresh zeroed n x n buffer of level r (cleared, so it holds 0 off the
// gasket; passes never write there), keeping the bytes held under the cap.
int new_buffer(sg_server *s, int r, uint8_t **out) {
  const uint64_t bytes = level_bytes(r);
  make_room(s, r, bytes);
  if (s->allocated + bytes > s->cap) return SG_ENOMEM;
  uint8_t *p = nullptr;
  if (hipMalloc((void **)&p, bytes) != hipSuccess) return SG_ENOMEM;
  s->owned.push_back(p);
  s->allocated += bytes;
  if (s->allocated > s->max_allocated) s->max_allocated = s->allocated;
  if (hipMemsetAsync(p, 0, bytes, s->stream) != hipSuccess) return SG_EHIP;
  *out = p;
  return SG_OK;
}

// A zeroed n x n buffer of level r: from the pool, or newly allocated.  The
// admission test keeps the footprints of resident requests under the cap,
// and buffers of other levels that sit idle in the pool are freed before an
// allocation would take the bytes held past it, so the device memory the
// server holds never exceeds the cap.
int take_buffer(sg_server *s, int r, uint8_t **out) {
  auto &free = s->pool[r];
  if (!free.empty()) {
    *out = free.back();
    free.pop_back();
    return SG_OK;
  }
  return new_buffer(s, r, out);
}

void release_held(sg_server *s) {
  for (auto &h : s->held) s->pool[h.first].push_back(h.second);
  s->held.clear();
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
    s->queue.push_back(Req{tag, r, steps, steps, d_init, d_out, {nullptr, nullptr}, 0});
    return SG_OK;
  });
}

SG_API int sg_server_step(sg_server *s, sg_server_done *done, int max_done, int *n_done) {
  return guarded([&]() -> int {
    if (!s || !n_done || max_done < 0 || (max_done > 0 && !done)) return SG_EINVAL;
    *n_done = 0;
    release_held(s);
    if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
    // admission, first come first served while the footprint fits
    while (!s->queue.empty()) {
      Req q = s->queue.front();
      const uint64_t fp = footprint(q.r);
      if (fp > s->cap) {  // can never fit
        if (*n_done >= max_done) break;
        s->queue.pop_front();
        done[(*n_done)++] = sg_server_done{q.tag, nullptr, 1};
        ++s->stats.rejected;
        continue;
      }
      if (s->used + fp > s->cap) break;
      int st = take_buffer(s, q.r, &q.buf[0]);
      if (st != SG_OK) return st;
      st = take_buffer(s, q.r, &q.buf[1]);
      if (st != SG_OK) {
        s->pool[q.r].push_back(q.buf[0]);  // stays owned, back in the pool
        return st;
      }
      if (hipMemcpyAsync(q.buf[0], q.init, (size_t)1 << (2 * q.r), hipMemcpyDeviceToDevice,
                         s->stream) != hipSuccess)
        return SG_EHIP;
      s->queue.pop_front();
      s->used += fp;
      s->active.push_back(q);
    }
    if (s->used > s->stats.max_resident_bytes) s->stats.max_resident_bytes = s->used;
    if (s->active.size() > s->stats.max_active) s->stats.max_active = s->active.size();
    if (s->active.empty()) return SG_OK;
    // passes, queued back to back until a request finishes or the horizon
    const int T = s->tune.steps_per_pass;
    uint64_t queued = 0;
    bool finished = false;
    while (!finished) {
      s->items.clear();
      uint64_t spent = 0;
      for (Req &q : s->active) {
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
      }
      for (size_t i = 0; i < s->active.size(); ++i) {
        Req &q = s->active[i];
        const int k = s->items[i].steps;
        if (k > 0) {
          q.remaining -= k;
          q.cur = 1 - q.cur;
        }
        finished |= q.remaining == 0;
      }
      queued += spent;
      if (!s->horizon || queued >= s->horizon) break;
    }
    // the callers' copies of finished results, ordered after the passes
    for (const Req &q : s->active)
      if (q.remaining == 0 && q.out &&
          hipMemcpyAsync(q.out, q.buf[q.cur], (size_t)1 << (2 * q.r), hipMemcpyDeviceToDevice,
                         s->stream) != hipSuccess)
        return SG_EHIP;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return SG_EHIP;
    ++s->stats.rounds;
    // retire finished requests (their result buffers stay valid until the next step)
    std::vector<Req> still;
    still.reserve(s->active.size());
    for (Req &q : s->active) {
      if (q.remaining > 0 || *n_done >= max_done) {
        still.push_back(q);
        continue;
      }
      done[(*n_done)++] = sg_server_done{q.tag, q.buf[q.cur], 0};
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

SG_API int sg_server_get_stats(const sg_server *s, sg_server_stats *out) {
  if (!s || !out) return SG_EINVAL;
  *out = s->stats;
  out->queued = s->queue.size();
  out->active = s->active.size();
  out->resident_bytes = s->used;
  out->allocated_bytes = s->allocated;
  out->max_allocated_bytes = s->max_allocated;
  return SG_OK;
}

SG_API void sg_server_destroy(sg_server *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  sg_pass_ctx_destroy(s->ctx);
  for (uint8_t *p : s->owned) (void)hipFree(p);
  delete s;
}

}  // extern "C"
