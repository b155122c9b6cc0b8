// Batched gaskets: planning, hipGraph capture, the per-iteration pass used by
// continuous batching, and the launch-shape autotuner.
//
// A batch runs many independent gaskets (uneven levels r, each with its own
// number of generations) through the temporally blocked life pass.  Every
// pass is one persistent launch over the lambda tiles of all gaskets still
// running; a gasket with P passes alternates its passes between `out` and
// `work` so that its last pass lands in `out`.
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/sg.h"
#include "sg_launch.h"

namespace {

uint64_t pow3(int e) {
  uint64_t v = 1;
  for (int i = 0; i < e; ++i) v *= 3;
  return v;
}

int rho_log2(int rho) {
  int k = 0;
  while ((1 << k) < rho) ++k;
  return k;
}

bool misaligned(const void *p) { return ((uintptr_t)p & 15u) != 0; }

bool overlaps(const void *a, const void *b, size_t bytes) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + bytes && pb < pa + bytes;
}

int hip_err(hipError_t e) { return e == hipSuccess ? SG_OK : SG_EHIP; }

int check_tune(const sg_tune *t) {
  if (!t) return SG_EINVAL;
  if (!sg::life_tb_supported(t->rho)) return SG_EINVAL;
  if (t->steps_per_pass < 1 || t->steps_per_pass > sg::kMaxStepsPerPass) return SG_EINVAL;
  if (t->groups_per_cu < 0 || t->groups_per_cu > 64) return SG_EINVAL;
  if (t->threads != 256 && t->threads != 512) return SG_EINVAL;
  return SG_OK;
}

// Compute units of the current device (cached per device).
int cu_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  cache[dev] = cus;
  return cus;
}

int groups_for(const sg_tune &t, uint64_t total_tiles) {
  if (t.groups_per_cu == 0 || total_tiles == 0)  // one workgroup per tile
    return (int)std::min<uint64_t>(total_tiles ? total_tiles : 1, 1u << 30);
  const int cus = cu_count();
  const uint64_t g = (uint64_t)(cus > 0 ? cus : 256) * (uint64_t)t.groups_per_cu;
  return (int)std::min<uint64_t>(g, total_tiles);
}

struct Pass {
  std::vector<sg::BatchItem> items;
  uint64_t total_tiles = 0;
  int max_steps = 0;
  uint64_t touched = 0;  // bytes the pass reads and writes (life_touched_bytes)
};

struct Plan {
  std::vector<Pass> passes;
  std::vector<const sg_gasket *> copies;  // gaskets with steps == 0: in -> out
  uint64_t cell_steps = 0;                // sum of 3^r * steps
};

// Tile side of a gasket of level r in a batch whose largest side is 2^kmax:
// the largest supported side (64..2^kmax) that fits in the gasket.
int item_k(int r, int kmax) { return r < kmax ? r : kmax; }

constexpr int kMinTileLog2 = 6;  // smallest temporally blocked tile: 64

int validate_gasket(const sg_gasket &g) {
  if (g.r < kMinTileLog2 || g.r > SG_MAX_R || g.steps < 0) return SG_EINVAL;
  if (!g.in || !g.out || misaligned(g.in) || misaligned(g.out)) return SG_EINVAL;
  const size_t bytes = ((size_t)1 << g.r) * ((size_t)1 << g.r);
  if (overlaps(g.in, g.out, bytes)) return SG_EALIAS;
  return SG_OK;
}

int make_plan(const sg_gasket *gs, int count, const sg_tune &t, Plan &plan) {
  if (!gs || count < 1) return SG_EINVAL;
  const int T = t.steps_per_pass, kmax = rho_log2(t.rho);
  int max_passes = 0;
  for (int i = 0; i < count; ++i) {
    const sg_gasket &g = gs[i];
    int st = validate_gasket(g);
    if (st != SG_OK) return st;
    const int P = (g.steps + T - 1) / T;
    if (P >= 2) {
      const size_t bytes = ((size_t)1 << g.r) * ((size_t)1 << g.r);
      if (!g.work || misaligned(g.work)) return SG_EINVAL;
      if (overlaps(g.work, g.in, bytes) || overlaps(g.work, g.out, bytes)) return SG_EALIAS;
    }
    max_passes = std::max(max_passes, P);
    plan.cell_steps += pow3(g.r) * (uint64_t)g.steps;
    if (g.steps == 0) plan.copies.push_back(&g);
  }
  plan.passes.resize(max_passes);
  for (int p = 0; p < max_passes; ++p) {
    Pass &pass = plan.passes[p];
    for (int i = 0; i < count; ++i) {
      const sg_gasket &g = gs[i];
      const int P = (g.steps + T - 1) / T;
      if (p >= P) continue;
      sg::BatchItem it;
      uint8_t *prev = ((P - 1 - (p - 1)) % 2 == 0) ? g.out : g.work;  // dst of pass p-1
      it.src = p == 0 ? g.in : prev;
      it.dst = ((P - 1 - p) % 2 == 0) ? g.out : g.work;
      it.r = g.r;
      it.steps = (int16_t)(p < P - 1 ? T : g.steps - (P - 1) * T);
      it.k = (int16_t)item_k(g.r, kmax);
      it.tile_begin = pass.total_tiles;
      pass.total_tiles += pow3(g.r - it.k);
      pass.max_steps = std::max(pass.max_steps, (int)it.steps);
      pass.touched += sg::life_touched_bytes(g.r);
      pass.items.push_back(it);
    }
  }
  return SG_OK;
}

// Launches every pass of a plan whose item tables are at d_tables[offsets[p]].
int launch_plan(const Plan &plan, const sg_tune &t, const sg::BatchItem *d_tables,
                const std::vector<size_t> &offsets, hipStream_t s) {
  for (const sg_gasket *g : plan.copies) {
    const size_t bytes = ((size_t)1 << g->r) * ((size_t)1 << g->r);
    const hipError_t e = hipMemcpyAsync(g->out, g->in, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return SG_EHIP;
  }
  for (size_t p = 0; p < plan.passes.size(); ++p) {
    const Pass &pass = plan.passes[p];
    const hipError_t e = sg::launch_life_tb_batch(
        t.rho, t.threads, d_tables + offsets[p], (int)pass.items.size(), pass.total_tiles,
        pass.max_steps, groups_for(t, pass.total_tiles), sg::life_stream_stores(pass.touched), s);
    if (e != hipSuccess) return SG_EHIP;
  }
  return SG_OK;
}

// Device copy of all pass tables; returns offsets (in items) per pass.
int upload_plan(const Plan &plan, sg::BatchItem **d_tables, std::vector<size_t> &offsets) {
  size_t total = 0;
  offsets.clear();
  for (const Pass &p : plan.passes) {
    offsets.push_back(total);
    total += p.items.size();
  }
  *d_tables = nullptr;
  if (total == 0) return SG_OK;
  std::vector<sg::BatchItem> host;
  host.reserve(total);
  for (const Pass &p : plan.passes) host.insert(host.end(), p.items.begin(), p.items.end());
  if (hipMalloc((void **)d_tables, total * sizeof(sg::BatchItem)) != hipSuccess) return SG_ENOMEM;
  if (hipMemcpy(*d_tables, host.data(), total * sizeof(sg::BatchItem), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(*d_tables);
    *d_tables = nullptr;
    return SG_EHIP;
  }
  return SG_OK;
}

}  // namespace

struct sg_batch {
  sg_tune tune;
  Plan plan;
  std::vector<sg_gasket> gaskets;  // plan.copies points into this
  sg::BatchItem *d_tables = nullptr;
  std::vector<size_t> offsets;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// A ring of upload slots, each with its own pinned staging area, device
// table and event, so the host can queue up to kPassRing passes ahead of the
// GPU: pass i uses slot i mod kPassRing and waits only for the upload that
// used the slot kPassRing passes earlier.
constexpr int kPassRing = 8;
struct sg_pass_ctx {
  int capacity = 0;
  int next = 0;                                  // slot of the next pass
  sg::BatchItem *d_items = nullptr;              // kPassRing tables of `capacity` items
  sg::BatchItem *h_stage = nullptr;              // pinned staging, same shape
  hipEvent_t staged[kPassRing] = {};             // slot's last upload has read its staging
  bool pending[kPassRing] = {};
};


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

SG_API int sg_tune_default(sg_tune *t) {
  if (!t) return SG_EINVAL;
  t->rho = 64;
  t->steps_per_pass = sg::kDefaultStepsPerPass;
  t->groups_per_cu = 0;
  t->threads = 256;
  return SG_OK;
}

SG_API int sg_batch_create(const sg_gasket *gaskets, int count, const sg_tune *tune,
                           sg_batch **out) {
  return guarded([&]() -> int {
    if (!out) return SG_EINVAL;
    *out = nullptr;
    int st = check_tune(tune);
    if (st != SG_OK) return st;
    std::unique_ptr<sg_batch, void (*)(sg_batch *)> b(new sg_batch(), sg_batch_destroy);
    b->tune = *tune;
    b->gaskets.assign(gaskets ? gaskets : nullptr, gaskets ? gaskets + std::max(count, 0) : nullptr);
    st = make_plan(b->gaskets.data(), count, b->tune, b->plan);
    if (st == SG_OK) st = upload_plan(b->plan, &b->d_tables, b->offsets);
    if (st == SG_OK && cu_count() <= 0) st = SG_EHIP;  // query the device before capturing
    if (st == SG_OK) {
      // capture every pass into one graph on a private stream
      hipStream_t cs = nullptr;
      st = hip_err(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      if (st == SG_OK) {
        st = hip_err(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (st == SG_OK) {
          const int lst = launch_plan(b->plan, b->tune, b->d_tables, b->offsets, cs);
          const hipError_t ec = hipStreamEndCapture(cs, &b->graph);
          st = lst != SG_OK ? lst : hip_err(ec);
        }
        if (st == SG_OK) st = hip_err(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        (void)hipStreamDestroy(cs);
      }
    }
    if (st != SG_OK) return st;  // the batch is destroyed on the way out
    *out = b.release();
    return SG_OK;
  });
}

SG_API int sg_batch_run(sg_batch *b, void *stream) {
  if (!b || !b->exec) return SG_EINVAL;
  if (sg::inject_hip_error()) return SG_EHIP;
  return hip_err(hipGraphLaunch(b->exec, (hipStream_t)stream));
}

SG_API int sg_batch_run_eager(sg_batch *b, void *stream) {
  if (!b) return SG_EINVAL;
  if (sg::inject_hip_error()) return SG_EHIP;
  return launch_plan(b->plan, b->tune, b->d_tables, b->offsets, (hipStream_t)stream);
}

SG_API int sg_batch_stats(const sg_batch *b, uint64_t *passes, uint64_t *cell_steps) {
  if (!b) return SG_EINVAL;
  if (passes) *passes = b->plan.passes.size();
  if (cell_steps) *cell_steps = b->plan.cell_steps;
  return SG_OK;
}

SG_API void sg_batch_destroy(sg_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_tables) (void)hipFree(b->d_tables);
  delete b;
}

SG_API int sg_batch_autotune(const sg_gasket *gaskets, int count, sg_tune *best,
                             float *best_ms, void *stream) {
  return guarded([&]() -> int {
    if (!best) return SG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return SG_EHIP;
    }
    float best_t = -1.0f;
    int st_any = SG_EINVAL;
    const int rhos[] = {64, 128, 256}, spps[] = {8, 16, 32}, gpcs[] = {0, 2, 4, 8}, thr[] = {256, 512};
    for (int rho : rhos) {
      for (int spp : spps)
        for (int gpc : gpcs)
          for (int th : thr) {
            sg_tune t{rho, spp, gpc, th};
            Plan plan;
            int st = make_plan(gaskets, count, t, plan);
            if (st != SG_OK) {
              st_any = st;
              continue;
            }
            sg::BatchItem *d = nullptr;
            std::vector<size_t> off;
            st = upload_plan(plan, &d, off);
            float ms = 0.0f;
            if (st == SG_OK) st = launch_plan(plan, t, d, off, s);  // warm-up
            if (st == SG_OK) st = hip_err(hipEventRecord(e0, s));
            if (st == SG_OK) st = launch_plan(plan, t, d, off, s);
            if (st == SG_OK) st = hip_err(hipEventRecord(e1, s));
            if (st == SG_OK) st = hip_err(hipEventSynchronize(e1));
            if (st == SG_OK) st = hip_err(hipEventElapsedTime(&ms, e0, e1));
            if (d) (void)hipFree(d);
            if (st != SG_OK) {
              (void)hipEventDestroy(e0);
              (void)hipEventDestroy(e1);
              return st;
            }
            st_any = SG_OK;
            if (best_t < 0.0f || ms < best_t) {
              best_t = ms;
              *best = t;
            }
          }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_t < 0.0f) return st_any;
    if (best_ms) *best_ms = best_t;
    return SG_OK;
  });
}

SG_API int sg_pass_ctx_create(int capacity, sg_pass_ctx **out) {
  return guarded([&]() -> int {
    if (!out || capacity < 1 || capacity > (1 << 24)) return SG_EINVAL;
    *out = nullptr;
    sg_pass_ctx *c = new sg_pass_ctx();
    c->capacity = capacity;
    const size_t bytes = (size_t)kPassRing * (size_t)capacity * sizeof(sg::BatchItem);
    int st = SG_OK;
    if (hipMalloc((void **)&c->d_items, bytes) != hipSuccess) st = SG_ENOMEM;
    if (st == SG_OK && hipHostMalloc((void **)&c->h_stage, bytes, hipHostMallocDefault) != hipSuccess)
      st = SG_ENOMEM;
    for (int k = 0; k < kPassRing && st == SG_OK; ++k)
      st = hip_err(hipEventCreateWithFlags(&c->staged[k], hipEventDisableTiming));
    if (st != SG_OK) {
      sg_pass_ctx_destroy(c);
      return st;
    }
    *out = c;
    return SG_OK;
  });
}

SG_API int sg_pass_run(sg_pass_ctx *ctx, const sg_pass_item *items, int count,
                       const sg_tune *tune, void *stream) {
  return guarded([&]() -> int {
    if (!ctx || count < 0 || count > ctx->capacity || (count > 0 && !items)) return SG_EINVAL;
    int st = check_tune(tune);
    if (st != SG_OK) return st;
    const int kmax = rho_log2(tune->rho);
    // validate everything before touching the staging buffer or the device
    int live = 0, max_steps = 0;
    for (int i = 0; i < count; ++i) {
      const sg_pass_item &it = items[i];
      if (it.steps < 0 || it.steps > tune->steps_per_pass) return SG_EINVAL;
      if (it.steps == 0) continue;
      if (it.r < kMinTileLog2 || it.r > SG_MAX_R || !it.src || !it.dst) return SG_EINVAL;
      if (misaligned(it.src) || misaligned(it.dst)) return SG_EINVAL;
      if (overlaps(it.src, it.dst, ((size_t)1 << it.r) * ((size_t)1 << it.r))) return SG_EALIAS;
      ++live;
      max_steps = std::max(max_steps, (int)it.steps);
    }
    if (live == 0) return SG_OK;
    if (sg::inject_hip_error()) return SG_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int slot = ctx->next;
    if (ctx->pending[slot] && hipEventSynchronize(ctx->staged[slot]) != hipSuccess) return SG_EHIP;
    sg::BatchItem *h_stage = ctx->h_stage + (size_t)slot * ctx->capacity;
    sg::BatchItem *d_items = ctx->d_items + (size_t)slot * ctx->capacity;
    uint64_t tiles = 0, touched = 0;
    int m = 0;
    for (int i = 0; i < count; ++i) {
      const sg_pass_item &it = items[i];
      if (it.steps == 0) continue;
      touched += sg::life_touched_bytes(it.r);
      sg::BatchItem b;
      b.src = it.src;
      b.dst = it.dst;
      b.r = it.r;
      b.steps = (int16_t)it.steps;
      b.k = (int16_t)item_k(it.r, kmax);
      b.tile_begin = tiles;
      tiles += pow3(it.r - b.k);
      h_stage[m++] = b;
    }
    st = hip_err(hipMemcpyAsync(d_items, h_stage, (size_t)m * sizeof(sg::BatchItem),
                                hipMemcpyHostToDevice, s));
    if (st != SG_OK) return st;
    st = hip_err(hipEventRecord(ctx->staged[slot], s));
    if (st != SG_OK) return st;
    ctx->pending[slot] = true;
    ctx->next = (slot + 1) % kPassRing;
    return hip_err(sg::launch_life_tb_batch(tune->rho, tune->threads, d_items, m, tiles,
                                            max_steps, groups_for(*tune, tiles),
                                            sg::life_stream_stores(touched), s));
  });
}

}  // extern "C"

// The item table of the allocation-free pass (sg_pass_run_static): one per
// GPU, in the code object's device memory, held until the process ends.
static __device__ __align__(256) sg::BatchItem scratch[SG_PASS_STATIC_MAX];

namespace {

// Items reach the table through kernel arguments, a chunk per launch: the
// runtime copies a launch's arguments when the launch is queued, so no host
// buffer has to outlive the call, and nothing is allocated.
constexpr int kStageChunk = 64;  // 64 items of 32 bytes: 2 KiB of arguments
struct StageChunk {
  sg::BatchItem items[kStageChunk];
};

__global__ __launch_bounds__(kStageChunk) void k_stage_items(StageChunk chunk, int count,
                                                             sg::BatchItem *table) {
  const int i = (int)threadIdx.x;
  if (i < count) table[i] = chunk.items[i];
}

// The device address of `scratch` on each device, looked up once per device
// (with that device current) by hipGetSymbolAddress.  Host code uses only
// these addresses: the array's own name is a host-side stand-in.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
sg::BatchItem *g_scratch[kMaxDevices] = {};

int scratch_table(sg::BatchItem **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SG_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return SG_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SG_EHIP;
    g_scratch[dev] = static_cast<sg::BatchItem *>(p);
  }
  *out = g_scratch[dev];
  return SG_OK;
}

}  // namespace

extern "C" {

SG_API int sg_pass_run_static(const sg_pass_item *items, int count, const sg_tune *tune,
                              void *stream) {
  if (count < 0 || count > SG_PASS_STATIC_MAX || (count > 0 && !items)) return SG_EINVAL;
  int st = check_tune(tune);
  if (st != SG_OK) return st;
  // validate everything before touching the device (as sg_pass_run)
  int live = 0, max_steps = 0;
  for (int i = 0; i < count; ++i) {
    const sg_pass_item &it = items[i];
    if (it.steps < 0 || it.steps > tune->steps_per_pass) return SG_EINVAL;
    if (it.steps == 0) continue;
    if (it.r < kMinTileLog2 || it.r > SG_MAX_R || !it.src || !it.dst) return SG_EINVAL;
    if (misaligned(it.src) || misaligned(it.dst)) return SG_EINVAL;
    if (overlaps(it.src, it.dst, ((size_t)1 << it.r) * ((size_t)1 << it.r))) return SG_EALIAS;
    ++live;
    max_steps = std::max(max_steps, (int)it.steps);
  }
  if (live == 0) return SG_OK;
  if (sg::inject_hip_error()) return SG_EHIP;
  sg::BatchItem *table = nullptr;
  st = scratch_table(&table);
  if (st != SG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int kmax = rho_log2(tune->rho);
  StageChunk chunk;
  uint64_t tiles = 0, touched = 0;
  int m = 0, c = 0;
  for (int i = 0; i < count; ++i) {
    const sg_pass_item &it = items[i];
    if (it.steps == 0) continue;
    touched += sg::life_touched_bytes(it.r);
    sg::BatchItem &b = chunk.items[c++];
    b.src = it.src;
    b.dst = it.dst;
    b.r = it.r;
    b.steps = (int16_t)it.steps;
    b.k = (int16_t)item_k(it.r, kmax);
    b.tile_begin = tiles;
    tiles += pow3(it.r - b.k);
    if (c == kStageChunk || m + c == live) {
      hipLaunchKernelGGL(k_stage_items, dim3(1), dim3(kStageChunk), 0, s, chunk, c, table + m);
      st = hip_err(hipGetLastError());
      if (st != SG_OK) return st;
      m += c;
      c = 0;
    }
  }
  return hip_err(sg::launch_life_tb_batch(tune->rho, tune->threads, table, m, tiles, max_steps,
                                          groups_for(*tune, tiles),
                                          sg::life_stream_stores(touched), s));
}

SG_API void sg_pass_ctx_destroy(sg_pass_ctx *ctx) {
  if (!ctx) return;
  for (int k = 0; k < kPassRing; ++k) {
    if (ctx->pending[k] && ctx->staged[k]) (void)hipEventSynchronize(ctx->staged[k]);
    if (ctx->staged[k]) (void)hipEventDestroy(ctx->staged[k]);
  }
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->d_items) (void)hipFree(ctx->d_items);
  delete ctx;
}

}  // extern "C"
