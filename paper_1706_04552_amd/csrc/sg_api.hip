// C entry points of libsg: argument validation (host only, before any HIP
// call), map/tile bookkeeping, and dispatch to the kernel launchers.
#include <stdlib.h>
#include <string.h>

#include "../../include/sg.h"
#include "sg_launch.h"

namespace {

thread_local char g_last_hip_error[256] = "";

int hip_status(hipError_t e) {
  if (e == hipSuccess) return SG_OK;
  const char *s = hipGetErrorString(e);
  strncpy(g_last_hip_error, s ? s : "unknown HIP error", sizeof(g_last_hip_error) - 1);
  g_last_hip_error[sizeof(g_last_hip_error) - 1] = '\0';
  return SG_EHIP;
}

uint64_t pow3(int e) {
  uint64_t v = 1;
  for (int i = 0; i < e; ++i) v *= 3;
  return v;
}

// log2 of a power-of-two rho in [1, SG_MAX_RHO], or -1.
int rho_log2(int rho) {
  if (rho < 1 || rho > SG_MAX_RHO || (rho & (rho - 1)) != 0) return -1;
  int k = 0;
  while ((1 << k) < rho) ++k;
  return k;
}

// Validates (r, rho) and returns r_b = r - log2(rho), or -1.
int block_level(int r, int rho) {
  if (r < 0 || r > SG_MAX_R) return -1;
  const int k = rho_log2(rho);
  if (k < 0 || k > r) return -1;
  return r - k;
}

// State arrays are read and written with 16-byte vector accesses.
bool misaligned(const void *p) { return ((uintptr_t)p & 15u) != 0; }

bool overlaps(const void *a, const void *b, size_t bytes) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + bytes && pb < pa + bytes;
}

// Steps of pass k (1-based) when `steps` are split over `passes` passes as
// evenly as possible: every pass runs floor or ceil of steps / passes, the
// longer ones last.  A pass costs a fixed part (load, list, store) plus a
// part per step that grows with its halo, so an even split does the least
// halo work for a given number of passes.
int pass_steps(int steps, int passes, int k) {
  const int q = steps / passes, rem = steps % passes;
  return q + (k > passes - rem ? 1 : 0);
}

int pass_args(int map, int r, int rho, void *stream, sg::PassArgs &a) {
  const int rb = block_level(r, rho);
  if (rb < 0 || (map != SG_MAP_LAMBDA && map != SG_MAP_BBOX)) return SG_EINVAL;
  a.r = r;
  a.rho = rho;
  a.rb = rb;
  a.lambda = map == SG_MAP_LAMBDA;
  a.ntiles = a.lambda ? pow3(rb) : (1ull << (2 * rb));
  a.stream = (hipStream_t)stream;
  return SG_OK;
}

}  // namespace

namespace sg {
int status_of(hipError_t e) { return hip_status(e); }
bool inject_hip_error() {
  static const bool on = getenv("SG_INJECT_HIP_ERROR") != nullptr;
  return on;
}
}  // namespace sg

#define SG_INJECT()                      \
  do {                                   \
    if (sg::inject_hip_error())          \
      return hip_status(hipErrorLaunchFailure); \
  } while (0)

extern "C" {

SG_API const char *sg_strerror(int code) {
  switch (code) {
    case SG_OK: return "success";
    case SG_EINVAL: return "invalid argument (r, rho, map kind, size or null pointer)";
    case SG_EALIAS: return "input and output arrays overlap";
    case SG_EHIP: return "HIP runtime error";
    case SG_ENOMEM: return "out of memory";
    default: return "unknown status";
  }
}

SG_API const char *sg_last_hip_error(void) { return g_last_hip_error; }

SG_API int sg_version(void) { return 1; }

SG_API int sg_lambda_grid(int r, int rho, uint64_t *W, uint64_t *H) {
  const int rb = block_level(r, rho);
  if (rb < 0 || !W || !H) return SG_EINVAL;
  *W = pow3(rb / 2);
  *H = pow3(rb - rb / 2);
  return SG_OK;
}

SG_API int sg_block_count(int map, int r, int rho, uint64_t *blocks) {
  sg::PassArgs a;
  if (!blocks) return SG_EINVAL;
  const int st = pass_args(map, r, rho, nullptr, a);
  if (st != SG_OK) return st;
  *blocks = a.ntiles;
  return SG_OK;
}

SG_API int sg_map_lambda(int r, int rho, uint32_t *d_bxy, void *stream) {
  const int rb = block_level(r, rho);
  if (rb < 0 || !d_bxy || ((uintptr_t)d_bxy & 7u)) return SG_EINVAL;
  SG_INJECT();
  return hip_status(sg::launch_map_lambda(rb, (uint32_t)pow3(rb), d_bxy, (hipStream_t)stream));
}

SG_API int sg_map_bbox(int r, int rho, uint8_t *d_mask, void *stream) {
  const int rb = block_level(r, rho);
  if (rb < 0 || !d_mask) return SG_EINVAL;
  SG_INJECT();
  return hip_status(sg::launch_map_bbox(rb, 1ull << (2 * rb), d_mask, (hipStream_t)stream));
}

SG_API int sg_write_pass(int map, int r, int rho, uint8_t *d_a, uint8_t value, void *stream) {
  sg::PassArgs a;
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!d_a || misaligned(d_a)) return SG_EINVAL;
  SG_INJECT();
  return hip_status(sg::launch_write(a, d_a, value));
}

SG_API int sg_write_pass_intra(int map, int intra, int r, int rho, uint8_t *d_a, uint8_t value,
                               void *stream) {
  sg::PassArgs a;
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (intra != SG_INTRA_SUBBOX && intra != SG_INTRA_UNROLL && intra != SG_INTRA_LUT) return SG_EINVAL;
  if (!d_a || misaligned(d_a)) return SG_EINVAL;
  if (intra != SG_INTRA_SUBBOX && rho > 32) return SG_EINVAL;
  SG_INJECT();
  if (intra == SG_INTRA_SUBBOX) return hip_status(sg::launch_write(a, d_a, value));
  return hip_status(sg::launch_write_intra(a, d_a, value, intra == SG_INTRA_LUT));
}

SG_API int sg_ca_step(int map, int r, int rho, const uint8_t *d_in, uint8_t *d_out,
                      void *stream) {
  sg::PassArgs a;
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!d_in || !d_out || misaligned(d_in) || misaligned(d_out)) return SG_EINVAL;
  const size_t bytes = ((size_t)1 << r) * ((size_t)1 << r);
  if (overlaps(d_in, d_out, bytes)) return SG_EALIAS;
  SG_INJECT();
  return hip_status(sg::launch_life(a, d_in, d_out));
}

}  // extern "C"

namespace {
// The checks of sg_ca_steps, before any HIP call; fills `a` and resolves
// steps_per_pass = 0 to the library's choice.
int ca_steps_args(int map, int r, int rho, int steps, int &steps_per_pass, const uint8_t *d_in,
                  const uint8_t *d_out, const uint8_t *d_work, void *stream, sg::PassArgs &a) {
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (steps < 0 || steps_per_pass < 0 || steps_per_pass > sg::kMaxStepsPerPass) return SG_EINVAL;
  const bool tb_ok = sg::life_tb_dense_supported(rho);
  const bool tbs_ok = sg::life_tbs_supported(rho);  // side 16: up to 16 per pass
  if (steps_per_pass == 0)
    steps_per_pass = tb_ok ? sg::kDefaultStepsPerPass : (tbs_ok ? sg::kMaxSmallTileSteps : 1);
  if (steps_per_pass > 1 && !tb_ok && !(tbs_ok && steps_per_pass <= sg::kMaxSmallTileSteps))
    return SG_EINVAL;
  if (!d_in || !d_out || misaligned(d_in) || misaligned(d_out)) return SG_EINVAL;
  const size_t bytes = ((size_t)1 << r) * ((size_t)1 << r);
  if (overlaps(d_in, d_out, bytes)) return SG_EALIAS;
  const int passes = (steps + steps_per_pass - 1) / steps_per_pass;
  if (passes >= 2) {
    if (!d_work || misaligned(d_work)) return SG_EINVAL;
    if (overlaps(d_work, d_in, bytes) || overlaps(d_work, d_out, bytes)) return SG_EALIAS;
  }
  return SG_OK;
}
}  // namespace

extern "C" {

SG_API int sg_ca_steps(int map, int r, int rho, int steps, int steps_per_pass,
                       const uint8_t *d_in, uint8_t *d_out, uint8_t *d_work, void *stream) {
  sg::PassArgs a;
  const int st = ca_steps_args(map, r, rho, steps, steps_per_pass, d_in, d_out, d_work, stream, a);
  if (st != SG_OK) return st;
  const bool tb_ok = sg::life_tb_dense_supported(rho);
  const size_t bytes = ((size_t)1 << r) * ((size_t)1 << r);
  const int passes = (steps + steps_per_pass - 1) / steps_per_pass;
  SG_INJECT();
  if (steps == 0)
    return hip_status(hipMemcpyAsync(d_out, d_in, bytes, hipMemcpyDeviceToDevice, a.stream));
  if (tb_ok && steps_per_pass > 1 && passes >= 2) {
    // between passes the state is bit-packed tiles, two of them in d_work
    // (each at most n^2 / 8 bytes): bytes in, bits, ..., bits, bytes out
    const size_t half = (sg::life_tb_bit_state_bytes(a) + 255) & ~(size_t)255;
    void *bits[2] = {d_work, d_work + half};
    for (int k = 1; k <= passes; ++k) {
      const int T = pass_steps(steps, passes, k);
      const bool first = k == 1, last = k == passes;
      const void *src = first ? static_cast<const void *>(d_in) : bits[k % 2];
      void *dst = last ? static_cast<void *>(d_out) : bits[(k + 1) % 2];
      const hipError_t e = sg::launch_life_tb_bits(a, T, src, !first, dst, !last);
      if (e != hipSuccess) return hip_status(e);
    }
    return SG_OK;
  }
  // the last pass must land in d_out: alternate d_out / d_work backwards
  const uint8_t *src = d_in;
  for (int k = 1; k <= passes; ++k) {
    uint8_t *dst = ((passes - k) % 2 == 0) ? d_out : d_work;
    const int T = pass_steps(steps, passes, k);
    const hipError_t e = T == 1 && steps_per_pass == 1 ? sg::launch_life(a, src, dst)
                         : tb_ok                          ? sg::launch_life_tb(a, T, src, dst)
                                                          : sg::launch_life_tbs(a, T, src, dst);
    if (e != hipSuccess) return hip_status(e);
    src = dst;
  }
  return SG_OK;
}

SG_API int sg_ca_steps_autotune(int map, int r, int steps, const uint8_t *d_in, uint8_t *d_out,
                                uint8_t *d_work, int *best_rho, int *best_steps_per_pass,
                                float *best_ms, void *stream) {
  if (!best_rho || !best_steps_per_pass || !best_ms || steps < 1 || !d_work) return SG_EINVAL;
  // every candidate is checked before any is timed
  const int rhos[] = {32, 64, 128, 256}, spps[] = {8, 16, 32};
  int candidates = 0;
  for (int rho : rhos) {
    if (r < 0 || r > SG_MAX_R || rho > (1 << r)) continue;
    for (int T : spps) {
      sg::PassArgs a;
      int spp = T;
      const int st = ca_steps_args(map, r, rho, steps, spp, d_in, d_out, d_work, stream, a);
      if (st != SG_OK) return st;
      ++candidates;
    }
  }
  if (candidates == 0) return SG_EINVAL;
  SG_INJECT();
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SG_EHIP;
  }
  int status = SG_OK;
  float best = -1.0f;
  for (int rho : rhos) {
    if (rho > (1 << r)) continue;
    for (int T : spps) {
      int st = sg_ca_steps(map, r, rho, steps, T, d_in, d_out, d_work, stream);  // warm-up
      if (st == SG_OK && hipEventRecord(e0, s) != hipSuccess) st = SG_EHIP;
      if (st == SG_OK) st = sg_ca_steps(map, r, rho, steps, T, d_in, d_out, d_work, stream);
      if (st == SG_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        st = SG_EHIP;
      float ms = 0.0f;
      if (st == SG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = SG_EHIP;
      if (st != SG_OK) {
        status = st;
        break;
      }
      if (best < 0.0f || ms < best) {
        best = ms;
        *best_rho = rho;
        *best_steps_per_pass = T;
      }
    }
    if (status != SG_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == SG_OK) *best_ms = best;
  return status;
}

SG_API int sg_diffuse_steps(int map, int r, int rho, int steps, int steps_per_pass,
                            const float *d_in, float *d_out, float *d_work, float alpha,
                            void *stream) {
  sg::PassArgs a;
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (steps < 0 || steps_per_pass < 0 || steps_per_pass > sg::kMaxDiffuseStepsPerPass)
    return SG_EINVAL;
  const bool tb_ok = sg::diffuse_tb_supported(rho);
  if (steps_per_pass == 0) steps_per_pass = tb_ok ? sg::diffuse_tb_default_steps(rho) : 1;
  if (steps_per_pass > 1 && !tb_ok) return SG_EINVAL;
  if (!d_in || !d_out || misaligned(d_in) || misaligned(d_out)) return SG_EINVAL;
  const size_t bytes = ((size_t)1 << r) * ((size_t)1 << r) * sizeof(float);
  if (overlaps(d_in, d_out, bytes)) return SG_EALIAS;
  const int passes = (steps + steps_per_pass - 1) / steps_per_pass;
  if (passes >= 2) {
    if (!d_work || misaligned(d_work)) return SG_EINVAL;
    if (overlaps(d_work, d_in, bytes) || overlaps(d_work, d_out, bytes)) return SG_EALIAS;
  }
  SG_INJECT();
  if (steps == 0)
    return hip_status(hipMemcpyAsync(d_out, d_in, bytes, hipMemcpyDeviceToDevice, a.stream));
  const float *src = d_in;
  for (int k = 1; k <= passes; ++k) {
    float *dst = ((passes - k) % 2 == 0) ? d_out : d_work;
    const int T = pass_steps(steps, passes, k);
    const hipError_t e = steps_per_pass == 1 ? sg::launch_diffuse(a, src, dst, alpha)
                                             : sg::launch_diffuse_tb(a, T, src, dst, alpha);
    if (e != hipSuccess) return hip_status(e);
    src = dst;
  }
  return SG_OK;
}

SG_API int sg_map_lambda_inverse(int r, int rho, int32_t *d_omega, void *stream) {
  const int rb = block_level(r, rho);
  if (rb < 0 || !d_omega || ((uintptr_t)d_omega & 3u)) return SG_EINVAL;
  if (pow3(rb) > 0x7fffffffull) return SG_EINVAL;  // omega must fit an int32
  SG_INJECT();
  return hip_status(sg::launch_map_lambda_inverse(rb, d_omega, (hipStream_t)stream));
}

SG_API int sg_compact_bytes(int r, int rho, uint64_t *bytes) {
  const int rb = block_level(r, rho);
  if (rb < 0 || !bytes || !sg::life_tb_supported(rho)) return SG_EINVAL;
  *bytes = pow3(rb) * (uint64_t)rho * (uint64_t)rho;
  return SG_OK;
}

namespace {
int compact_copy(int r, int rho, const uint8_t *src, uint8_t *dst, bool pack, void *stream) {
  sg::PassArgs a;
  const int st = pass_args(SG_MAP_LAMBDA, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!sg::life_tb_supported(rho) || !src || !dst || misaligned(src) || misaligned(dst))
    return SG_EINVAL;
  const size_t dense = ((size_t)1 << r) * ((size_t)1 << r);
  const size_t packed = (size_t)pow3(a.rb) * (size_t)rho * (size_t)rho;
  const uint8_t *lo = src < dst ? src : dst;
  const uint8_t *hi = src < dst ? dst : src;
  const size_t lo_bytes = (lo == (pack ? src : dst)) ? dense : packed;
  if ((uintptr_t)lo + lo_bytes > (uintptr_t)hi) return SG_EALIAS;
  SG_INJECT();
  return hip_status(sg::launch_compact_copy(a, pack, src, dst));
}
}  // namespace

SG_API int sg_compact_init_bernoulli(int r, int rho, uint64_t seed, uint64_t threshold,
                                     uint8_t *d_compact, void *stream) {
  sg::PassArgs a;
  const int st = pass_args(SG_MAP_LAMBDA, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!sg::life_tb_supported(rho) || !d_compact || misaligned(d_compact)) return SG_EINVAL;
  SG_INJECT();
  return hip_status(sg::launch_compact_init(a, seed, threshold, d_compact));
}

SG_API int sg_compact_pack(int r, int rho, const uint8_t *d_dense, uint8_t *d_compact,
                           void *stream) {
  return compact_copy(r, rho, d_dense, d_compact, true, stream);
}

SG_API int sg_compact_unpack(int r, int rho, const uint8_t *d_compact, uint8_t *d_dense,
                             void *stream) {
  return compact_copy(r, rho, d_compact, d_dense, false, stream);
}

SG_API int sg_ca_steps_compact(int r, int rho, int steps, int steps_per_pass,
                               const uint8_t *d_in, uint8_t *d_out, uint8_t *d_work,
                               void *stream) {
  sg::PassArgs a;
  const int st = pass_args(SG_MAP_LAMBDA, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!sg::life_tb_supported(rho) || steps < 0 || steps_per_pass < 0 ||
      steps_per_pass > sg::kMaxStepsPerPass)
    return SG_EINVAL;
  if (steps_per_pass == 0) steps_per_pass = sg::kDefaultStepsPerPass;
  if (!d_in || !d_out || misaligned(d_in) || misaligned(d_out)) return SG_EINVAL;
  const size_t bytes = (size_t)pow3(a.rb) * (size_t)rho * (size_t)rho;
  if (overlaps(d_in, d_out, bytes)) return SG_EALIAS;
  const int passes = (steps + steps_per_pass - 1) / steps_per_pass;
  if (passes >= 2) {
    if (!d_work || misaligned(d_work)) return SG_EINVAL;
    if (overlaps(d_work, d_in, bytes) || overlaps(d_work, d_out, bytes)) return SG_EALIAS;
  }
  SG_INJECT();
  if (steps == 0)
    return hip_status(hipMemcpyAsync(d_out, d_in, bytes, hipMemcpyDeviceToDevice, a.stream));
  if (passes == 1) return hip_status(sg::launch_life_tb_compact(a, steps, d_in, d_out));
  // between passes the state is bit-packed tiles, two of them in d_work
  // (each an eighth of a compact state): bytes in, bits, ..., bits, bytes out
  const size_t half = (sg::life_tb_bit_state_bytes(a) + 255) & ~(size_t)255;
  void *bits[2] = {d_work, d_work + half};
  for (int k = 1; k <= passes; ++k) {
    const int T = pass_steps(steps, passes, k);
    const bool first = k == 1, last = k == passes;
    const void *src = first ? static_cast<const void *>(d_in) : bits[k % 2];
    void *dst = last ? static_cast<void *>(d_out) : bits[(k + 1) % 2];
    const hipError_t e = sg::launch_life_tb_compact_bits(a, T, src, !first, dst, !last);
    if (e != hipSuccess) return hip_status(e);
  }
  return SG_OK;
}

SG_API int sg_diffuse_step(int map, int r, int rho, const float *d_in, float *d_out,
                           float alpha, void *stream) {
  sg::PassArgs a;
  const int st = pass_args(map, r, rho, stream, a);
  if (st != SG_OK) return st;
  if (!d_in || !d_out || misaligned(d_in) || misaligned(d_out)) return SG_EINVAL;
  const size_t bytes = ((size_t)1 << r) * ((size_t)1 << r) * sizeof(float);
  if (overlaps(d_in, d_out, bytes)) return SG_EALIAS;
  SG_INJECT();
  return hip_status(sg::launch_diffuse(a, d_in, d_out, alpha));
}

}  // extern "C"
