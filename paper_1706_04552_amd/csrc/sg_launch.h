// Host-side launchers of the gasket kernels (internal to libsg).  Arguments
// reach these functions already validated by the C entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

// Test hook: when the environment variable SG_INJECT_HIP_ERROR is set at
// library load, every entry point that would launch work reports a launch
// failure (SG_EHIP) instead, after validating its arguments.
bool inject_hip_error();

// SG_OK, or SG_EHIP with the HIP error's text kept for sg_last_hip_error.
int status_of(hipError_t e);

// Output stores of a life pass go non-temporal when the bytes it moves
// exceed the 256 MB Infinity Cache: then its output would only evict the
// input lines that neighbouring tiles still read, while a working set that
// fits (r <= 15) is served from the cache and ordinary stores are faster.
// A uint8 state touches about (4/3)^6 * 3^r bytes in 64-byte granules.
constexpr uint64_t kCacheBytes = 256ull << 20;
inline uint64_t life_touched_bytes(int r) {
  uint64_t v = 1;
  for (int i = 0; i < r; ++i) v *= 3;
  return 2 * v * 4096 / 729;  // input and output state
}
inline bool life_stream_stores(uint64_t touched_bytes) { return touched_bytes > kCacheBytes; }

// One pass over the tiles of a map.
struct PassArgs {
  int r;            // level: n = 2^r
  int rho;          // tile side, a power of two in [1, 32]
  int rb;           // block level r - log2(rho)
  bool lambda;      // lambda map (3^rb tiles) or bounding box (4^rb tiles)
  uint64_t ntiles;  // number of tiles the map launches
  hipStream_t stream;
};

hipError_t launch_map_lambda(int rb, uint32_t count, uint32_t *d_bxy, hipStream_t s);
hipError_t launch_map_bbox(int rb, uint64_t count, uint8_t *d_mask, hipStream_t s);
hipError_t launch_write(const PassArgs &a, uint8_t *d, uint8_t value);
// Write pass with thread-level lambda ("further unrolling", lut = false) or a
// shared table of in-tile offsets (lut = true); rho <= 32.
hipError_t launch_write_intra(const PassArgs &a, uint8_t *d, uint8_t value, bool lut);
hipError_t launch_life(const PassArgs &a, const uint8_t *in, uint8_t *out);
hipError_t launch_diffuse(const PassArgs &a, const float *in, float *out, float alpha);

// Temporally blocked life: T generations per pass, T in [1, kMaxStepsPerPass],
// for tile sides rho in {64, 128, 256}.
constexpr int kMaxStepsPerPass = 32;
constexpr int kDefaultStepsPerPass = 32;  // what steps_per_pass = 0 selects
// Tile sides of the compact, batched and served paths (64, 128, 256), and of
// the dense pass (those and 32).
bool life_tb_supported(int rho);
bool life_tb_dense_supported(int rho);
hipError_t launch_life_tb(const PassArgs &a, int T, const uint8_t *in, uint8_t *out);
// The dense pass with bit-packed tiles (one bit per cell, 3^rb tiles in
// lambda order, rho^2 / 32 words each, 16-byte aligned) as its input
// (in_bits) and/or its output (out_bits), the byte embedding on the other
// side: the state between the passes of a multi-pass run.  Bytes of one
// such state (0 for an unsupported rho):
size_t life_tb_bit_state_bytes(const PassArgs &a);
hipError_t launch_life_tb_bits(const PassArgs &a, int T, const void *in, bool in_bits, void *out,
                               bool out_bits);
// The same for tiles of side 16 (byte planes, one 16-cell chunk of halo):
// T in [1, kMaxSmallTileSteps].
constexpr int kMaxSmallTileSteps = 16;
bool life_tbs_supported(int rho);
hipError_t launch_life_tbs(const PassArgs &a, int T, const uint8_t *in, uint8_t *out);

// Block-compacted storage (tiles of side rho in {64, 128, 256}, lambda order).
hipError_t launch_map_lambda_inverse(int rb, int32_t *d_out, hipStream_t s);
hipError_t launch_compact_copy(const PassArgs &a, bool pack, const uint8_t *src, uint8_t *dst);
hipError_t launch_compact_init(const PassArgs &a, uint64_t seed, uint64_t threshold,
                               uint8_t *dst);
hipError_t launch_life_tb_compact(const PassArgs &a, int T, const uint8_t *in, uint8_t *out);
// The compact pass with bit-packed tiles (as launch_life_tb_bits) as its
// input and/or output, compact byte tiles on the other side.
hipError_t launch_life_tb_compact_bits(const PassArgs &a, int T, const void *in, bool in_bits,
                                       void *out, bool out_bits);

// Temporally blocked FP32 diffusion: T steps per pass, T in
// [1, kMaxDiffuseStepsPerPass], for tile sides rho in {16, 32, 64}.
constexpr int kMaxDiffuseStepsPerPass = 16;
bool diffuse_tb_supported(int rho);
// What steps_per_pass = 0 selects: the measured best pass length at this
// tile side (16 at rho = 16 and 64; 8 at 32, where a longer pass's wider
// region costs more than its fewer passes save).
int diffuse_tb_default_steps(int rho);
hipError_t launch_diffuse_tb(const PassArgs &a, int T, const float *in, float *out,
                             float alpha);

// One pass over many gaskets (device table of items, sorted by tile_begin,
// every item with at least one tile and 1 <= steps <= max_steps).
struct BatchItem {
  const uint8_t *src;   // state before the pass
  uint8_t *dst;         // state after the pass
  uint64_t tile_begin;  // global index of the item's first lambda tile
  int32_t r;            // level: n = 2^r (r >= k)
  int16_t steps;        // generations in this pass
  int16_t k;            // this item's tile side is 2^k: 6, 7 or 8 (64, 128, 256)
};
// Tiles of every side up to max_rho may appear in one launch.  stream_out:
// non-temporal output stores (life_stream_stores of the items' bytes).
hipError_t launch_life_tb_batch(int max_rho, int threads, const BatchItem *d_items, int count,
                                uint64_t total_tiles, int max_steps, int groups,
                                bool stream_out, hipStream_t stream);

}  // namespace sg
