// Block-compacted storage of a gasket and the inverse block map.
//
// A gasket of level r in tiles of side rho = 2^k has 3^(r-k) fractal tiles
// (Lemma 1 in block space); storing only those, tile omega (lambda order) at
// byte omega * rho^2 with rho-byte rows, takes (4/3)^k * 3^r bytes instead of
// the n^2 of the embedding, and every tile row is one contiguous segment.
// The inverse map omega(bx, by) (lambda_encode) finds a tile's neighbours.
#include "../../include/sg.h"
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kWG) void k_map_lambda_inverse(int32_t *__restrict__ out, int rb,
                                                            uint64_t base, uint64_t count) {
  const uint64_t t = base + (uint64_t)blockIdx.x * kWG + threadIdx.x;
  if (t >= count) return;
  const uint32_t by = (uint32_t)(t >> rb);
  const uint32_t bx = (uint32_t)(t & ((1ull << rb) - 1ull));
  out[t] = (bx & by) == 0u ? (int32_t)lambda_encode(bx, by, rb) : -1;
}

// One workgroup per fractal tile: copy its rho rows between the embedding and
// the compact store (PACK: embedding -> compact).
template <int RHO, bool PACK>
__global__ __launch_bounds__(kCopyThreads) void k_compact_copy(const uint8_t *__restrict__ src,
                                                               uint8_t *__restrict__ dst, int r,
                                                               int rb, uint64_t tile_base,
                                                               uint64_t ntiles) {
  const uint64_t t = tile_base + blockIdx.x;
  if (t >= ntiles) return;
  uint32_t bx, by;
  lambda_decode((uint32_t)t, rb, bx, by);
  const size_t n = (size_t)1 << r;
  const size_t X0 = (size_t)bx * RHO, Y0 = (size_t)by * RHO;
  const size_t tile = (size_t)t * RHO * RHO;
  constexpr int CPR = RHO / 16;
  for (int e = threadIdx.x; e < RHO * CPR; e += kCopyThreads) {
    const int ty = e / CPR, c = e - (e / CPR) * CPR;
    const size_t dense = (Y0 + ty) * n + X0 + 16 * c, packed = tile + (size_t)ty * RHO + 16 * c;
    if (PACK)
      *reinterpret_cast<uint4 *>(dst + packed) = *reinterpret_cast<const uint4 *>(src + dense);
    else
      *reinterpret_cast<uint4 *>(dst + dense) = *reinterpret_cast<const uint4 *>(src + packed);
  }
}

// Output c (counting from 0) of the SplitMix64 generator seeded with `seed`
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): the state after c + 1 additions of the golden-ratio gamma,
// passed through the generator's 64-bit finaliser.  Counter-based, so any
// cell's value is computed on its own.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// One workgroup per fractal tile: gasket cell (x, y) of the tile is 1 iff
// splitmix64_at(seed, y * 2^32 + x) < threshold, every other byte 0; written
// in 16-byte chunks of the compact store.
template <int RHO>
__global__ __launch_bounds__(kCopyThreads) void k_compact_init(uint8_t *__restrict__ dst, int rb,
                                                               uint64_t tile_base, uint64_t ntiles,
                                                               uint64_t seed, uint64_t threshold) {
  const uint64_t t = tile_base + blockIdx.x;
  if (t >= ntiles) return;
  uint32_t bx, by;
  lambda_decode((uint32_t)t, rb, bx, by);
  const uint32_t X0 = bx * RHO, Y0 = by * RHO;
  const size_t tile = (size_t)t * RHO * RHO;
  constexpr int CPR = RHO / 16;
  for (int e = threadIdx.x; e < RHO * CPR; e += kCopyThreads) {
    const int ty = e / CPR, c = e - (e / CPR) * CPR;
    const uint32_t y = Y0 + (uint32_t)ty, x0 = X0 + 16u * (uint32_t)c;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if ((x0 & y) == 0u) {  // the chunk holds a gasket cell (x0 is a multiple of 16)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t x = x0 + (uint32_t)j;
        if ((x & y) != 0u) continue;
        const uint64_t v = splitmix64_at(seed, ((uint64_t)y << 32) | x);
        w[j >> 2] |= (v < threshold ? 1u : 0u) << (8 * (j & 3));
      }
    }
    *reinterpret_cast<uint4 *>(dst + tile + (size_t)ty * RHO + 16 * c) =
        make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int RHO>
hipError_t compact_init_rho(const PassArgs &a, uint64_t seed, uint64_t threshold, uint8_t *dst) {
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    hipLaunchKernelGGL((k_compact_init<RHO>), dim3((unsigned)g), dim3(kCopyThreads), 0, a.stream,
                       dst, a.rb, g0, a.ntiles, seed, threshold);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO, bool PACK>
hipError_t compact_copy_rho(const PassArgs &a, const uint8_t *src, uint8_t *dst) {
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    hipLaunchKernelGGL((k_compact_copy<RHO, PACK>), dim3((unsigned)g), dim3(kCopyThreads), 0,
                       a.stream, src, dst, a.r, a.rb, g0, a.ntiles);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_map_lambda_inverse(int rb, int32_t *d_out, hipStream_t s) {
  const uint64_t count = 1ull << (2 * rb);
  const uint64_t per_launch = (uint64_t)kWG << 22;
  for (uint64_t b0 = 0; b0 < count; b0 += per_launch) {
    const uint64_t c = count - b0 < per_launch ? count - b0 : per_launch;
    hipLaunchKernelGGL(k_map_lambda_inverse, dim3((unsigned)((c + kWG - 1) / kWG)), dim3(kWG), 0,
                       s, d_out, rb, b0, count);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_compact_copy(const PassArgs &a, bool pack, const uint8_t *src, uint8_t *dst) {
  switch (a.rho) {
    case 64: return pack ? compact_copy_rho<64, true>(a, src, dst) : compact_copy_rho<64, false>(a, src, dst);
    case 128: return pack ? compact_copy_rho<128, true>(a, src, dst) : compact_copy_rho<128, false>(a, src, dst);
    case 256: return pack ? compact_copy_rho<256, true>(a, src, dst) : compact_copy_rho<256, false>(a, src, dst);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_compact_init(const PassArgs &a, uint64_t seed, uint64_t threshold,
                               uint8_t *dst) {
  switch (a.rho) {
    case 64: return compact_init_rho<64>(a, seed, threshold, dst);
    case 128: return compact_init_rho<128>(a, seed, threshold, dst);
    case 256: return compact_init_rho<256>(a, seed, threshold, dst);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
