// Temporally blocked FP32 diffusion on the gasket (gfx950).
//
// One workgroup owns one rho x rho tile (rho in {32, 64}) of the map and
// advances it by T <= 8 explicit diffusion steps per pass:
//  1. load the tile plus a halo of T rows above/below and 8 cells left/right
//     (two float4 chunks) into an LDS plane, skipping chunks with no gasket
//     cell;
//  2. list, once, the 4-cell chunks that hold a gasket cell (wavefront ballot
//     + prefix count), each as one word: its region index, which of its
//     cells are on the gasket, and every cell's count of in-grid gasket
//     neighbours (the only per-cell data the update needs besides values);
//  3. T times: every listed chunk applies diffuse_cell, the same function
//     the one-step kernels use, to its 4 cells; planes ping-pong with a
//     barrier between steps.  The 4-neighbour stencil moves information one
//     cell per step, so cells outside the region are taken as 0 and the wrong
//     values this makes at the region's cut edges never reach the tile in
//     T <= 8 steps; chunks that cannot reach the tile in the steps left are
//     skipped;
//  4. store the tile, every 64-byte granule that holds a gasket cell in full.
//
// Plane rows have a pitch of the region width + 4 floats: the 4 floats before
// a row's first chunk are 0, so the west neighbour of the first chunk and the
// east neighbour of the last chunk (the next row's first float) read 0.
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kDtHalo = 8;  // halo columns each side: two float4 chunks

template <int RHO>
struct DtGeom {
  static constexpr int CW = RHO + 2 * kDtHalo;  // region columns (floats)
  static constexpr int CC = CW / 4;              // region chunks per row
  static constexpr int PW = CW + 4;              // plane pitch (one zero chunk per row)
  static constexpr int NT = RHO >= 64 ? 512 : 256;
};

template <int RHO>
size_t dt_lds_bytes(int T) {
  using G = DtGeom<RHO>;
  const int R = RHO + 2 * T;
  return sizeof(float) * (size_t)(2 * (R * G::PW + 4)) + sizeof(uint32_t) * (size_t)(R * G::CC);
}

// Chunk word: region chunk index (11 bits) | gasket cells (4 bits) << 11 |
// neighbour count of cell j (3 bits) << (15 + 3j).
constexpr int kChunkBits = 11;

template <int RHO, bool LAMBDA>
__global__ __launch_bounds__(DtGeom<RHO>::NT) void k_diffuse_tb(const float *__restrict__ in,
                                                                float *__restrict__ out, int r,
                                                                int rb, uint64_t tile_base,
                                                                uint64_t ntiles, int T,
                                                                float alpha) {
  using G = DtGeom<RHO>;
  constexpr int NT = G::NT;
  static_assert((RHO + 2 * 8) * G::CC < (1 << kChunkBits), "chunk index fits its field");
  extern __shared__ __align__(16) float flds[];
  __shared__ uint32_t nchunk;
  const uint64_t t = tile_base + logical_group();
  if (t >= ntiles) return;
  uint32_t bx, by;
  if constexpr (LAMBDA) {
    pass_decode((uint32_t)t, rb, bx, by);
  } else {
    by = (uint32_t)(t >> rb);
    bx = (uint32_t)(t & ((1ull << rb) - 1ull));
    if ((bx & by) != 0u) return;
  }
  const int tid = threadIdx.x;
  const int n = 1 << r;
  const int X0 = (int)bx * RHO, Y0 = (int)by * RHO;
  const int xr0 = X0 - kDtHalo, yr0 = Y0 - T;  // region origin
  const int R = RHO + 2 * T;
  // region cell (i, c) of a plane is at i * PW + 4 + c; 4 trailing zero
  // floats after the last row serve its last chunk's east neighbour
  float *plane0 = flds;
  float *plane1 = flds + R * G::PW + 4;
  uint32_t *chunks = reinterpret_cast<uint32_t *>(plane1 + R * G::PW + 4);  // R * CC

  for (int k = tid; k < 2 * (R * G::PW + 4); k += NT) flds[k] = 0.0f;
  if (tid == 0) nchunk = 0u;
  __syncthreads();

  // 1. load
  for (int e = tid; e < R * G::CC; e += NT) {
    const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
    const int y = yr0 + i, x = xr0 + 4 * c;
    if (y < 0 || y >= n || x < 0 || x >= n || (x & y) != 0) continue;
    const float4 v = *reinterpret_cast<const float4 *>(in + (size_t)y * n + x);
    *reinterpret_cast<float4 *>(plane0 + i * G::PW + 4 + 4 * c) = v;
  }

  // 2. the chunks that hold a gasket cell, with their cells' data
  const int lane = __lane_id();
  for (int base = 0; base < R * G::CC; base += NT) {
    const int e = base + tid;
    uint32_t word = 0u;
    bool live = false;
    if (e < R * G::CC) {
      const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
      const int y = yr0 + i, x = xr0 + 4 * c;
      live = y >= 0 && y < n && x >= 0 && x < n && (x & y) == 0;
      if (live) {
        word = (uint32_t)e;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int xj = x + j;
          const bool self = (xj & y) == 0;
          const int deg = (int)(xj > 0 && ((xj - 1) & y) == 0) +
                          (int)(xj + 1 < n && ((xj + 1) & y) == 0) +
                          (int)(y > 0 && (xj & (y - 1)) == 0) +
                          (int)(y + 1 < n && (xj & (y + 1)) == 0);
          word |= ((uint32_t)self << (kChunkBits + j)) | ((uint32_t)deg << (15 + 3 * j));
        }
      }
    }
    const uint64_t ball = __ballot(live);
    const uint32_t before = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    uint32_t off = 0u;
    if (lane == 0 && ball != 0ull) off = atomicAdd(&nchunk, (uint32_t)__popcll(ball));
    off = __shfl(off, 0);
    if (live) chunks[off + before] = word;
  }
  __syncthreads();
  const int nc = (int)nchunk;

  // 3. T steps
  for (int s = 0; s < T; ++s) {
    const float *src = (s & 1) ? plane1 : plane0;
    float *dst = (s & 1) ? plane0 : plane1;
    const int reach = T - s - 1;  // steps left after this one
    for (int k = tid; k < nc; k += NT) {
      const uint32_t word = chunks[k];
      const int e = (int)(word & ((1u << kChunkBits) - 1u));
      const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
      // skip chunks that cannot reach the tile in the steps left
      if (i < T - reach || i >= T + RHO + reach) continue;
      if (4 * c + 4 <= kDtHalo - reach || 4 * c >= kDtHalo + RHO + reach) continue;
      const float *p = src + i * G::PW + 4 + 4 * c;
      const float4 C = *reinterpret_cast<const float4 *>(p);
      const float4 N = *reinterpret_cast<const float4 *>(p - G::PW);
      const float4 S = *reinterpret_cast<const float4 *>(p + G::PW);
      const float Wn = p[-1], En = p[4];
      const float cu[4] = {C.x, C.y, C.z, C.w}, nu[4] = {N.x, N.y, N.z, N.w};
      const float su[4] = {S.x, S.y, S.z, S.w};
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float w = j == 0 ? Wn : cu[j - 1];
        const float ee = j == 3 ? En : cu[j + 1];
        const float deg = (float)((word >> (15 + 3 * j)) & 7u);
        const bool self = (word >> (kChunkBits + j)) & 1u;
        o[j] = diffuse_cell(cu[j], w, ee, nu[j], su[j], deg, self, alpha);
      }
      *reinterpret_cast<float4 *>(dst + i * G::PW + 4 + 4 * c) =
          make_float4(o[0], o[1], o[2], o[3]);
    }
    __syncthreads();
  }
  const float *fin = (T & 1) ? plane1 : plane0;

  // 4. store the tile, whole 64-byte granules (16 floats)
  constexpr int TC = RHO / 4;
  for (int e = tid; e < RHO * TC; e += NT) {
    const int ty = e / TC, c = e - (e / TC) * TC;
    const int y = Y0 + ty, x = X0 + 4 * c;
    if (((x & ~15) & y) != 0) continue;
    const float4 v =
        *reinterpret_cast<const float4 *>(fin + (T + ty) * G::PW + 4 + kDtHalo + 4 * c);
    *reinterpret_cast<float4 *>(out + (size_t)y * n + x) = v;
  }
}

template <int RHO>
hipError_t diffuse_tb_rho(const PassArgs &a, int T, const float *in, float *out, float alpha) {
  const size_t lds = dt_lds_bytes<RHO>(T);
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    if (a.lambda)
      hipLaunchKernelGGL((k_diffuse_tb<RHO, true>), dim3((unsigned)g), dim3(DtGeom<RHO>::NT),
                         lds, a.stream, in, out, a.r, a.rb, g0, a.ntiles, T, alpha);
    else
      hipLaunchKernelGGL((k_diffuse_tb<RHO, false>), dim3((unsigned)g), dim3(DtGeom<RHO>::NT),
                         lds, a.stream, in, out, a.r, a.rb, g0, a.ntiles, T, alpha);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

bool diffuse_tb_supported(int rho) { return rho == 32 || rho == 64; }

hipError_t launch_diffuse_tb(const PassArgs &a, int T, const float *in, float *out,
                             float alpha) {
  if (T < 1 || T > kMaxDiffuseStepsPerPass) return hipErrorInvalidValue;
  switch (a.rho) {
    case 32: return diffuse_tb_rho<32>(a, T, in, out, alpha);
    case 64: return diffuse_tb_rho<64>(a, T, in, out, alpha);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
