// Temporally blocked FP32 diffusion on the gasket (gfx950).
//
// One workgroup owns one rho x rho tile (rho in {16, 32, 64}) of the map and
// advances it by T <= 8 explicit diffusion steps per pass:
//  1. load the tile plus a halo of T rows above/below and 8 cells left/right
//     (two float4 chunks) into registers, every load issued before the first
//     wait, skipping chunks with no gasket cell; while the loads are in
//     flight, list the 4-cell chunks that hold a gasket cell and can reach
//     the tile in T steps (wavefront ballot + prefix count), each as one
//     word: its region index and its distance to the tile.  The list is
//     built in the second plane's memory, which is not in use yet; then
//     write the first plane;
//  2. each thread takes its listed chunks into registers: the chunk's LDS
//     offset, the number of steps in which it can still reach the tile, and
//     per cell its count deg of in-grid gasket neighbours and a weight
//     (alpha on the gasket, 0 off it);
//  3. clear the second plane, then T times: every
//     held chunk updates its 4 cells with the arithmetic of diffuse_cell, the
//     function the one-step kernels use, as
//     fma(w, fma(-deg, u, (W + E) + (N + S)), u); off the gasket w = 0 keeps
//     the value, which is 0 (the inner fma is finite there).  A chunk's own values stay in registers; the
//     neighbours come from the other plane, and the planes ping-pong with a
//     barrier between steps;
//  4. store the tile, every 64-byte granule that holds a gasket cell in full.
//
// The 4-neighbour stencil moves information one cell per step.  Cells outside
// the region hold wrong values (the plane has no cells there: a row's west
// neighbour of its first chunk is the previous row's last cell, and so on),
// and a chunk stops updating once it can no longer reach the tile in the
// steps left, which leaves stale values behind it.  Every such cell is more
// steps away from the tile than remain, so the tile's values are exactly
// those of T one-step passes.  Rows 0 and R - 1 of the region are T cells from
// the tile, so no updated chunk reads outside the plane.
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kDtHalo = 8;  // halo columns each side: two float4 chunks

template <int RHO>
struct DtGeom {
  static constexpr int CW = RHO + 2 * kDtHalo;  // region columns = plane pitch (floats)
  static constexpr int CC = CW / 4;              // region chunks per row
  static constexpr int NT = RHO >= 64 ? 512 : 256;
  // chunks of the largest region, and how many one thread may hold
  static constexpr int SLOTS = (RHO + 2 * kMaxDiffuseStepsPerPass) * CC;
  static constexpr int KMAX = (SLOTS + NT - 1) / NT;
};

template <int RHO>
size_t dt_lds_bytes(int T) {
  using G = DtGeom<RHO>;
  return sizeof(float) * 2 * (size_t)(RHO + 2 * T) * G::CW;
}

// List word: region chunk index (11 bits) | distance to the tile (< T) << 27.
constexpr int kChunkBits = 11;
constexpr int kDistShift = 27;

// Gasket cells of a 4-cell chunk whose first cell (column x, a multiple of 4)
// is on the gasket in row y, one byte per cell (byte j = 1 iff cell x + j is
// on the gasket): x + j and y share no bit iff x & y == 0 and j & (y mod 4)
// == 0.  `ymod4` is y mod 4.
__device__ __forceinline__ uint32_t chunk_row_bytes(uint32_t ymod4) {
  const uint32_t nib = (0x135Fu >> (4u * ymod4)) & 0xFu;  // bit j: j & ymod4 == 0
  return (nib * 0x00204081u) & 0x01010101u;              // bit j -> byte j
}

// Distance (in steps of the 4-neighbour stencil) from region chunk (i, c) to
// the tile, whose rows are T .. T + RHO - 1 and columns kDtHalo .. kDtHalo +
// RHO - 1 of the region.
template <int RHO>
__device__ __forceinline__ int chunk_distance(int i, int c, int T) {
  const int dy = max(0, max(T - i, i - (T + RHO - 1)));
  const int dx = max(0, max(kDtHalo - 4 * c - 3, 4 * c - kDtHalo - RHO + 1));
  return max(dx, dy);
}

template <int RHO, bool LAMBDA>
__global__ __launch_bounds__(DtGeom<RHO>::NT) void k_diffuse_tb(const float *__restrict__ in,
                                                                float *__restrict__ out, int r,
                                                                int rb, uint64_t tile_base,
                                                                uint64_t ntiles, int T,
                                                                float alpha) {
  using G = DtGeom<RHO>;
  constexpr int NT = G::NT;
  constexpr int KS = G::KMAX;
  static_assert(G::SLOTS < (1 << kChunkBits), "chunk index fits its field");
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
  const int lane = __lane_id();
  const int n = 1 << r;
  const int X0 = (int)bx * RHO, Y0 = (int)by * RHO;
  const int xr0 = X0 - kDtHalo, yr0 = Y0 - T;  // region origin
  const int R = RHO + 2 * T;
  const int nslots = R * G::CC;
  // region cell (i, x) of a plane is at i * CW + x
  float *plane0 = flds;
  float *plane1 = flds + R * G::CW;

  if (tid == 0) nchunk = 0u;
  __syncthreads();  // the count is zero before any wave adds to it

  // 1. load, and list the chunks while the loads are in flight (the list is
  //    built in plane1's memory)
  const uint64_t lanes_below = (1ull << lane) - 1ull;
  uint32_t *list = reinterpret_cast<uint32_t *>(plane1);
  float4 v[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int e = tid + kk * NT;
    const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
    const int y = yr0 + i, x = xr0 + 4 * c;
    const bool has = e < nslots && y >= 0 && y < n && x >= 0 && x < n && (x & y) == 0;
    v[kk] = has ? *reinterpret_cast<const float4 *>(in + (size_t)y * n + x)
                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int d = chunk_distance<RHO>(i, c, T);
    const bool live = has && d < T;
    const uint64_t ball = __ballot(live);
    if (ball != 0ull) {  // uniform: every lane of the wave is here
      uint32_t base = 0u;
      if (lane == 0) base = atomicAdd(&nchunk, (uint32_t)__popcll(ball));
      base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
      if (live) list[base + (uint32_t)__popcll(ball & lanes_below)] = (uint32_t)e | ((uint32_t)d << kDistShift);
    }
  }
  // plane0 takes the loaded values (chunk e starts at float 4e, since rows are
  // CW = 4 CC floats)
  float4 *q0 = reinterpret_cast<float4 *>(plane0);
  float4 *q1 = reinterpret_cast<float4 *>(plane1);
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int e = tid + kk * NT;
    if (e < nslots) q0[e] = v[kk];
  }
  __syncthreads();
  const int nc = (int)nchunk;
  const int kheld = (nc + NT - 1) / NT;  // register slots in use (uniform)

  // 2. this thread's chunks, in registers
  int off[KS], steps_live[KS];
  float deg[KS][4], wt[KS][4];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = tid + kk * NT;
    off[kk] = 0;
    steps_live[kk] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) deg[kk][j] = wt[kk][j] = 0.0f;
    if (kk < kheld && k < nc) {
      const uint32_t word = list[k];
      const int e = (int)(word & ((1u << kChunkBits) - 1u));
      off[kk] = 4 * e;  // rows are CW = 4 CC floats, so chunk e starts at float 4e
      steps_live[kk] = T - (int)(word >> kDistShift);
      // neighbour counts, one byte per cell: north + south + west + east,
      // each 0 or 1 (a listed chunk's first cell is on the gasket)
      const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
      const int y = yr0 + i, x = xr0 + 4 * c;
      const uint32_t S = chunk_row_bytes((uint32_t)y & 3u);
      const uint32_t U = (y > 0 && (x & (y - 1)) == 0) ? chunk_row_bytes((uint32_t)(y - 1) & 3u) : 0u;
      const uint32_t D = (y + 1 < n && (x & (y + 1)) == 0) ? chunk_row_bytes((uint32_t)(y + 1) & 3u) : 0u;
      const uint32_t wb = (x > 0 && ((x - 1) & y) == 0) ? 1u : 0u;
      const uint32_t eb = (x + 4 < n && ((x + 4) & y) == 0) ? 0x01000000u : 0u;
      const uint32_t degs = U + D + ((S << 8) | wb) + ((S >> 8) | eb);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        deg[kk][j] = (float)((degs >> (8 * j)) & 0xFFu);  // one v_cvt_f32_ubyte<j>
        wt[kk][j] = ((S >> (8 * j)) & 1u) ? alpha : 0.0f;
      }
    }
  }
  __syncthreads();  // the list is read before plane1 is cleared

  // 3. plane1 cleared, then T steps
  for (int e = tid; e < nslots; e += NT) q1[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  float4 cur[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk)
    cur[kk] = kk < kheld && steps_live[kk] > 0 ? *reinterpret_cast<const float4 *>(plane0 + off[kk])
                                 : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int s = 0; s < T; ++s) {
    const float *src = (s & 1) ? plane1 : plane0;
    float *dst = (s & 1) ? plane0 : plane1;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      if (kk >= kheld) break;             // no thread holds a chunk here
      if (s >= steps_live[kk]) continue;  // cannot reach the tile any more
      const float *p = src + off[kk];
      const float4 N = *reinterpret_cast<const float4 *>(p - G::CW);
      const float4 S = *reinterpret_cast<const float4 *>(p + G::CW);
      const float Wn = p[-1], En = p[4];
      const float cu[4] = {cur[kk].x, cur[kk].y, cur[kk].z, cur[kk].w};
      const float nu[4] = {N.x, N.y, N.z, N.w}, su[4] = {S.x, S.y, S.z, S.w};
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float w = j == 0 ? Wn : cu[j - 1];
        const float ee = j == 3 ? En : cu[j + 1];
        o[j] = __builtin_fmaf(wt[kk][j],
                              __builtin_fmaf(-deg[kk][j], cu[j], (w + ee) + (nu[j] + su[j])), cu[j]);
      }
      cur[kk] = make_float4(o[0], o[1], o[2], o[3]);
      *reinterpret_cast<float4 *>(dst + off[kk]) = cur[kk];
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
    const float4 w = *reinterpret_cast<const float4 *>(fin + (T + ty) * G::CW + kDtHalo + 4 * c);
    *reinterpret_cast<float4 *>(out + (size_t)y * n + x) = w;
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

bool diffuse_tb_supported(int rho) { return rho == 16 || rho == 32 || rho == 64; }

hipError_t launch_diffuse_tb(const PassArgs &a, int T, const float *in, float *out,
                             float alpha) {
  if (T < 1 || T > kMaxDiffuseStepsPerPass) return hipErrorInvalidValue;
  switch (a.rho) {
    case 16: return diffuse_tb_rho<16>(a, T, in, out, alpha);
    case 32: return diffuse_tb_rho<32>(a, T, in, out, alpha);
    case 64: return diffuse_tb_rho<64>(a, T, in, out, alpha);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
