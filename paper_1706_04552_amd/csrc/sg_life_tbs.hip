// Temporally blocked B3/S23 life for tiles of side 16 on the gasket (gfx950),
// below the 32-cell words of k_life_tb.  Written for any side that is a
// multiple of 16; side 32 is served by k_life_tb, which is faster there.
//
// One workgroup owns one rho x rho tile of the map and advances it by T <= 16
// generations per pass:
//  1. load the tile plus a halo of T rows above/below and 16 cells left/right
//     (one 16-byte chunk) into registers, every load issued before the first
//     wait, skipping chunks with no gasket cell, and write them to the first
//     LDS plane (one byte per cell, rows of 16 * CC bytes);
//  2. list the chunks that hold a gasket cell and can reach the tile in T
//     generations (wavefront ballot + prefix count), each as one word: its
//     region index and its distance to the tile (Chebyshev, in cells: the
//     8-neighbour rule moves information one cell per generation).  The list
//     is built in the second plane's memory, which is not in use yet;
//  3. each thread takes its listed chunks into registers: the LDS offset, the
//     generations in which the chunk can still reach the tile, its cells'
//     gasket mask (the bounding sub-box test of Section III-D per byte) and
//     its state;
//  4. clear the second plane, then T times: every held chunk applies the rule
//     in SWAR over its 16 bytes -- column sums of the rows above, at and below
//     (bytes <= 3), the 3-wide horizontal sum by byte shifts with the edge
//     cells of the neighbouring chunks, count = sum - self, alive iff
//     (count | self) == 3, masked to the gasket -- the arithmetic of the
//     one-generation kernels.  Planes ping-pong with a barrier between
//     generations;
//  5. store the tile rows (whole 32-byte granules for rho = 32), every chunk
//     whose granule holds a gasket cell.
//
// Cells outside the region hold wrong values (a row's west neighbour of its
// first chunk is the previous row's last cell), and a chunk stops updating
// once it can no longer reach the tile in the generations left, leaving stale
// values behind it; every such cell is more generations away from the tile
// than remain, so the tile is exactly T one-generation passes.  Rows 0 and
// R - 1 of the region are T cells from the tile and never updated, so an
// updated chunk reads at most one byte beyond either end of its plane, into
// a zero pad.
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kLsHalo = 16;  // halo cells each side: one chunk

template <int RHO>
struct LsGeom {
  static constexpr int CW = RHO + 2 * kLsHalo;  // region columns = plane pitch (bytes)
  static constexpr int CC = CW / 16;             // chunks per region row
  static constexpr int NT = 256;
  static constexpr int SLOTS = (RHO + 2 * kMaxSmallTileSteps) * CC;
  static constexpr int KMAX = (SLOTS + NT - 1) / NT;
  static constexpr int STORE = RHO >= 32 ? 32 : 16;  // store granule (bytes)
};

// Two planes between 16-byte zero pads: the diagonal neighbours of the first
// chunk of row 1 and of the last chunk of row R - 2 are one byte outside the
// planes (cells beyond the tile's reach, which must still read as 0 or 1).
constexpr int kLsPad = 16;

template <int RHO>
size_t ls_lds_bytes(int T) {
  return 2 * (size_t)(RHO + 2 * T) * LsGeom<RHO>::CW + 2 * kLsPad;
}

// List word: region chunk index (11 bits) | distance to the tile (< T) << 27.
constexpr int kLsChunkBits = 11;
constexpr int kLsDistShift = 27;

template <int RHO>
__device__ __forceinline__ int ls_distance(int i, int c, int T) {
  const int dy = max(0, max(T - i, i - (T + RHO - 1)));
  const int dx = max(0, max(kLsHalo - 16 * c - 15, 16 * c - kLsHalo - RHO + 1));
  return max(dx, dy);
}

// Byte j <- byte j - 1 of the 16-byte row, byte 0 <- `in`.
__device__ __forceinline__ void ls_shift_in_left(uint32_t o[4], const uint32_t v[4],
                                                 uint32_t in) {
  o[0] = (v[0] << 8) | in;
#pragma unroll
  for (int k = 1; k < 4; ++k) o[k] = (v[k] << 8) | (v[k - 1] >> 24);
}

// Byte j <- byte j + 1, byte 15 <- `in`.
__device__ __forceinline__ void ls_shift_in_right(uint32_t o[4], const uint32_t v[4],
                                                  uint32_t in) {
#pragma unroll
  for (int k = 0; k < 3; ++k) o[k] = (v[k] >> 8) | (v[k + 1] << 24);
  o[3] = (v[3] >> 8) | (in << 24);
}

template <int RHO, bool LAMBDA>
__global__ __launch_bounds__(LsGeom<RHO>::NT) void k_life_tbs(const uint8_t *__restrict__ in,
                                                              uint8_t *__restrict__ out, int r,
                                                              int rb, uint64_t tile_base,
                                                              uint64_t ntiles, int T) {
  using G = LsGeom<RHO>;
  constexpr int NT = G::NT;
  constexpr int KS = G::KMAX;
  constexpr int CW = G::CW;
  static_assert(G::SLOTS < (1 << kLsChunkBits), "chunk index fits its field");
  extern __shared__ __align__(16) uint8_t blds[];
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
  const int xr0 = X0 - kLsHalo, yr0 = Y0 - T;  // region origin
  const int R = RHO + 2 * T;
  const int nslots = R * G::CC;
  // region cell (i, x) of a plane is at byte i * CW + x; chunk e = i * CC + c
  // starts at byte 16 e
  uint8_t *plane0 = blds + kLsPad;
  uint8_t *plane1 = plane0 + R * CW;
  uint4 *q0 = reinterpret_cast<uint4 *>(plane0);
  uint4 *q1 = reinterpret_cast<uint4 *>(plane1);

  // 1. load
  uint4 v[KS];
  bool has[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int e = tid + kk * NT;
    const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
    const int y = yr0 + i, x = xr0 + 16 * c;
    has[kk] = e < nslots && y >= 0 && y < n && x >= 0 && x < n && (x & y) == 0;
    v[kk] = has[kk] ? *reinterpret_cast<const uint4 *>(in + (size_t)y * n + x)
                    : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int e = tid + kk * NT;
    if (e < nslots) q0[e] = v[kk];
  }
  if (tid == 0) nchunk = 0u;
  if (tid < 2)  // the pads
    *reinterpret_cast<uint4 *>(tid == 0 ? blds : plane1 + R * CW) = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();

  // 2. the list, built in plane1's memory
  uint32_t *list = reinterpret_cast<uint32_t *>(plane1);
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int e = tid + kk * NT;
    const int i = e / G::CC, c = e - (e / G::CC) * G::CC;
    const int d = ls_distance<RHO>(i, c, T);
    const bool live = has[kk] && d < T;
    const uint32_t word = (uint32_t)e | ((uint32_t)d << kLsDistShift);
    const uint64_t ball = __ballot(live);
    const uint32_t before = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    uint32_t base = 0u;
    if (lane == 0 && ball != 0ull) base = atomicAdd(&nchunk, (uint32_t)__popcll(ball));
    base = __shfl(base, 0);
    if (live) list[base + before] = word;
  }
  __syncthreads();
  const int nc = (int)nchunk;
  const int kheld = (nc + NT - 1) / NT;  // register slots in use (uniform)

  // 3. this thread's chunks, in registers
  int off[KS], steps_live[KS];
  uint32_t mask[KS][4];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = tid + kk * NT;
    off[kk] = 0;
    steps_live[kk] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) mask[kk][j] = 0u;
    if (kk < kheld && k < nc) {
      const uint32_t word = list[k];
      const int e = (int)(word & ((1u << kLsChunkBits) - 1u));
      off[kk] = 16 * e;
      steps_live[kk] = T - (int)(word >> kLsDistShift);
      const int i = e / G::CC;
      const uint32_t y = (uint32_t)(yr0 + i);  // listed chunks are in the grid and hold a
#pragma unroll                                 // gasket cell: x & y == 0 for their first x
      for (int j = 0; j < 4; ++j) mask[kk][j] = row_mask_word<16>(j, y & 15u);
    }
  }
  __syncthreads();  // the list is read before plane1 is cleared

  // 4. plane1 cleared, then T generations
  for (int e = tid; e < nslots; e += NT) q1[e] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  uint32_t cur[KS][4];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const uint4 c4 = kk < kheld && steps_live[kk] > 0
                         ? *reinterpret_cast<const uint4 *>(plane0 + off[kk])
                         : make_uint4(0u, 0u, 0u, 0u);
    cur[kk][0] = c4.x;
    cur[kk][1] = c4.y;
    cur[kk][2] = c4.z;
    cur[kk][3] = c4.w;
  }
  for (int s = 0; s < T; ++s) {
    const uint8_t *src = (s & 1) ? plane1 : plane0;
    uint8_t *dst = (s & 1) ? plane0 : plane1;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      if (kk >= kheld) break;             // no thread holds a chunk here
      if (s >= steps_live[kk]) continue;  // cannot reach the tile any more
      const uint8_t *p = src + off[kk];
      const uint4 N = *reinterpret_cast<const uint4 *>(p - CW);
      const uint4 S = *reinterpret_cast<const uint4 *>(p + CW);
      const uint32_t vl = (uint32_t)p[-1 - CW] + p[-1] + p[-1 + CW];  // west column
      const uint32_t vr = (uint32_t)p[16 - CW] + p[16] + p[16 + CW];  // east column
      const uint32_t nw[4] = {N.x, N.y, N.z, N.w}, sw[4] = {S.x, S.y, S.z, S.w};
      uint32_t V[4], L[4], Rr[4], O[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) V[k] = nw[k] + cur[kk][k] + sw[k];
      ls_shift_in_left(L, V, vl);
      ls_shift_in_right(Rr, V, vr);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t cnt = L[k] + V[k] + Rr[k] - cur[kk][k];  // live neighbours
        const uint32_t xx = (cnt | cur[kk][k]) ^ 0x03030303u;   // B3/S23: (cnt | self) == 3
        uint32_t z = xx | (xx >> 1);
        z |= z >> 2;
        O[k] = ~z & mask[kk][k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[kk][k] = O[k];
      *reinterpret_cast<uint4 *>(dst + off[kk]) = make_uint4(O[0], O[1], O[2], O[3]);
    }
    __syncthreads();
  }
  const uint8_t *fin = (T & 1) ? plane1 : plane0;

  // 5. store the tile
  constexpr int TC = RHO / 16;  // chunks per tile row
  for (int e = tid; e < RHO * TC; e += NT) {
    const int ty = e / TC, c = e - (e / TC) * TC;
    const int y = Y0 + ty, x = X0 + 16 * c;
    if (((x & ~(G::STORE - 1)) & y) != 0) continue;  // no gasket cell in its granule
    const uint4 w = *reinterpret_cast<const uint4 *>(fin + (T + ty) * CW + kLsHalo + 16 * c);
    *reinterpret_cast<uint4 *>(out + (size_t)y * n + x) = w;
  }
}

template <int RHO>
hipError_t life_tbs_rho(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  const size_t lds = ls_lds_bytes<RHO>(T);
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    if (a.lambda)
      hipLaunchKernelGGL((k_life_tbs<RHO, true>), dim3((unsigned)g), dim3(LsGeom<RHO>::NT), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T);
    else
      hipLaunchKernelGGL((k_life_tbs<RHO, false>), dim3((unsigned)g), dim3(LsGeom<RHO>::NT), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

bool life_tbs_supported(int rho) { return rho == 16; }

hipError_t launch_life_tbs(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  if (T < 1 || T > kMaxSmallTileSteps) return hipErrorInvalidValue;
  switch (a.rho) {
    case 16: return life_tbs_rho<16>(a, T, in, out);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
