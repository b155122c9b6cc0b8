// Temporally blocked FP32 diffusion on the gasket (gfx950).
//
// One workgroup owns one rho x rho tile (rho in {16, 32, 64}) of the map and
// advances it by T <= 16 explicit diffusion steps per pass, over a region of
// the tile plus T rows above and below and H columns each side (H = 8 for
// T <= 8, else 16):
//  1. every thread takes entries of a compile-time table of the region's
//     4-cell chunks (DtTable: the chunks that hold a gasket cell within H
//     stencil steps of the tile, whatever block they lie in), keeps those
//     whose block holds gasket cells and that lie within T steps, and loads
//     them; while the loads are in flight the LDS planes are cleared.
//     Then the loaded chunks go to the first plane, and the ones that can
//     still reach the tile (distance < T) are listed (wavefront ballot +
//     prefix count), each as one word: its region index, its distance, its
//     gasket cells and the count deg of in-grid gasket neighbours of each
//     cell;
//  2. each thread takes its listed chunks into registers: the chunk's LDS
//     offset, the number of steps in which it can still reach the tile, and
//     per cell deg and a weight (alpha on the gasket, 0 off it);
//  3. T times: every held chunk updates its 4 cells with the arithmetic of
//     diffuse_cell, the function the one-step kernels use, as
//     fma(w, fma(-deg, u, (W + E) + (N + S)), u); off the gasket w = 0 keeps
//     the value, which is 0 (the inner fma is finite there).  A chunk's own
//     values stay in registers.  At rho >= 32 the neighbours come from one
//     plane updated in place: every held chunk reads its neighbours and
//     computes, a barrier, it stores its new values, a barrier (one plane
//     lets twice the workgroups share a compute unit at rho = 64).  At
//     rho = 16, whose workgroups already fill a compute unit's wave slots,
//     two planes ping-pong with one barrier per step;
//  4. store the tile, every 64-byte granule that holds a gasket cell in full.
//
// The 4-neighbour stencil moves information one cell per step, so a cell at
// Manhattan distance D from the tile reaches it after D steps.  By induction
// over the steps, every cell within T - t of the tile holds its exact value
// after t steps: its neighbours are within T - t + 1, and its chunk (whose
// distance is that of its nearest cell) was loaded (distance <= T) and
// updated in every step so far (a chunk at distance d updates while t <
// T - d).  Every other cell may hold a wrong value (a cell that was never
// loaded reads as 0, a chunk that stopped keeps a stale one, and a row's west
// neighbour of its first chunk is the previous row's last cell), which
// cannot reach the tile in the steps left.  Rows 0 and R - 1 of the region
// are T cells from the tile, so no updated chunk reads outside the plane.
#include <atomic>

#include <type_traits>

#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

// Halo columns each side of a pass of T steps: whole float4 chunks, 8 or 16.
constexpr int dt_halo(int T) { return T <= 8 ? 8 : 16; }
static_assert(dt_halo(kMaxDiffuseStepsPerPass) >= kMaxDiffuseStepsPerPass, "the halo covers a pass");

template <int RHO, int H>
struct DtGeom {
  static constexpr int CW = RHO + 2 * H;  // region columns = plane pitch (floats)
  static constexpr int CC = CW / 4;       // region chunks per row
  // one plane updated in place (rho >= 32), or two that ping-pong (rho = 16)
  static constexpr bool kInPlace = RHO >= 32;
  // plane stride (floats): the largest region's rows, so a second plane is a
  // fixed offset from the first and every LDS access of a step is a base
  // register plus an immediate
  static constexpr int PLANE = (RHO + 2 * H) * CW;
  static_assert(PLANE * 4 + (2 * CW + 4) * 4 < 65536, "LDS offsets fit their 16-bit field");
  static constexpr int NT = RHO >= 64 ? 512 : 256;
  // chunks of the largest region (T = H)
  static constexpr int SLOTS = (RHO + 2 * H) * CC;
};

// The region chunks of a tile pass, fixed per tile side.
//
// Inside every block of the gasket's block grid that holds gasket cells,
// cell (xl, yl) is on the gasket iff xl & yl == 0, and two such blocks touch
// only at single cells: cell (0, 0) of a block has its west and north
// neighbours in the blocks to its west and north (their cells (rho - 1, 0)
// and (0, rho - 1), on the gasket whenever the block is), cell (rho - 1, 0)
// its east one in the block to its east, and cell (0, rho - 1) its south one
// in the block below; no other gasket cell has a neighbour outside its block.
// So the chunks of a pass's region, their distance to the tile and the
// neighbour counts of their cells are fixed per tile side, up to which of the
// 3 x 3 blocks around the tile hold gasket cells (and lie in the grid).  The
// table of a halo H lists, row by row, every chunk that holds a gasket cell
// within H steps (Manhattan distance) of the tile, as two words:
//   w0: region chunk column j (5 bits) | region row + H (7) << 5 |
//       block (dbx + 1) + 3 (dby + 1) (4) << 12 | distance (5) << 16
//   w1: in-block neighbour count of each cell (3 bits each) | gasket cells
//       (4) << 12 | block whose cells add one neighbour to cell 0 or 3 (4)
//       << 16 | block that adds one to cell 0 (4) << 20 | 1 << 24 when the
//       first adds to cell 3 | 1 << 25 when cell 0's west neighbour is a
//       gasket cell of the same block | 1 << 26 when cell 3's east one is;
//       15 names no block.
// Every gasket cell has a gasket neighbour in its own block (a block is a
// connected gasket of side rho >= 2), so a cell is on the gasket iff its
// neighbour count is not 0.
constexpr int kDtMaxChunks = 768;
constexpr uint32_t kDtNone = 15u;

struct DtTable {
  int n = 0;
  uint32_t w0[kDtMaxChunks] = {};
  uint32_t w1[kDtMaxChunks] = {};
};

template <int RHO, int H>
constexpr DtTable make_dt_table() {
  DtTable t{};
  constexpr int CC = DtGeom<RHO, H>::CC;
  auto on = [](int xl, int yl) {
    return xl >= 0 && yl >= 0 && xl < RHO && yl < RHO && (xl & yl) == 0;
  };
  auto block = [](int dbx, int dby) -> uint32_t {
    // every neighbour block a listed cell reaches is one of the 3 x 3
    return (dbx < -1 || dbx > 1 || dby < -1 || dby > 1) ? 0xFFFFu
                                                        : (uint32_t)((dbx + 1) + 3 * (dby + 1));
  };
  for (int irel = -H; irel < RHO + H; ++irel)
    for (int j = 0; j < CC; ++j) {
      const int xrel = 4 * j - H;  // first cell's column, relative to the tile's
      const int dby = irel < 0 ? -1 : (irel >= RHO ? 1 : 0);
      const int dbx = xrel < 0 ? -1 : (xrel >= RHO ? 1 : 0);
      const int yl = irel - dby * RHO, xl = xrel - dbx * RHO;
      if ((xl & yl) != 0) continue;  // no gasket cell in the chunk (xl is a multiple of 4)
      const int dy = irel < 0 ? -irel : (irel > RHO - 1 ? irel - (RHO - 1) : 0);
      const int dx = xrel + 3 < 0 ? -(xrel + 3) : (xrel > RHO - 1 ? xrel - (RHO - 1) : 0);
      const int d = dx + dy;
      if (d > H) continue;
      uint32_t deg = 0, cells = 0;
      for (int c = 0; c < 4; ++c) {
        const int x = xl + c;
        if (!on(x, yl)) continue;
        cells |= 1u << c;
        const int k = (int)on(x - 1, yl) + (int)on(x + 1, yl) + (int)on(x, yl - 1) + (int)on(x, yl + 1);
        deg |= (uint32_t)k << (3 * c);
      }
      uint32_t a = kDtNone, b = kDtNone, a3 = 0;
      if (xl == 0 && yl == 0) {
        a = block(dbx - 1, dby);  // west neighbour of cell 0
        b = block(dbx, dby - 1);  // north neighbour of cell 0
      } else if (xl == RHO - 4 && yl == 0) {
        a = block(dbx + 1, dby);  // east neighbour of cell 3
        a3 = 1;
      } else if (xl == 0 && yl == RHO - 1) {
        b = block(dbx, dby + 1);  // south neighbour of cell 0
      }
      // A neighbour block beyond the 3 x 3 is met only by a cell on the far
      // side of a neighbour block, rho >= H steps from the tile: that cell
      // never reaches the tile, so its count may leave the block out.
      const int cx = a3 ? xrel + 3 : xrel;  // the cell the cross terms belong to
      const int cd = (irel < 0 ? -irel : (irel > RHO - 1 ? irel - (RHO - 1) : 0)) +
                     (cx < 0 ? -cx : (cx > RHO - 1 ? cx - (RHO - 1) : 0));
      if ((a > kDtNone || b > kDtNone) && cd < H) {
        t.n = -1;  // a case the table cannot express: rejected below
        return t;
      }
      if (a > kDtNone) a = kDtNone;
      if (b > kDtNone) b = kDtNone;
      if (t.n == kDtMaxChunks) {
        t.n = -1;
        return t;
      }
      t.w0[t.n] = (uint32_t)j | (uint32_t)(irel + H) << 5 | block(dbx, dby) << 12 |
                  (uint32_t)d << 16;
      const uint32_t west = (uint32_t)on(xl - 1, yl), east = (uint32_t)on(xl + 4, yl);
      t.w1[t.n++] = deg | cells << 12 | a << 16 | b << 20 | a3 << 24 | west << 25 | east << 26;
    }
  return t;
}

template <int RHO, int H>
struct DtTableOf {
  static constexpr DtTable table = make_dt_table<RHO, H>();
  static_assert(table.n > 0, "the region's chunks fit the table");
  static_assert(RHO + 2 * H < 128 && DtGeom<RHO, H>::CC < 32, "the table's fields hold the region");
  static constexpr int n = table.n;
};
template <int RHO, int H>
__constant__ DtTable kDtTable = DtTableOf<RHO, H>::table;

template <int RHO, int H>
size_t dt_lds_bytes(int T) {
  using G = DtGeom<RHO, H>;
  const size_t planes = G::kInPlace ? (size_t)(RHO + 2 * T) * G::CW
                                    : (size_t)G::PLANE + (size_t)(RHO + 2 * T) * G::CW;
  return sizeof(float) * planes + sizeof(uint32_t) * DtTableOf<RHO, H>::n;
}

// Lane i receives lane i - 1's (wave_shr:1) or lane i + 1's (wave_shl:1)
// value; lanes 0 and 63 receive 0.
__device__ __forceinline__ float prev_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float next_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// List word: region chunk index (12 bits) | distance to the tile (5) << 12 |
// 1 << 17 when cell 0's west neighbour is a gasket cell | 1 << 18 when cell
// 3's east neighbour is | neighbour count of each cell (3 bits each) << 19.
constexpr int kChunkBits = 12;
static_assert(DtGeom<64, 16>::SLOTS < (1 << kChunkBits), "chunk index fits its field");

template <int RHO, bool LAMBDA, int H>
__global__ __launch_bounds__((DtGeom<RHO, H>::NT)) void k_diffuse_tb(const float *__restrict__ in,
                                                                   float *__restrict__ out, int r,
                                                                   int rb, uint64_t tile_base,
                                                                   uint64_t ntiles, int T,
                                                                   float alpha) {
  using G = DtGeom<RHO, H>;
  constexpr int NT = G::NT;
  constexpr int NE = DtTableOf<RHO, H>::n;   // table entries
  constexpr int KE = (NE + NT - 1) / NT;     // entries per thread
  extern __shared__ __align__(16) float flds[];
  __shared__ uint32_t nchunk;
  const int tid = threadIdx.x;
  // this thread's table entries, first: they depend on nothing else
  uint32_t ew0[KE], ew1[KE];
#pragma unroll
  for (int kk = 0; kk < KE; ++kk) {
    const int k = tid + kk * NT;
    ew0[kk] = k < NE ? kDtTable<RHO, H>.w0[k] : 0xFFFFFFFFu;
    ew1[kk] = k < NE ? kDtTable<RHO, H>.w1[k] : 0u;
  }
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
  const int lane = __lane_id();
  const int n = 1 << r;
  const int nbk = 1 << rb;  // blocks per grid side
  const int X0 = (int)bx * RHO, Y0 = (int)by * RHO;
  const int R = RHO + 2 * T;
  const int nslots = R * G::CC;
  // region cell (i, x) of a plane is at i * CW + x
  float *plane0 = flds;
  float *plane1 = G::kInPlace ? plane0 : flds + G::PLANE;  // the ping-pong partner
  uint32_t *list = reinterpret_cast<uint32_t *>(plane1 + R * G::CW);

  // the 3 x 3 blocks around the tile that hold gasket cells: bit b =
  // (dbx + 1) + 3 (dby + 1), lane b testing block b
  uint32_t live;
  {
    const int b = lane < 9 ? lane : 0, q = (b * 11) >> 5;  // q = b / 3
    const int Bx = (int)bx + (b - 3 * q) - 1, By = (int)by + q - 1;
    live = (uint32_t)__ballot(lane < 9 && Bx >= 0 && By >= 0 && Bx < nbk && By < nbk &&
                              (Bx & By) == 0);
  }

  // 1. the region loads, in flight while the planes are cleared
  float4 v[KE];
#pragma unroll
  for (int kk = 0; kk < KE; ++kk) {
    const uint32_t w = ew0[kk];
    const int d = (int)((w >> 16) & 31u);
    const bool has = ((live >> ((w >> 12) & 15u)) & 1u) != 0u && d <= T;
    const int y = Y0 + (int)((w >> 5) & 127u) - H;
    const int x = X0 + 4 * (int)(w & 31u) - H;
    v[kk] = has ? *reinterpret_cast<const float4 *>(in + (size_t)y * n + x)
                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  {
    float4 *z = reinterpret_cast<float4 *>(flds);
    const int n4 = G::kInPlace ? nslots : G::PLANE / 4 + nslots;
    for (int e = tid; e < n4; e += NT) z[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  if (tid == 0) nchunk = 0u;
  __syncthreads();

  // the loaded chunks go to plane 0; those within T - 1 steps are listed
  const uint64_t lanes_below = (1ull << lane) - 1ull;
  float4 *q0 = reinterpret_cast<float4 *>(plane0);
#pragma unroll
  for (int kk = 0; kk < KE; ++kk) {
    if (tid + kk * NT - lane >= NE) break;  // no entry in this wave (uniform)
    const uint32_t w = ew0[kk], w1 = ew1[kk];
    const int d = (int)((w >> 16) & 31u);
    const bool has = ((live >> ((w >> 12) & 15u)) & 1u) != 0u && d <= T;
    const int e = ((int)((w >> 5) & 127u) - H + T) * G::CC + (int)(w & 31u);
    if (has) q0[e] = v[kk];
    const bool listed = has && d < T;
    const uint64_t ball = __ballot(listed);
    if (ball != 0ull) {  // uniform: every lane of the wave is here
      uint32_t base = 0u;
      if (lane == 0) base = atomicAdd(&nchunk, (uint32_t)__popcll(ball));
      base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
      // neighbour counts with the neighbours in other blocks
      const uint32_t xa = (live >> ((w1 >> 16) & 15u)) & 1u;
      const uint32_t xb = (live >> ((w1 >> 20) & 15u)) & 1u;
      const uint32_t a3 = (w1 >> 24) & 1u;
      const uint32_t deg = (w1 & 0xFFFu) + (xa << (a3 * 9u)) + xb;
      const uint32_t west = ((w1 >> 25) & 1u) | (xa & (a3 ^ 1u));  // block A: west of cell 0
      const uint32_t east = ((w1 >> 26) & 1u) | (xa & a3);         // or east of cell 3
      if (listed)
        list[base + (uint32_t)__popcll(ball & lanes_below)] =
            (uint32_t)e | (uint32_t)d << kChunkBits | west << 17 | east << 18 | deg << 19;
    }
  }
  __syncthreads();
  const int nc = (int)nchunk;
  const int kheld = (nc + NT - 1) / NT;  // register slots in use (uniform)

  // 2. this thread's chunks, in registers.  A chunk's west neighbour cell
  //    (that of its cell 0) is 0 off the gasket; on it, it is the last cell
  //    of the previous list entry, which the previous lane holds when that
  //    entry is the adjacent chunk (wave shift), else it is read from the
  //    plane (lane 0, or a chunk loaded but not listed).  Likewise east.
  constexpr uint32_t kIdx = (1u << kChunkBits) - 1u;
  int off[KE], steps_live[KE];
  uint32_t nb[KE];  // bit 0 / 1: west from the lane / the plane; bit 2 / 3: east
  float deg[KE][4], wt[KE][4];
#pragma unroll
  for (int kk = 0; kk < KE; ++kk) {
    const int k = tid + kk * NT;
    off[kk] = 0;
    steps_live[kk] = 0;
    nb[kk] = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) deg[kk][j] = wt[kk][j] = 0.0f;
    if (kk < kheld && k < nc) {
      const uint32_t word = list[k];
      const uint32_t e = word & kIdx;
      off[kk] = 4 * (int)e;  // rows are CW = 4 CC floats
      steps_live[kk] = T - (int)((word >> kChunkBits) & 31u);
      const bool wl = lane > 0 && (list[k - 1] & kIdx) == e - 1u;
      const bool el = lane < 63 && k + 1 < nc && (list[k + 1] & kIdx) == e + 1u;
      const bool wg = (word >> 17) & 1u, eg = (word >> 18) & 1u;
      nb[kk] = (wg && wl ? 1u : 0u) | (wg && !wl ? 2u : 0u) | (eg && el ? 4u : 0u) |
               (eg && !el ? 8u : 0u);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t dj = (word >> (19 + 3 * j)) & 7u;
        deg[kk][j] = (float)dj;
        wt[kk][j] = dj != 0u ? alpha : 0.0f;
      }
    }
  }

  // 3. T steps
  float4 cur[KE];
#pragma unroll
  for (int kk = 0; kk < KE; ++kk)
    cur[kk] = kk < kheld && steps_live[kk] > 0 ? *reinterpret_cast<const float4 *>(plane0 + off[kk])
                                 : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // One step from the plane at float offset SRC to the one at DST (0 or
  // PLANE; both 0 in place): every access is relative to the chunk's north
  // neighbour in plane 0, so its address is one register plus an immediate.
  auto step = [&](int s, auto src_off, auto dst_off) {
    constexpr int SRC = decltype(src_off)::value, DST = decltype(dst_off)::value;
#pragma unroll
    for (int kk = 0; kk < KE; ++kk) {
      if (kk >= kheld) break;  // no thread holds a chunk here
      // the neighbouring lanes' cells, before any lane leaves
      const float wlane = prev_lane(cur[kk].w), elane = next_lane(cur[kk].x);
      if (s >= steps_live[kk]) continue;  // cannot reach the tile any more
      float *q = plane0 + off[kk] - G::CW;  // the north neighbour in plane 0
      const float4 N = *reinterpret_cast<const float4 *>(q + SRC);
      const float4 S = *reinterpret_cast<const float4 *>(q + SRC + 2 * G::CW);
      float Wn = (nb[kk] & 1u) ? wlane : 0.0f, En = (nb[kk] & 4u) ? elane : 0.0f;
      if (nb[kk] & 2u) Wn = q[SRC + G::CW - 1];
      if (nb[kk] & 8u) En = q[SRC + G::CW + 4];
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
      if constexpr (!G::kInPlace) *reinterpret_cast<float4 *>(q + DST + G::CW) = cur[kk];
    }
    __syncthreads();  // in place: every read of the step is done
    if constexpr (G::kInPlace) {
#pragma unroll
      for (int kk = 0; kk < KE; ++kk) {
        if (kk >= kheld) break;
        if (s >= steps_live[kk]) continue;
        *reinterpret_cast<float4 *>(plane0 + off[kk]) = cur[kk];
      }
      __syncthreads();
    }
  };
  using Zero = std::integral_constant<int, 0>;
  using Second = std::integral_constant<int, G::PLANE>;
  if constexpr (G::kInPlace) {
    for (int s = 0; s < T; ++s) step(s, Zero{}, Zero{});
  } else {
    int s = 0;
    for (; s + 1 < T; s += 2) {
      step(s, Zero{}, Second{});
      step(s + 1, Second{}, Zero{});
    }
    if (s < T) step(s, Zero{}, Second{});
  }
  const float *fin = (T & 1) ? plane1 : plane0;

  // 4. store the tile, whole 64-byte granules (16 floats)
  constexpr int TC = RHO / 4;
  for (int e = tid; e < RHO * TC; e += NT) {
    const int ty = e / TC, c = e - (e / TC) * TC;
    const int y = Y0 + ty, x = X0 + 4 * c;
    if (((x & ~15) & y) != 0) continue;
    const float4 w = *reinterpret_cast<const float4 *>(fin + (T + ty) * G::CW + H + 4 * c);
    *reinterpret_cast<float4 *>(out + (size_t)y * n + x) = w;
  }
}

// The current device's LDS per workgroup, queried once per device.
hipError_t max_lds_per_block(size_t &bytes) {
  constexpr int kDevices = 64;
  static std::atomic<int> cached[kDevices];  // 0: not queried yet (every writer stores the same)
  int dev = 0, v = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const bool slot = dev >= 0 && dev < kDevices;
  if (slot && (v = cached[dev].load(std::memory_order_relaxed)) > 0) {
    bytes = (size_t)v;
    return hipSuccess;
  }
  e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if (slot) cached[dev].store(v, std::memory_order_relaxed);
  bytes = (size_t)v;
  return hipSuccess;
}

template <int RHO, int H>
hipError_t diffuse_tb_rho(const PassArgs &a, int T, const float *in, float *out, float alpha) {
  const size_t lds = dt_lds_bytes<RHO, H>(T);
  size_t max_lds = 0;
  hipError_t e = max_lds_per_block(max_lds);
  if (e != hipSuccess) return e;
  if (lds > max_lds) return hipErrorInvalidValue;  // (160 KB on gfx950: every pass fits)
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    if (a.lambda)
      hipLaunchKernelGGL((k_diffuse_tb<RHO, true, H>), dim3((unsigned)g),
                         dim3(DtGeom<RHO, H>::NT), lds, a.stream, in, out, a.r, a.rb, g0,
                         a.ntiles, T, alpha);
    else
      hipLaunchKernelGGL((k_diffuse_tb<RHO, false, H>), dim3((unsigned)g),
                         dim3(DtGeom<RHO, H>::NT), lds, a.stream, in, out, a.r, a.rb, g0,
                         a.ntiles, T, alpha);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO>
hipError_t diffuse_tb_rho(const PassArgs &a, int T, const float *in, float *out, float alpha) {
  return dt_halo(T) == 8 ? diffuse_tb_rho<RHO, 8>(a, T, in, out, alpha)
                         : diffuse_tb_rho<RHO, 16>(a, T, in, out, alpha);
}

}  // namespace

bool diffuse_tb_supported(int rho) { return rho == 16 || rho == 32 || rho == 64; }
int diffuse_tb_default_steps(int rho) { return rho == 32 ? 8 : 16; }

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
