// Temporally blocked B3/S23 life on the gasket (gfx950).
//
// One workgroup owns one rho x rho tile of the map (lambda or bounding box)
// and advances it by T generations per pass (T <= 16), so HBM is read and
// written once per T steps instead of once per step.
//
//  1. Load the tile plus a halo of T rows above/below and one 16-byte chunk
//     left/right (T <= 16 cells) from HBM, skipping chunks with no gasket
//     cell, and bit-pack each 16-byte chunk of 0/1 bytes into 16 bits of an
//     LDS plane (one bit per cell, 32 cells per word).
//  2. List, once, the plane words that hold a gasket cell (wavefront ballot +
//     prefix count), with each word's gasket mask (bounding sub-box test
//     x & y == 0 applied to 32 cells at once).
//  3. T times: every listed word computes its next state from the 3 x 3
//     words around it with a bit-sliced adder (counts of the 8 neighbours as
//     bit planes) and the B3/S23 rule, masked to the gasket; planes ping-pong
//     with a barrier between generations.  Cells outside the region are taken
//     as dead; the wrong values this makes at the region's cut edges move
//     inward one cell per generation and never reach the tile in T <= 16.
//  4. Unpack the tile and store every 64-byte granule that holds a gasket
//     cell in full.
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kTbThreads = 256;

// 16 bytes holding 0/1 -> 16 bits (bit i = byte i).
__device__ __forceinline__ uint32_t pack16(const uint4 v) {
  auto p4 = [](uint32_t w) { return (w | (w >> 7) | (w >> 14) | (w >> 21)) & 0xFu; };
  return p4(v.x) | (p4(v.y) << 4) | (p4(v.z) << 8) | (p4(v.w) << 12);
}

// 16 bits -> 16 bytes holding 0/1.
__device__ __forceinline__ uint4 unpack16(uint32_t b) {
  auto u4 = [](uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; };
  return make_uint4(u4(b & 0xFu), u4((b >> 4) & 0xFu), u4((b >> 8) & 0xFu),
                    u4((b >> 12) & 0xFu));
}

// Gasket cells of a 32-cell word starting at a multiple of 32 in row y, for a
// word whose first cell is on the gasket: bit i set iff (i & y) == 0.
__device__ __forceinline__ uint32_t word_pattern(uint32_t y) {
  uint32_t m = 0xFFFFFFFFu;
  if (y & 1u) m &= 0x55555555u;
  if (y & 2u) m &= 0x33333333u;
  if (y & 4u) m &= 0x0F0F0F0Fu;
  if (y & 8u) m &= 0x00FF00FFu;
  if (y & 16u) m &= 0x0000FFFFu;
  return m;
}

// Next state of 32 cells.  a, b, c: the word in the rows above, at and below;
// *L / *R: the words to their left / right.  Neighbour counts are summed as
// bit planes: each row contributes (lsb, carry) of its 3 (or 2) cells, the
// three lsbs add to bit0 + 2k, and the count is 2 or 3 iff exactly one of
// (carry_a, carry_b, carry_c, k) is set.
__device__ __forceinline__ uint32_t life_word(uint32_t a, uint32_t aL, uint32_t aR,
                                              uint32_t b, uint32_t bL, uint32_t bR,
                                              uint32_t c, uint32_t cL, uint32_t cR) {
  const uint32_t aw = __builtin_amdgcn_alignbit(a, aL, 31);  // west neighbours
  const uint32_t ae = __builtin_amdgcn_alignbit(aR, a, 1);   // east neighbours
  const uint32_t bw = __builtin_amdgcn_alignbit(b, bL, 31);
  const uint32_t be = __builtin_amdgcn_alignbit(bR, b, 1);
  const uint32_t cw = __builtin_amdgcn_alignbit(c, cL, 31);
  const uint32_t ce = __builtin_amdgcn_alignbit(cR, c, 1);
  const uint32_t sa = aw ^ a ^ ae, ca = (aw & a) | (aw & ae) | (a & ae);
  const uint32_t sb = bw ^ be, cb = bw & be;
  const uint32_t sc = cw ^ c ^ ce, cc = (cw & c) | (cw & ce) | (c & ce);
  const uint32_t bit0 = sa ^ sb ^ sc;
  const uint32_t k = (sa & sb) | (sa & sc) | (sb & sc);
  const uint32_t x3 = ca ^ cb ^ cc;
  const uint32_t m3 = (ca & cb) | (ca & cc) | (cb & cc);
  const uint32_t o3 = ca | cb | cc;
  const uint32_t e3 = x3 & ~m3;                   // exactly one carry
  const uint32_t eq1 = (e3 & ~k) | (~o3 & k);     // exactly one of four
  return eq1 & (bit0 | b);
}

template <int RHO, bool LAMBDA>
__global__ __launch_bounds__(kTbThreads) void k_life_tb(const uint8_t *__restrict__ in,
                                                        uint8_t *__restrict__ out, int r,
                                                        int rb, uint64_t tile_base,
                                                        uint64_t ntiles, int T) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t nitems;
  constexpr int W = RHO / 32 + 2;   // region words per row
  constexpr int PW = W + 2;         // plane pitch (zero guard word each side)
  constexpr int CH = RHO / 16 + 2;  // loaded 16-byte chunks per region row
  const int R = RHO + 2 * T;        // region rows
  const int PR = R + 2;             // plane rows (zero guard row each side)
  const int tid = threadIdx.x;

  const uint64_t t = tile_base + blockIdx.x;
  if (t >= ntiles) return;
  uint32_t bx, by;
  if constexpr (LAMBDA) {
    lambda_decode((uint32_t)t, rb, bx, by);
  } else {
    by = (uint32_t)(t >> rb);
    bx = (uint32_t)(t & ((1ull << rb) - 1ull));
    if ((bx & by) != 0u) return;
  }
  const int64_t n = (int64_t)1 << r;
  const int64_t X0 = (int64_t)bx * RHO, Y0 = (int64_t)by * RHO;
  const int64_t yr0 = Y0 - T;  // row of region row 0

  uint32_t *plane0 = lds;
  uint32_t *plane1 = lds + PR * PW;
  uint32_t *items = plane1 + PR * PW;
  uint32_t *imask = items + R * W;

  for (int i = tid; i < 2 * PR * PW; i += kTbThreads) lds[i] = 0u;
  if (tid == 0) nitems = 0u;
  __syncthreads();

  // 1. load and bit-pack the region
  uint16_t *p0h = reinterpret_cast<uint16_t *>(plane0);
  for (int e = tid; e < R * CH; e += kTbThreads) {
    const int i = e / CH, j = e - (e / CH) * CH;
    const int64_t y = yr0 + i, x = X0 - 16 + 16 * j;
    if (y < 0 || y >= n || x < 0 || x >= n || (x & y) != 0) continue;
    const uint4 v = *reinterpret_cast<const uint4 *>(in + y * n + x);
    const int w = (j + 1) >> 1, half = (j + 1) & 1;
    p0h[((i + 1) * PW + (w + 1)) * 2 + half] = (uint16_t)pack16(v);
  }

  // 2. compact list of the words that hold a gasket cell
  const int lane = __lane_id();
  for (int base = 0; base < R * W; base += kTbThreads) {
    const int e = base + tid;
    uint32_t m = 0u;
    int idx = 0;
    if (e < R * W) {
      const int i = e / W, w = e - (e / W) * W;
      const int64_t y = yr0 + i, xw = X0 - 32 + 32 * w;
      if (y >= 0 && y < n && xw >= 0 && xw < n && (xw & y) == 0) m = word_pattern((uint32_t)y);
      idx = (i + 1) * PW + (w + 1);
    }
    const uint64_t ball = __ballot(m != 0u);
    const uint32_t before = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    uint32_t off = 0u;
    if (lane == 0 && ball != 0ull) off = atomicAdd(&nitems, (uint32_t)__popcll(ball));
    off = __shfl(off, 0);
    if (m != 0u) {
      items[off + before] = (uint32_t)idx;
      imask[off + before] = m;
    }
  }
  __syncthreads();
  const int ni = (int)nitems;

  // 3. T generations in LDS
  for (int s = 0; s < T; ++s) {
    const uint32_t *src = (s & 1) ? plane1 : plane0;
    uint32_t *dst = (s & 1) ? plane0 : plane1;
    for (int e = tid; e < ni; e += kTbThreads) {
      const int idx = (int)items[e];
      const uint32_t *p = src + idx;
      dst[idx] = life_word(p[-PW], p[-PW - 1], p[-PW + 1], p[0], p[-1], p[1], p[PW],
                           p[PW - 1], p[PW + 1]) &
                 imask[e];
    }
    __syncthreads();
  }
  const uint16_t *fin = reinterpret_cast<const uint16_t *>((T & 1) ? plane1 : plane0);

  // 4. unpack and store the tile, whole 64-byte granules
  constexpr int TC = RHO / 16;
  for (int e = tid; e < RHO * TC; e += kTbThreads) {
    const int ty = e / TC, j = e - (e / TC) * TC;
    const int64_t y = Y0 + ty, x = X0 + 16 * j;
    if (((x & ~(int64_t)63) & y) != 0) continue;
    const int w = 1 + (j >> 1), half = j & 1;
    const uint32_t bits = fin[((T + ty + 1) * PW + (w + 1)) * 2 + half];
    *reinterpret_cast<uint4 *>(out + y * n + x) = unpack16(bits);
  }
}

template <int RHO>
size_t tb_lds_bytes(int T) {
  const int W = RHO / 32 + 2, PW = W + 2, R = RHO + 2 * T, PR = R + 2;
  return sizeof(uint32_t) * (size_t)(2 * PR * PW + 2 * R * W);
}

template <int RHO>
hipError_t life_tb_rho(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  const size_t lds = tb_lds_bytes<RHO>(T);
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    if (a.lambda)
      hipLaunchKernelGGL((k_life_tb<RHO, true>), dim3((unsigned)g), dim3(kTbThreads), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T);
    else
      hipLaunchKernelGGL((k_life_tb<RHO, false>), dim3((unsigned)g), dim3(kTbThreads), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

bool life_tb_supported(int rho) { return rho == 64 || rho == 128 || rho == 256; }

hipError_t launch_life_tb(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  if (T < 1 || T > kMaxStepsPerPass) return hipErrorInvalidValue;
  switch (a.rho) {
    case 64: return life_tb_rho<64>(a, T, in, out);
    case 128: return life_tb_rho<128>(a, T, in, out);
    case 256: return life_tb_rho<256>(a, T, in, out);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
