// Rectangular blocks of rho_x = 2^a columns by rho_y = 2^b rows (Section
// III-B, which defines blocks of rho_x x rho_y threads; the analysis there
// takes rho_x = rho_y).  For a >= b a block (bx, by) holds a gasket cell iff
// bx & (by >> (a-b)) == 0: the 2^(a-b) blocks stacked in one 2^a x 2^a
// square are kept or dropped together, so the map decodes the square with
// lambda at level r - a and takes the position in the stack from the lowest
// bits of the block index (for b > a the roles of x and y swap).  With a = b
// it is lambda.  Wide, short blocks keep whole 64-byte rows with few cells
// per block.
#include "../../include/sg.h"
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

struct RectArgs {
  int r, a, b, rb, d;  // rho_x = 2^a, rho_y = 2^b, rb = r - max(a, b), d = |a - b|
  uint64_t ntiles;
};

// Canonical table (the square's omega in lambda's linear order, then the
// position in the stack).
__global__ __launch_bounds__(kWG) void k_map_lambda_rect(RectArgs p, uint32_t count,
                                                         uint2 *__restrict__ out) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const uint32_t j = i & ((1u << p.d) - 1u);
  uint32_t sx, sy;
  lambda_decode(i >> p.d, p.rb, sx, sy);
  out[i] = p.a >= p.b ? make_uint2(sx, (sy << p.d) | j) : make_uint2((sx << p.d) | j, sy);
}

template <bool LAMBDA>
__device__ __forceinline__ bool rect_tile(const RectArgs &p, uint64_t t, uint32_t &bx,
                                          uint32_t &by) {
  if (t >= p.ntiles) return false;
  if constexpr (LAMBDA) {
    const uint32_t j = (uint32_t)t & ((1u << p.d) - 1u);
    uint32_t sx, sy;
    pass_decode((uint32_t)(t >> p.d), p.rb, sx, sy);
    bx = p.a >= p.b ? sx : (sx << p.d) | j;
    by = p.a >= p.b ? (sy << p.d) | j : sy;
    return true;
  } else {
    const int cols = p.r - p.a;  // blocks per row: 2^(r - a)
    by = (uint32_t)(t >> cols);
    bx = (uint32_t)(t & ((1ull << cols) - 1ull));
    return p.a >= p.b ? (bx & (by >> p.d)) == 0u : ((bx >> p.d) & by) == 0u;
  }
}

// One lane per chunk of CW = min(rho_x, 16) bytes of a block row.
template <int RHOX, bool LAMBDA>
__global__ __launch_bounds__(kWG) void k_write_rect(RectArgs p, uint64_t tile_base, int tpg,
                                                    int lanes_per_tile, uint8_t *__restrict__ a,
                                                    uint32_t value) {
  constexpr int CW = RHOX < 16 ? RHOX : 16;
  constexpr int CPR = RHOX / CW;
  const uint64_t t0 = tile_base + (uint64_t)logical_group() * tpg;
  const size_t n = (size_t)1 << p.r;
  for (int e = threadIdx.x; e < tpg * lanes_per_tile; e += kWG) {
    const int slot = e / lanes_per_tile, l = e - slot * lanes_per_tile;
    uint32_t bx, by;
    if (!rect_tile<LAMBDA>(p, t0 + slot, bx, by)) continue;
    const int row = l / CPR, c = l - row * CPR;
    const size_t y = ((size_t)by << p.b) + row;
    const size_t x0 = ((size_t)bx << p.a) + (size_t)c * CW;
    if constexpr (RHOX >= 64) {
      if (((x0 & ~(size_t)63) & y) != 0) continue;  // no gasket cell in this 64-byte granule
    }
    const uint32_t on = (x0 & y) == 0 ? value : 0u;
    U8Row<CW> w;
#pragma unroll
    for (int k = 0; k < U8Row<CW>::NW; ++k) w.w[k] = row_mask_word<CW>(k, (uint32_t)(y & (CW - 1))) * on;
    store_row<CW>(a + y * n + x0, w);
  }
}

template <int RHOX>
hipError_t write_rect_rhox(const RectArgs &p, bool lambda, uint8_t *d, uint32_t value,
                           hipStream_t s) {
  constexpr int CW = RHOX < 16 ? RHOX : 16;
  const int lanes = (RHOX / CW) << p.b;
  const int tpg = lanes >= kWG ? 1 : kWG / lanes;
  const uint64_t groups = (p.ntiles + tpg - 1) / tpg;
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < groups; g0 += per_launch) {
    const uint64_t g = groups - g0 < per_launch ? groups - g0 : per_launch;
    if (lambda)
      hipLaunchKernelGGL((k_write_rect<RHOX, true>), dim3((unsigned)g), dim3(kWG), 0, s, p,
                         g0 * (uint64_t)tpg, tpg, lanes, d, value);
    else
      hipLaunchKernelGGL((k_write_rect<RHOX, false>), dim3((unsigned)g), dim3(kWG), 0, s, p,
                         g0 * (uint64_t)tpg, tpg, lanes, d, value);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int log2_pow2(int v) {
  if (v < 1 || v > SG_MAX_RHO || (v & (v - 1)) != 0) return -1;
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

int rect_args(int map, int r, int rho_x, int rho_y, RectArgs &p) {
  if (map != SG_MAP_LAMBDA && map != SG_MAP_BBOX) return SG_EINVAL;
  const int a = log2_pow2(rho_x), b = log2_pow2(rho_y);
  if (r < 0 || r > SG_MAX_R || a < 0 || b < 0 || a > r || b > r) return SG_EINVAL;
  p.r = r;
  p.a = a;
  p.b = b;
  p.rb = r - (a > b ? a : b);
  p.d = a > b ? a - b : b - a;
  uint64_t l = 1;
  for (int i = 0; i < p.rb; ++i) l *= 3;
  p.ntiles = map == SG_MAP_LAMBDA ? l << p.d : 1ull << (2 * r - a - b);
  return SG_OK;
}

}  // namespace
}  // namespace sg

extern "C" {

SG_API int sg_block_count_rect(int map, int r, int rho_x, int rho_y, uint64_t *blocks) {
  sg::RectArgs p;
  if (!blocks || sg::rect_args(map, r, rho_x, rho_y, p) != SG_OK) return SG_EINVAL;
  *blocks = p.ntiles;
  return SG_OK;
}

SG_API int sg_map_lambda_rect(int r, int rho_x, int rho_y, uint32_t *d_bxy, void *stream) {
  sg::RectArgs p;
  if (!d_bxy || ((uintptr_t)d_bxy & 7u)) return SG_EINVAL;
  if (sg::rect_args(SG_MAP_LAMBDA, r, rho_x, rho_y, p) != SG_OK) return SG_EINVAL;
  if (p.ntiles > 0x7fffffffull) return SG_EINVAL;
  if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
  const uint32_t count = (uint32_t)p.ntiles;
  hipLaunchKernelGGL(sg::k_map_lambda_rect, dim3((count + sg::kWG - 1) / sg::kWG), dim3(sg::kWG),
                     0, (hipStream_t)stream, p, count, (uint2 *)d_bxy);
  return sg::status_of(hipGetLastError());
}

SG_API int sg_write_pass_rect(int map, int r, int rho_x, int rho_y, uint8_t *d_a, uint8_t value,
                              void *stream) {
  sg::RectArgs p;
  if (!d_a || ((uintptr_t)d_a & 15u)) return SG_EINVAL;
  if (sg::rect_args(map, r, rho_x, rho_y, p) != SG_OK) return SG_EINVAL;
  if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
  const bool lam = map == SG_MAP_LAMBDA;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (rho_x) {
    case 1: e = sg::write_rect_rhox<1>(p, lam, d_a, value, s); break;
    case 2: e = sg::write_rect_rhox<2>(p, lam, d_a, value, s); break;
    case 4: e = sg::write_rect_rhox<4>(p, lam, d_a, value, s); break;
    case 8: e = sg::write_rect_rhox<8>(p, lam, d_a, value, s); break;
    case 16: e = sg::write_rect_rhox<16>(p, lam, d_a, value, s); break;
    case 32: e = sg::write_rect_rhox<32>(p, lam, d_a, value, s); break;
    case 64: e = sg::write_rect_rhox<64>(p, lam, d_a, value, s); break;
    case 128: e = sg::write_rect_rhox<128>(p, lam, d_a, value, s); break;
    default: e = sg::write_rect_rhox<256>(p, lam, d_a, value, s); break;
  }
  return sg::status_of(e);
}

}  // extern "C"
