// HIP kernels for gfx950: the lambda and bounding-box block maps, and the
// passes they feed (write, B3/S23 life, FP32 diffusion).
//
// Every pass shares one tile body between the two maps; only the block ->
// tile assignment differs:
//   lambda: workgroup slot s of workgroup g takes omega = g * TPG + s and
//           decodes it with lambda (Eq. 4-10): 3^r_b tiles, all fractal.
//   bbox:   the same slot takes block t = g * TPG + s of the n_b x n_b grid
//           under the identity (bx, by) = (t mod n_b, t div n_b) and discards
//           the tile's lanes unless bx & by == 0: 4^r_b tiles.
// Inside a fractal tile the lanes use bounding sub-boxes (Section III-D):
// every lane keeps its cells and masks those with (tx & ty) != 0.
//
// Two lane layouts:
//   rows  (rho <= 16): one lane per tile row, 64/rho tiles per wave; the rows
//         above/below come from the neighbouring lanes (DPP wave shifts).
//   strip (rho >= 32): lanes run along x in 16-byte chunks, so one wave
//         instruction covers whole 128-byte lines of a tile row; each lane
//         walks down a band of 16 rows holding the band plus its two halo rows
//         in registers, and the left/right neighbour cells of interior chunks
//         come from the adjacent lanes (DPP wave shifts).
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

// Tile assignment for slot `slot` of this workgroup.  Returns false when the
// slot holds no fractal tile (ragged tail, or a discarded bbox block).
template <bool LAMBDA>
__device__ __forceinline__ bool tile_of(uint64_t tile_base, uint64_t ntiles,
                                        int tpg, int slot, int rb, uint32_t &bx,
                                        uint32_t &by) {
  const uint64_t t = tile_base + (uint64_t)logical_group() * (uint64_t)tpg + (uint64_t)slot;
  if (t >= ntiles) return false;
  if constexpr (LAMBDA) {
    pass_decode((uint32_t)t, rb, bx, by);
    return true;
  } else {
    by = (uint32_t)(t >> rb);
    bx = (uint32_t)(t & ((1ull << rb) - 1ull));
    return (bx & by) == 0u;
  }
}

// ------------------------------------------------------------------ maps

__global__ __launch_bounds__(kWG) void k_map_lambda(uint2 *__restrict__ out,
                                                    int rb, uint32_t count) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  uint32_t bx, by;
  lambda_decode(i, rb, bx, by);
  out[i] = make_uint2(bx, by);
}

__global__ __launch_bounds__(kWG) void k_map_bbox(uint8_t *__restrict__ mask,
                                                  int rb, uint64_t base,
                                                  uint64_t count) {
  const uint64_t t = base + (uint64_t)blockIdx.x * kWG + threadIdx.x;
  if (t >= count) return;
  const uint32_t by = (uint32_t)(t >> rb);
  const uint32_t bx = (uint32_t)(t & ((1ull << rb) - 1ull));
  mask[t] = (uint8_t)((bx & by) == 0u);
}

// ------------------------------------------------------------------ write pass

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__(NT) void k_write(uint8_t *__restrict__ a, int r,
                                               int rb, uint64_t tile_base,
                                               uint64_t ntiles, uint32_t value) {
  constexpr int TPG = NT / RHO;
  const int slot = threadIdx.x / RHO;
  const uint32_t ty = threadIdx.x % RHO;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, TPG, slot, rb, bx, by)) return;
  const size_t n = (size_t)1 << r;
  const size_t y = (size_t)by * RHO + ty;
  const size_t x0 = (size_t)bx * RHO;
  U8Row<RHO> row;
#pragma unroll
  for (int k = 0; k < U8Row<RHO>::NW; ++k) row.w[k] = row_mask_word<RHO>(k, ty) * value;
  store_row<RHO>(a + y * n + x0, row);
}

// ------------------------------------------------------------------ life

// Byte i <- byte i-1 of the row, byte 0 <- `in` (a 0..255 value).
template <int RHO>
__device__ __forceinline__ void shift_in_left(U8Row<RHO> &o, const U8Row<RHO> &v,
                                              uint32_t in) {
  constexpr int NW = U8Row<RHO>::NW;
  if constexpr (RHO < 4) {
    o.w[0] = ((v.w[0] << 8) | in) & ((1u << (8 * RHO)) - 1u);
  } else {
    o.w[0] = (v.w[0] << 8) | in;
#pragma unroll
    for (int k = 1; k < NW; ++k) o.w[k] = (v.w[k] << 8) | (v.w[k - 1] >> 24);
  }
}

// Byte i <- byte i+1 of the row, byte RHO-1 <- `in`.
template <int RHO>
__device__ __forceinline__ void shift_in_right(U8Row<RHO> &o, const U8Row<RHO> &v,
                                               uint32_t in) {
  constexpr int NW = U8Row<RHO>::NW;
  if constexpr (RHO < 4) {
    o.w[0] = (v.w[0] >> 8) | (in << (8 * (RHO - 1)));
  } else {
#pragma unroll
    for (int k = 0; k < NW - 1; ++k) o.w[k] = (v.w[k] >> 8) | (v.w[k + 1] << 24);
    o.w[NW - 1] = (v.w[NW - 1] >> 8) | (in << 24);
  }
}

__device__ __forceinline__ bool on_gasket(size_t x, size_t y) { return (x & y) == 0; }

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__(NT) void k_life(const uint8_t *__restrict__ in,
                                              uint8_t *__restrict__ out, int r,
                                              int rb, uint64_t tile_base,
                                              uint64_t ntiles) {
  constexpr int TPG = NT / RHO;
  constexpr int NW = U8Row<RHO>::NW;
  const int slot = threadIdx.x / RHO;
  const uint32_t ty = threadIdx.x % RHO;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, TPG, slot, rb, bx, by)) return;

  const size_t n = (size_t)1 << r;
  const size_t X0 = (size_t)bx * RHO, Y0 = (size_t)by * RHO;
  const size_t y = Y0 + ty;
  const bool has_l = X0 > 0, has_r = X0 + RHO < n;
  const size_t xl = X0 - 1, xr = X0 + RHO;

  // every load of the lane is issued before the first wait: its own row and
  // left/right neighbour cells, and, on the tile's first / last row, the halo
  // row above / below with its corner cells
  U8Row<RHO> C, HU, HD;
  zero_row<RHO>(HU);
  zero_row<RHO>(HD);
  load_row<RHO>(C, in + y * n + X0);
  uint32_t cl = (has_l && on_gasket(xl, y)) ? in[y * n + xl] : 0u;
  uint32_t cr = (has_r && on_gasket(xr, y)) ? in[y * n + xr] : 0u;
  uint32_t hul = 0u, hur = 0u, hdl = 0u, hdr = 0u;
  if (ty == 0 && Y0 > 0) {
    const size_t yu = Y0 - 1;
    if (on_gasket(X0, yu)) load_row<RHO>(HU, in + yu * n + X0);
    if (has_l && on_gasket(xl, yu)) hul = in[yu * n + xl];
    if (has_r && on_gasket(xr, yu)) hur = in[yu * n + xr];
  }
  if (ty == RHO - 1 && Y0 + RHO < n) {
    const size_t yd = Y0 + RHO;
    if (on_gasket(X0, yd)) load_row<RHO>(HD, in + yd * n + X0);
    if (has_l && on_gasket(xl, yd)) hdl = in[yd * n + xl];
    if (has_r && on_gasket(xr, yd)) hdr = in[yd * n + xr];
  }

  // rows above / below: neighbouring lanes, or the halo row at the tile edges
  U8Row<RHO> U, D;
  uint32_t ul = from_prev_lane(cl), ur = from_prev_lane(cr);
  uint32_t dl = from_next_lane(cl), dr = from_next_lane(cr);
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    U.w[k] = from_prev_lane(C.w[k]);
    D.w[k] = from_next_lane(C.w[k]);
  }
  if (ty == 0) {
    U = HU;
    ul = hul;
    ur = hur;
  }
  if (ty == RHO - 1) {
    D = HD;
    dl = hdl;
    dr = hdr;
  }

  // column sums of the 3 rows, then the 3-wide horizontal sum (bytes <= 9)
  U8Row<RHO> V, L, R, O;
#pragma unroll
  for (int k = 0; k < NW; ++k) V.w[k] = U.w[k] + C.w[k] + D.w[k];
  shift_in_left<RHO>(L, V, ul + cl + dl);
  shift_in_right<RHO>(R, V, ur + cr + dr);
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t cnt = L.w[k] + V.w[k] + R.w[k] - C.w[k];  // live neighbours
    // B3/S23: alive iff (cnt | self) == 3, tested per byte on 4-bit values
    const uint32_t x = (cnt | C.w[k]) ^ 0x03030303u;
    uint32_t z = x | (x >> 1);
    z |= z >> 2;
    O.w[k] = ~z & row_mask_word<RHO>(k, ty);
  }
  store_row<RHO>(out + y * n + X0, O);
}

// ------------------------------------------------------------------ diffusion

template <int RHO>
struct F32Row {
  float v[RHO];
};

template <int RHO>
__device__ __forceinline__ void load_frow(F32Row<RHO> &row, const float *p) {
  if constexpr (RHO == 1) {
    row.v[0] = p[0];
  } else if constexpr (RHO == 2) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    row.v[0] = t.x;
    row.v[1] = t.y;
  } else {
#pragma unroll
    for (int k = 0; k < RHO / 4; ++k) {
      const float4 t = reinterpret_cast<const float4 *>(p)[k];
      row.v[4 * k + 0] = t.x;
      row.v[4 * k + 1] = t.y;
      row.v[4 * k + 2] = t.z;
      row.v[4 * k + 3] = t.w;
    }
  }
}

template <int RHO>
__device__ __forceinline__ void store_frow(float *p, const F32Row<RHO> &row) {
  if constexpr (RHO == 1) {
    p[0] = row.v[0];
  } else if constexpr (RHO == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(row.v[0], row.v[1]);
  } else {
#pragma unroll
    for (int k = 0; k < RHO / 4; ++k)
      reinterpret_cast<float4 *>(p)[k] =
          make_float4(row.v[4 * k], row.v[4 * k + 1], row.v[4 * k + 2], row.v[4 * k + 3]);
  }
}

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__(NT) void k_diffuse(const float *__restrict__ in,
                                                 float *__restrict__ out, int r,
                                                 int rb, uint64_t tile_base,
                                                 uint64_t ntiles, float alpha) {
  constexpr int TPG = NT / RHO;
  const int slot = threadIdx.x / RHO;
  const uint32_t ty = threadIdx.x % RHO;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, TPG, slot, rb, bx, by)) return;

  const size_t n = (size_t)1 << r;
  const size_t X0 = (size_t)bx * RHO, Y0 = (size_t)by * RHO;
  const size_t y = Y0 + ty;
  const bool has_l = X0 > 0, has_r = X0 + RHO < n;
  const bool has_u = y > 0, has_d = y + 1 < n;
  const size_t xl = X0 - 1, xr = X0 + RHO;

  // all loads first (own row, left/right cells, halo rows at the tile edges)
  F32Row<RHO> C, U, D, O, HU, HD;
#pragma unroll
  for (int i = 0; i < RHO; ++i) HU.v[i] = HD.v[i] = 0.0f;
  load_frow<RHO>(C, in + y * n + X0);
  const bool ml = has_l && on_gasket(xl, y), mr = has_r && on_gasket(xr, y);
  const float cl = ml ? in[y * n + xl] : 0.0f;
  const float cr = mr ? in[y * n + xr] : 0.0f;
  if (ty == 0 && Y0 > 0 && on_gasket(X0, Y0 - 1)) load_frow<RHO>(HU, in + (Y0 - 1) * n + X0);
  if (ty == RHO - 1 && Y0 + RHO < n && on_gasket(X0, Y0 + RHO))
    load_frow<RHO>(HD, in + (Y0 + RHO) * n + X0);
#pragma unroll
  for (int i = 0; i < RHO; ++i) {
    U.v[i] = from_prev_lane(C.v[i]);
    D.v[i] = from_next_lane(C.v[i]);
  }
  if (ty == 0) U = HU;
  if (ty == RHO - 1) D = HD;

#pragma unroll
  for (int i = 0; i < RHO; ++i) {
    const size_t x = X0 + i;
    const float u = C.v[i];
    const bool mw = (i == 0) ? ml : on_gasket(x - 1, y);
    const bool me = (i == RHO - 1) ? mr : on_gasket(x + 1, y);
    const bool mn = has_u && on_gasket(x, y - 1);
    const bool ms = has_d && on_gasket(x, y + 1);
    const float w = (i == 0) ? cl : C.v[i - 1];
    const float e = (i == RHO - 1) ? cr : C.v[i + 1];
    O.v[i] = diffuse_cell(u, w, e, U.v[i], D.v[i], mw, me, mn, ms, on_gasket(x, y), alpha);
  }
  store_frow<RHO>(out + y * n + X0, O);
}


// ------------------------------------------------------------------ strip layout

constexpr int kBand = 16;  // rows per lane band in the strip layout

// HBM stores below a 64-byte granule cost a read-modify-write (measured at
// r = 16: the write pass stores 4.2x the gasket's bytes in 32-byte granules
// and 5.6x in 64-byte ones, yet takes 82.7 us against 49 us), and sparse reads
// run fastest as whole 128-byte lines.  The strip kernels store every granule
// of the largest size a tile row spans (64 bytes, or the 32-byte row of a
// rho = 32 u8 tile) that holds a gasket cell in full (0 on its off-gasket
// cells), and load every 128-byte line (or the whole row, if shorter) that
// holds one.  A granule that holds a gasket cell is exactly one whose first
// cell does: x0 & y == 0 for a granule starting at x0 (a multiple of its size).
template <int ROW_BYTES>
struct Granules {
  static constexpr int STORE = ROW_BYTES >= 64 ? 64 : (ROW_BYTES >= 32 ? 32 : 16);
  static constexpr int LOAD = ROW_BYTES >= 128 ? 128 : (ROW_BYTES >= 64 ? 64 : 16);
};

template <int RHO, int CHUNK, int NT>
struct Strip {
  static constexpr int CPR = RHO / CHUNK;         // chunks per tile row
  static constexpr int LPT = CPR * (RHO / kBand); // lanes per tile
  static constexpr int WGS = LPT > NT ? LPT : NT;
  static constexpr int TPG = WGS / LPT;           // tiles per workgroup
};

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__((Strip<RHO, 16, NT>::WGS)) void k_write_strip(
    uint8_t *__restrict__ a, int r, int rb, uint64_t tile_base, uint64_t ntiles,
    uint32_t value) {
  using G = Strip<RHO, 16, NT>;
  const int slot = threadIdx.x / G::LPT, lt = threadIdx.x % G::LPT;
  const int band = lt / G::CPR, c = lt % G::CPR;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, G::TPG, slot, rb, bx, by)) return;
  const size_t n = (size_t)1 << r;
  const size_t x = (size_t)bx * RHO + 16 * c;
  const size_t y0 = (size_t)by * RHO + (size_t)band * kBand;
#pragma unroll
  for (int i = 0; i < kBand; ++i) {
    const size_t y = y0 + i;
    constexpr size_t gmask = ~(size_t)(Granules<RHO>::STORE - 1);
    if (((x & gmask) & y) != 0) continue;  // no gasket cell in this granule
    // cells of this chunk are on the gasket iff x & y == 0 and (i & y) == 0
    const uint32_t v = (x & y) == 0 ? value : 0u;
    U8Row<16> row;
#pragma unroll
    for (int k = 0; k < 4; ++k) row.w[k] = row_mask_word<16>(k, (uint32_t)(y & 15)) * v;
    store_row<16>(a + y * n + x, row);
  }
}

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__((Strip<RHO, 16, NT>::WGS)) void k_life_strip(
    const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int r, int rb,
    uint64_t tile_base, uint64_t ntiles, int stream_out) {
  using G = Strip<RHO, 16, NT>;
  const int slot = threadIdx.x / G::LPT, lt = threadIdx.x % G::LPT;
  const int band = lt / G::CPR, c = lt % G::CPR;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, G::TPG, slot, rb, bx, by)) return;
  const size_t n = (size_t)1 << r;
  const size_t X0 = (size_t)bx * RHO, Y0 = (size_t)by * RHO;
  const size_t x = X0 + 16 * c;
  const size_t y0 = Y0 + (size_t)band * kBand;
  const bool left_edge = c == 0, right_edge = c == G::CPR - 1;
  const bool has_l = X0 > 0, has_r = X0 + RHO < n;
  const size_t xl = X0 - 1, xr = X0 + RHO;

  // the band's rows y0 .. y0+15 and the halo rows y0-1, y0+16
  U8Row<16> w[kBand + 2];
  uint32_t hl[kBand + 2], hr[kBand + 2];
#pragma unroll
  for (int i = 0; i < kBand + 2; ++i) {
    const bool ok = (i > 0 || y0 > 0) && (i < kBand + 1 || y0 + kBand < n);
    const size_t yy = y0 + i - 1;
    zero_row<16>(w[i]);
    hl[i] = hr[i] = 0u;
    constexpr size_t lmask = ~(size_t)(Granules<RHO>::LOAD - 1);
    if (ok && ((x & lmask) & yy) == 0) load_row<16>(w[i], in + yy * n + x);
    if (left_edge && ok && has_l && (xl & yy) == 0) hl[i] = in[yy * n + xl];
    if (right_edge && ok && has_r && (xr & yy) == 0) hr[i] = in[yy * n + xr];
  }
#pragma unroll
  for (int i = 1; i <= kBand; ++i) {
    const size_t y = y0 + i - 1;
    U8Row<16> V, L, R, O;
#pragma unroll
    for (int k = 0; k < 4; ++k) V.w[k] = w[i - 1].w[k] + w[i].w[k] + w[i + 1].w[k];
    const uint32_t from_l = from_prev_lane(V.w[3]) >> 24;   // byte 15 of chunk c-1
    const uint32_t from_r = from_next_lane(V.w[0]) & 0xffu;  // byte 0 of chunk c+1
    const uint32_t vl = left_edge ? hl[i - 1] + hl[i] + hl[i + 1] : from_l;
    const uint32_t vr = right_edge ? hr[i - 1] + hr[i] + hr[i + 1] : from_r;
    shift_in_left<16>(L, V, vl);
    shift_in_right<16>(R, V, vr);
    const uint32_t ym = (uint32_t)(y & 15);
    const uint32_t chunk_on = (x & y) == 0 ? ~0u : 0u;  // chunk holds gasket cells
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t cnt = L.w[k] + V.w[k] + R.w[k] - w[i].w[k];
      const uint32_t xx = (cnt | w[i].w[k]) ^ 0x03030303u;
      uint32_t z = xx | (xx >> 1);
      z |= z >> 2;
      O.w[k] = ~z & row_mask_word<16>(k, ym) & chunk_on;
    }
    constexpr size_t smask = ~(size_t)(Granules<RHO>::STORE - 1);
    if (((x & smask) & y) == 0) {
      // whole granules (rho >= 64) may stream; 32-byte rows never do
      if (RHO >= 64 && stream_out)
        store_row<16, true>(out + y * n + x, O);
      else
        store_row<16>(out + y * n + x, O);
    }
  }
}

template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__((Strip<RHO, 4, NT>::WGS)) void k_diffuse_strip(
    const float *__restrict__ in, float *__restrict__ out, int r, int rb,
    uint64_t tile_base, uint64_t ntiles, float alpha) {
  using G = Strip<RHO, 4, NT>;
  const int slot = threadIdx.x / G::LPT, lt = threadIdx.x % G::LPT;
  const int band = lt / G::CPR, c = lt % G::CPR;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, G::TPG, slot, rb, bx, by)) return;
  const size_t n = (size_t)1 << r;
  const size_t X0 = (size_t)bx * RHO, Y0 = (size_t)by * RHO;
  const size_t x = X0 + 4 * c;
  const size_t y0 = Y0 + (size_t)band * kBand;
  const bool left_edge = c == 0, right_edge = c == G::CPR - 1;
  const bool has_l = X0 > 0, has_r = X0 + RHO < n;
  const size_t xl = X0 - 1, xr = X0 + RHO;

  F32Row<4> w[kBand + 2];
  float hl[kBand + 2], hr[kBand + 2];
#pragma unroll
  for (int i = 0; i < kBand + 2; ++i) {
    const bool ok = (i > 0 || y0 > 0) && (i < kBand + 1 || y0 + kBand < n);
    const size_t yy = y0 + i - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i].v[j] = 0.0f;
    hl[i] = hr[i] = 0.0f;
    constexpr size_t lmask = ~(size_t)(Granules<4 * RHO>::LOAD / 4 - 1);
    if (ok && ((x & lmask) & yy) == 0) load_frow<4>(w[i], in + yy * n + x);
    if (left_edge && ok && has_l && (xl & yy) == 0) hl[i] = in[yy * n + xl];
    if (right_edge && ok && has_r && (xr & yy) == 0) hr[i] = in[yy * n + xr];
  }
#pragma unroll
  for (int i = 1; i <= kBand; ++i) {
    const size_t y = y0 + i - 1;
    const float from_l = from_prev_lane(w[i].v[3]);
    const float from_r = from_next_lane(w[i].v[0]);
    const float west0 = left_edge ? hl[i] : from_l;
    const float east3 = right_edge ? hr[i] : from_r;
    F32Row<4> O;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const size_t xj = x + j;
      const float u = w[i].v[j];
      const float west = j == 0 ? west0 : w[i].v[j - 1];
      const float east = j == 3 ? east3 : w[i].v[j + 1];
      const bool mw = xj > 0 && on_gasket(xj - 1, y);
      const bool me = xj + 1 < n && on_gasket(xj + 1, y);
      const bool mn = y > 0 && on_gasket(xj, y - 1);
      const bool ms = y + 1 < n && on_gasket(xj, y + 1);
      O.v[j] = diffuse_cell(u, west, east, w[i - 1].v[j], w[i + 1].v[j], mw, me, mn, ms,
                            on_gasket(xj, y), alpha);
    }
    constexpr size_t smask = ~(size_t)(Granules<4 * RHO>::STORE / 4 - 1);
    if (((x & smask) & y) == 0) store_frow<4>(out + y * n + x, O);
  }
}

// ------------------------------------------------------------------ launchers

// HIP bounds gridDim.x * blockDim.x below 2^32; launches are split into
// chunks of at most this many workgroups.
constexpr uint64_t kMaxGroupsPerLaunch = 1ull << 23;

template <typename F>
hipError_t launch_tiles(uint64_t ntiles, int tpg, hipStream_t s, F &&launch_one) {
  const uint64_t groups = (ntiles + tpg - 1) / tpg;
  const uint64_t per_launch = kMaxGroupsPerLaunch / 4;  // up to 1024 threads per group
  for (uint64_t g0 = 0; g0 < groups; g0 += per_launch) {
    const uint64_t g = groups - g0 < per_launch ? groups - g0 : per_launch;
    launch_one(dim3((unsigned)g), g0 * (uint64_t)tpg, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Workgroup size of a one-step pass: launches of fewer than kSmallLaunchWaves
// waves (small gaskets, where a pass is one latency chain) run one wave per
// workgroup, so they spread over more CUs; larger launches run four.
#ifndef SG_SMALL_LAUNCH_WAVES
#define SG_SMALL_LAUNCH_WAVES 2048
#endif
constexpr uint64_t kSmallLaunchWaves = SG_SMALL_LAUNCH_WAVES;
inline bool small_launch(uint64_t ntiles, int lanes_per_tile) {
  return ntiles * (uint64_t)lanes_per_tile < kSmallLaunchWaves * 64;
}

// Launches kernel K<NT> over all tiles with NT = 64 or 256 threads per group.
#define SG_LAUNCH_PASS(KERNEL, TPG_OF, WGS_OF, LANES, ...)                                 \
  do {                                                                                     \
    if (small_launch(a.ntiles, LANES))                                                     \
      return launch_tiles(a.ntiles, TPG_OF(64), a.stream, [&](dim3 g, uint64_t base, hipStream_t s) { \
        if (a.lambda)                                                                      \
          hipLaunchKernelGGL((KERNEL<RHO, true, 64>), g, dim3(WGS_OF(64)), 0, s, __VA_ARGS__); \
        else                                                                               \
          hipLaunchKernelGGL((KERNEL<RHO, false, 64>), g, dim3(WGS_OF(64)), 0, s, __VA_ARGS__); \
      });                                                                                  \
    return launch_tiles(a.ntiles, TPG_OF(256), a.stream, [&](dim3 g, uint64_t base, hipStream_t s) { \
      if (a.lambda)                                                                        \
        hipLaunchKernelGGL((KERNEL<RHO, true, 256>), g, dim3(WGS_OF(256)), 0, s, __VA_ARGS__); \
      else                                                                                 \
        hipLaunchKernelGGL((KERNEL<RHO, false, 256>), g, dim3(WGS_OF(256)), 0, s, __VA_ARGS__); \
    });                                                                                    \
  } while (0)

#define SG_ROWS_TPG(NT) ((NT) / RHO)
#define SG_ROWS_WGS(NT) (NT)
#define SG_STRIP16_TPG(NT) (Strip<RHO, 16, NT>::TPG)
#define SG_STRIP16_WGS(NT) (Strip<RHO, 16, NT>::WGS)
#define SG_STRIP4_TPG(NT) (Strip<RHO, 4, NT>::TPG)
#define SG_STRIP4_WGS(NT) (Strip<RHO, 4, NT>::WGS)

template <int RHO>
hipError_t write_strip(const PassArgs &a, uint8_t *d, uint32_t value) {
  SG_LAUNCH_PASS(k_write_strip, SG_STRIP16_TPG, SG_STRIP16_WGS, (Strip<RHO, 16, 64>::LPT),
                 d, a.r, a.rb, base, a.ntiles, value);
}

template <int RHO>
hipError_t life_strip(const PassArgs &a, const uint8_t *in, uint8_t *out) {
  const int stream_out = life_stream_stores(life_touched_bytes(a.r)) ? 1 : 0;
  SG_LAUNCH_PASS(k_life_strip, SG_STRIP16_TPG, SG_STRIP16_WGS, (Strip<RHO, 16, 64>::LPT),
                 in, out, a.r, a.rb, base, a.ntiles, stream_out);
}

template <int RHO>
hipError_t diffuse_strip(const PassArgs &a, const float *in, float *out, float alpha) {
  SG_LAUNCH_PASS(k_diffuse_strip, SG_STRIP4_TPG, SG_STRIP4_WGS, (Strip<RHO, 4, 64>::LPT),
                 in, out, a.r, a.rb, base, a.ntiles, alpha);
}

template <int RHO>
hipError_t write_rho(const PassArgs &a, uint8_t *d, uint32_t value) {
  SG_LAUNCH_PASS(k_write, SG_ROWS_TPG, SG_ROWS_WGS, RHO, d, a.r, a.rb, base, a.ntiles, value);
}

template <int RHO>
hipError_t life_rho(const PassArgs &a, const uint8_t *in, uint8_t *out) {
  SG_LAUNCH_PASS(k_life, SG_ROWS_TPG, SG_ROWS_WGS, RHO, in, out, a.r, a.rb, base, a.ntiles);
}

template <int RHO>
hipError_t diffuse_rho(const PassArgs &a, const float *in, float *out, float alpha) {
  SG_LAUNCH_PASS(k_diffuse, SG_ROWS_TPG, SG_ROWS_WGS, RHO, in, out, a.r, a.rb, base, a.ntiles,
                 alpha);
}

// ------------------------------------------------------------------ intra-block variants
//
// The paper's other two intra-block mappings (Section III-D), for the write
// pass: instead of rho x rho threads with a bounding sub-box test, only the
// 3^k threads that own a gasket cell of the tile are launched, and each finds
// its cell either by applying lambda again at thread level ("further
// unrolling": the tile is itself a gasket of level k) or by reading a table
// of the 3^k in-tile offsets shared by all tiles ("shared lookup table"),
// built once per workgroup in LDS.  One byte is stored per thread.

constexpr int pow3c(int k) { return k == 0 ? 1 : 3 * pow3c(k - 1); }
constexpr int log2c(int v) { return v <= 1 ? 0 : 1 + log2c(v / 2); }

template <int RHO, bool LAMBDA, bool LUT>
__global__ __launch_bounds__(kWG) void k_write_intra(uint8_t *__restrict__ a, int r, int rb,
                                                     uint64_t tile_base, uint64_t ntiles,
                                                     uint32_t value) {
  constexpr int K = log2c(RHO);
  constexpr int CELLS = pow3c(K);      // gasket cells per tile
  constexpr int TPG = kWG / CELLS;     // tiles per workgroup
  __shared__ uint32_t table[LUT ? CELLS : 1];
  const int tid = threadIdx.x;
  if constexpr (LUT) {
    for (int i = tid; i < CELLS; i += kWG) {
      uint32_t tx, ty;
      lambda_decode((uint32_t)i, K, tx, ty);
      table[i] = tx | (ty << 16);
    }
    __syncthreads();
  }
  const int slot = tid / CELLS, cell = tid - slot * CELLS;
  if (slot >= TPG) return;
  uint32_t bx, by;
  if (!tile_of<LAMBDA>(tile_base, ntiles, TPG, slot, rb, bx, by)) return;
  uint32_t tx, ty;
  if constexpr (LUT) {
    const uint32_t e = table[cell];
    tx = e & 0xffffu;
    ty = e >> 16;
  } else {
    lambda_decode((uint32_t)cell, K, tx, ty);
  }
  const size_t n = (size_t)1 << r;
  a[((size_t)by * RHO + ty) * n + (size_t)bx * RHO + tx] = (uint8_t)value;
}

template <int RHO, bool LUT>
hipError_t write_intra_rho(const PassArgs &a, uint8_t *d, uint32_t value) {
  constexpr int TPG = kWG / pow3c(log2c(RHO));
  return launch_tiles(a.ntiles, TPG, a.stream, [&](dim3 grid, uint64_t base, hipStream_t s) {
    if (a.lambda)
      hipLaunchKernelGGL((k_write_intra<RHO, true, LUT>), grid, dim3(kWG), 0, s, d, a.r, a.rb, base, a.ntiles, value);
    else
      hipLaunchKernelGGL((k_write_intra<RHO, false, LUT>), grid, dim3(kWG), 0, s, d, a.r, a.rb, base, a.ntiles, value);
  });
}

}  // namespace

hipError_t launch_map_lambda(int rb, uint32_t count, uint32_t *d_bxy, hipStream_t s) {
  const uint32_t groups = (count + kWG - 1) / kWG;
  if (groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_lambda, dim3(groups), dim3(kWG), 0, s,
                     reinterpret_cast<uint2 *>(d_bxy), rb, count);
  return hipGetLastError();
}

hipError_t launch_map_bbox(int rb, uint64_t count, uint8_t *d_mask, hipStream_t s) {
  return launch_tiles(count, kWG, s, [&](dim3 grid, uint64_t base, hipStream_t st) {
    hipLaunchKernelGGL(k_map_bbox, grid, dim3(kWG), 0, st, d_mask, rb, base, count);
  });
}

hipError_t launch_write(const PassArgs &a, uint8_t *d, uint8_t value) {
  switch (a.rho) {
    case 1: return write_rho<1>(a, d, value);
    case 2: return write_rho<2>(a, d, value);
    case 4: return write_rho<4>(a, d, value);
    case 8: return write_rho<8>(a, d, value);
    case 16: return write_rho<16>(a, d, value);
    case 32: return write_strip<32>(a, d, value);
    case 64: return write_strip<64>(a, d, value);
    case 128: return write_strip<128>(a, d, value);
    case 256: return write_strip<256>(a, d, value);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_write_intra(const PassArgs &a, uint8_t *d, uint8_t value, bool lut) {
  switch (a.rho) {
    case 1: return lut ? write_intra_rho<1, true>(a, d, value) : write_intra_rho<1, false>(a, d, value);
    case 2: return lut ? write_intra_rho<2, true>(a, d, value) : write_intra_rho<2, false>(a, d, value);
    case 4: return lut ? write_intra_rho<4, true>(a, d, value) : write_intra_rho<4, false>(a, d, value);
    case 8: return lut ? write_intra_rho<8, true>(a, d, value) : write_intra_rho<8, false>(a, d, value);
    case 16: return lut ? write_intra_rho<16, true>(a, d, value) : write_intra_rho<16, false>(a, d, value);
    case 32: return lut ? write_intra_rho<32, true>(a, d, value) : write_intra_rho<32, false>(a, d, value);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_life(const PassArgs &a, const uint8_t *in, uint8_t *out) {
  switch (a.rho) {
    case 1: return life_rho<1>(a, in, out);
    case 2: return life_rho<2>(a, in, out);
    case 4: return life_rho<4>(a, in, out);
    case 8: return life_rho<8>(a, in, out);
    case 16: return life_rho<16>(a, in, out);
    case 32: return life_strip<32>(a, in, out);
    case 64: return life_strip<64>(a, in, out);
    case 128: return life_strip<128>(a, in, out);
    case 256: return life_strip<256>(a, in, out);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_diffuse(const PassArgs &a, const float *in, float *out, float alpha) {
  switch (a.rho) {
    case 1: return diffuse_rho<1>(a, in, out, alpha);
    case 2: return diffuse_rho<2>(a, in, out, alpha);
    case 4: return diffuse_rho<4>(a, in, out, alpha);
    case 8: return diffuse_rho<8>(a, in, out, alpha);
    case 16: return diffuse_rho<16>(a, in, out, alpha);
    case 32: return diffuse_strip<32>(a, in, out, alpha);
    case 64: return diffuse_strip<64>(a, in, out, alpha);
    case 128: return diffuse_strip<128>(a, in, out, alpha);
    case 256: return diffuse_strip<256>(a, in, out, alpha);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
