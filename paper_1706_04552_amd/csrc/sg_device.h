// Device-side building blocks shared by the gasket kernels (gfx950, wave64).
//
// Tile model.  A "tile" is one rho x rho block of the n x n embedding.  One
// lane owns one row of one tile (rho <= 32 contiguous cells), so a wave holds
// 64/rho whole tiles with the tile's rows in consecutive lanes.  Row-major
// loads of a tile row are contiguous (coalesced into rho bytes, or 4*rho for
// FP32, per lane); the rows above and below come from the neighbouring lanes
// through DPP wave shifts, and only the tile's first and last rows fetch a
// halo row from memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

constexpr int kWG = 256;  // threads per workgroup: 4 wave64

// lambda(omega) decoded per block (Theorem 1, Eq. 4-10).
//
// omega is the linear index omega_y * W + omega_x with W = 3^floor(rb/2), so
// the base-3 digits of omega are omega_x's digits (low floor(rb/2) digits)
// followed by omega_y's.  Digit j of omega_x is beta at scale level
// mu = 2j + 2 and digit j of omega_y is beta at mu = 2j + 1 (Eq. 4), each
// contributing 2^(mu-1) (Eq. 6-7).  beta = 2 sets the x bit and beta >= 1 the
// y bit (Eq. 5).  The result is reflected into the build frame:
// by = n_b - 1 - lambda_y, i.e. the complement of lambda_y's r_b bits.
__device__ __forceinline__ void lambda_decode(uint32_t w, int rb, uint32_t &bx,
                                              uint32_t &by) {
  uint32_t lx = 0, ly = 0;
  const int hx = rb >> 1;
  for (int j = 0; j < rb; ++j) {
    const uint32_t q = w / 3u;
    const uint32_t d = w - 3u * q;
    w = q;
    const int bit = (j < hx) ? (2 * j + 1) : (2 * (j - hx));
    lx |= (uint32_t)(d == 2u) << bit;
    ly |= (uint32_t)(d != 0u) << bit;
  }
  bx = lx;
  by = ly ^ ((1u << rb) - 1u);
}

// The pass kernels read the digits of their workgroup index in level order:
// digit j is the region index beta at level mu = j + 1.  This is lambda
// composed with a fixed relabelling of the W x H grid (the digit of level mu
// belongs to omega_y for odd mu and to omega_x for even mu, Eq. 4, so the two
// enumerate the same (omega_x, omega_y) pairs); it makes 3^m consecutive
// workgroups one level-m sub-gasket of 2^m x 2^m blocks, so neighbouring
// tiles run together.
#ifndef SG_PASS_ORDER
#define SG_PASS_ORDER 1
#endif
// Bits (x, y) of two consecutive levels for each base-9 digit d = d0 + 3 d1
// (d0 the lower level): 2 bits per entry, entry d at bit 2d.
constexpr uint32_t level_pair_table(bool x) {
  uint32_t t = 0;
  for (uint32_t d = 0; d < 9; ++d) {
    const uint32_t d0 = d % 3, d1 = d / 3;
    const uint32_t b = x ? ((d0 == 2) | ((d1 == 2) << 1)) : ((d0 != 0) | ((d1 != 0) << 1));
    t |= b << (2 * d);
  }
  return t;
}
constexpr uint32_t kPairX = level_pair_table(true), kPairY = level_pair_table(false);

__device__ __forceinline__ void lambda_decode_levels(uint32_t t, int rb, uint32_t &bx,
                                                     uint32_t &by) {
  // two levels per step: t mod 9 indexes the (x, y) bit pairs of levels
  // 2i + 1 and 2i + 2; an odd rb ends with a digit d1 = 0
  uint32_t lx = 0, ly = 0;
  for (int j = 0; j < rb; j += 2) {
    const uint32_t q = t / 9u;
    const uint32_t d2 = (t - 9u * q) << 1;
    t = q;
    lx |= ((kPairX >> d2) & 3u) << j;
    ly |= ((kPairY >> d2) & 3u) << j;
  }
  bx = lx;
  by = ly ^ ((1u << rb) - 1u);
}
__device__ __forceinline__ void pass_decode(uint32_t t, int rb, uint32_t &bx, uint32_t &by) {
#if SG_PASS_ORDER
  lambda_decode_levels(t, rb, bx, by);
#else
  lambda_decode(t, rb, bx, by);
#endif
}

// Logical index of this workgroup.  Workgroups are dispatched round robin
// over the 8 XCDs (each with its own L2); renumbering them so that each XCD
// runs one contiguous range of the logical order keeps neighbouring tiles,
// which share halo rows, in one L2.
#ifndef SG_XCD_REMAP
#define SG_XCD_REMAP 1
#endif
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t logical_group() {
#if SG_XCD_REMAP
  const uint32_t G = gridDim.x, g = blockIdx.x;
  const uint32_t q = G / kXcds, rm = G % kXcds, x = g % kXcds;
  return x * q + (x < rm ? x : rm) + g / kXcds;
#else
  return blockIdx.x;
#endif
}

// Inverse of lambda_decode: the linear omega of the fractal block (bx, by)
// (build frame, bx & by == 0).  In the paper frame, bit mu-1 of
// (lambda_x, lambda_y) is (Delta^x_mu, Delta^y_mu), so the region index at
// level mu is beta = Delta^x + Delta^y (Eq. 5 read backwards); it is the
// digit of omega_y (odd mu) or omega_x (even mu) of weight
// 3^(ceil(mu/2)-1) (Eq. 4), and omega = omega_y * 3^floor(rb/2) + omega_x.
__device__ __forceinline__ uint32_t lambda_encode(uint32_t bx, uint32_t by, int rb) {
  const uint32_t ly = by ^ ((1u << rb) - 1u);
  const int hx = rb >> 1;
  uint32_t wx = 0, wy = 0, px = 1, py = 1;
  for (int mu = 1; mu <= rb; ++mu) {
    const uint32_t beta = ((bx >> (mu - 1)) & 1u) + ((ly >> (mu - 1)) & 1u);
    if (mu & 1) {
      wy += beta * py;
      py *= 3u;
    } else {
      wx += beta * px;
      px *= 3u;
    }
  }
  uint32_t W = 1;
  for (int j = 0; j < hx; ++j) W *= 3u;
  return wy * W + wx;
}

// Lane i receives lane i-1's value (DPP wave_shr:1); lane 0 receives 0.
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
// Lane i receives lane i+1's value (DPP wave_shl:1); lane 63 receives 0.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_prev_lane(float v) {
  return __uint_as_float(from_prev_lane(__float_as_uint(v)));
}
__device__ __forceinline__ float from_next_lane(float v) {
  return __uint_as_float(from_next_lane(__float_as_uint(v)));
}

// ---------------------------------------------------------------- u8 rows
//
// A row of RHO bytes lives in NW 32-bit words, little-endian: byte i of the
// row is byte (i & 3) of word i >> 2.  For RHO < 4 only the low RHO bytes of
// word 0 are meaningful and the loads zero-extend.

template <int RHO>
struct U8Row {
  static constexpr int NW = RHO >= 4 ? RHO / 4 : 1;
  uint32_t w[NW];
};

template <int RHO>
__device__ __forceinline__ void load_row(U8Row<RHO> &row, const uint8_t *p) {
  if constexpr (RHO == 1) {
    row.w[0] = p[0];
  } else if constexpr (RHO == 2) {
    row.w[0] = *reinterpret_cast<const uint16_t *>(p);
  } else if constexpr (RHO == 4) {
    row.w[0] = *reinterpret_cast<const uint32_t *>(p);
  } else if constexpr (RHO == 8) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    row.w[0] = v.x;
    row.w[1] = v.y;
  } else {
#pragma unroll
    for (int k = 0; k < RHO / 16; ++k) {
      const uint4 v = reinterpret_cast<const uint4 *>(p)[k];
      row.w[4 * k + 0] = v.x;
      row.w[4 * k + 1] = v.y;
      row.w[4 * k + 2] = v.z;
      row.w[4 * k + 3] = v.w;
    }
  }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Stores a row of a tile.  STREAM: non-temporal stores, for passes that read
// the previous state and write the next one, so the written lines do not
// take cache space from the reads (neighbouring tiles share the read halo
// rows); the write pass, which only writes, keeps ordinary stores.
template <int RHO, bool STREAM = false>
__device__ __forceinline__ void store_row(uint8_t *p, const U8Row<RHO> &row) {
  if constexpr (RHO == 1) {
    p[0] = (uint8_t)row.w[0];
  } else if constexpr (RHO == 2) {
    *reinterpret_cast<uint16_t *>(p) = (uint16_t)row.w[0];
  } else if constexpr (RHO == 4) {
    if constexpr (STREAM)
      __builtin_nontemporal_store(row.w[0], reinterpret_cast<uint32_t *>(p));
    else
      *reinterpret_cast<uint32_t *>(p) = row.w[0];
  } else if constexpr (RHO == 8) {
    if constexpr (STREAM) {
      const u32x2 v = {row.w[0], row.w[1]};
      __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(p));
    } else {
      *reinterpret_cast<uint2 *>(p) = make_uint2(row.w[0], row.w[1]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < RHO / 16; ++k) {
      if constexpr (STREAM) {
        const u32x4 v = {row.w[4 * k], row.w[4 * k + 1], row.w[4 * k + 2], row.w[4 * k + 3]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p) + k);
      } else {
        reinterpret_cast<uint4 *>(p)[k] =
            make_uint4(row.w[4 * k], row.w[4 * k + 1], row.w[4 * k + 2], row.w[4 * k + 3]);
      }
    }
  }
}

template <int RHO>
__device__ __forceinline__ void zero_row(U8Row<RHO> &row) {
#pragma unroll
  for (int k = 0; k < U8Row<RHO>::NW; ++k) row.w[k] = 0u;
}

// Bounding sub-box test for a whole tile row (Section III-D): byte i of word
// set to 1 iff (i & ty) == 0, i.e. cell (X0 + i, Y0 + ty) of a fractal tile
// lies on the gasket (X0 & Y0 == 0 and both are multiples of rho).
template <int RHO>
__device__ __forceinline__ uint32_t row_mask_word(int k, uint32_t ty) {
  uint32_t m = 0x01010101u;
  if (ty & 1u) m &= 0x00010001u;
  if (ty & 2u) m &= 0x00000101u;
  if (((uint32_t)k << 2) & ty) m = 0u;
  if constexpr (RHO < 4) m &= (1u << (8 * RHO)) - 1u;
  return m;
}

// One explicit diffusion update of a cell (FP32): with deg the number of the
// cell's in-grid gasket neighbours, u + alpha * sum_nb (u_nb - u) is taken as
//   t = (w + e) + (nn + ss) - deg * u   (one fma),   out = u + alpha * t,
// which relies on every neighbour off the grid or off the gasket holding 0
// (the state invariant); a cell off the gasket is 0.  Every diffusion kernel
// goes through this function with its neighbours' values and deg, so they
// agree bit for bit.
__device__ __forceinline__ float diffuse_cell(float u, float w, float e, float nn, float ss,
                                              float deg, bool self, float alpha) {
  const float t = __builtin_fmaf(-deg, u, (w + e) + (nn + ss));
  return self ? __builtin_fmaf(alpha, t, u) : 0.0f;
}
__device__ __forceinline__ float diffuse_cell(float u, float w, float e, float nn, float ss,
                                              bool mw, bool me, bool mn, bool ms, bool self,
                                              float alpha) {
  return diffuse_cell(u, w, e, nn, ss, (float)((int)mw + (int)me + (int)mn + (int)ms), self,
                      alpha);
}

}  // namespace sg
