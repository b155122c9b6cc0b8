// Other embedded fractals F^{k,s} with s = 1/m (Section III-A), and the
// block-space map generalised to them (Section V): the fractal keeps k of the
// m x m sub-squares at every scale, given by their offsets (the motif).  The
// map's helper function is the base-k digit of omega at each scale level, its
// offset function is the motif entry of that digit and its weight is
// m^(mu-1) -- with m = 2, k = 3 and the gasket's motif this is lambda.
//
// One workgroup runs TPG tiles of rho x rho cells (rho = m^q), one thread per
// cell in a strided loop: consecutive threads take consecutive cells of a
// tile row, so row accesses coalesce.  The tiles of a workgroup are decoded
// once, into LDS.  Inside a fractal tile a cell is on the fractal iff its q
// local digit pairs are kept offsets (the bounding sub-box test of
// Section III-D, generalised); cells off the fractal hold 0.
#include "../../include/sg.h"
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

constexpr int kFracThreads = 256;

// The motif as kernel arguments: offsets packed 2 bits per entry (m <= 4).
struct FracArgs {
  uint32_t k;     // kept sub-squares
  uint32_t kept;  // bit dx + m * dy set for every kept offset
  uint32_t dxw;   // dx of entry i at bits 2i, 2i+1
  uint32_t dyw;
};

template <int M>
__device__ __forceinline__ bool kept_digits(const FracArgs &f, uint32_t x, uint32_t y,
                                            int levels) {
  bool ok = true;
  for (int j = 0; j < levels; ++j) {
    const uint32_t qx = x / M, qy = y / M;
    ok &= (f.kept >> ((x - qx * M) + M * (y - qy * M))) & 1u;
    x = qx;
    y = qy;
  }
  return ok;
}

// Level-order decode (the pass kernels' numbering of the launch grid): digit
// j of t in base k is the motif entry of scale level j + 1.
template <int M>
__device__ __forceinline__ void frac_decode_levels(const FracArgs &f, uint32_t t, int rb,
                                                   uint32_t &bx, uint32_t &by) {
  uint32_t px = 0, py = 0, w = 1;
  for (int j = 0; j < rb; ++j) {
    const uint32_t q = t / f.k;
    const uint32_t d = t - q * f.k;
    t = q;
    px += ((f.dxw >> (2 * d)) & 3u) * w;
    py += ((f.dyw >> (2 * d)) & 3u) * w;
    w *= M;
  }
  bx = px;
  by = py;
}

// Canonical table: omega = omega_y * W + omega_x (W = k^floor(rb/2)); odd
// levels take their digit from omega_y, even levels from omega_x (Eq. 4).
template <int M>
__global__ __launch_bounds__(kWG) void k_frac_map(FracArgs f, int rb, uint32_t W, uint32_t count,
                                                  uint2 *__restrict__ out) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  uint32_t wx = i % W, wy = i / W;
  uint32_t px = 0, py = 0, w = 1;
  for (int mu = 1; mu <= rb; ++mu) {
    uint32_t d;
    if (mu & 1) {
      d = wy % f.k;
      wy /= f.k;
    } else {
      d = wx % f.k;
      wx /= f.k;
    }
    px += ((f.dxw >> (2 * d)) & 3u) * w;
    py += ((f.dyw >> (2 * d)) & 3u) * w;
    w *= M;
  }
  out[i] = make_uint2(px, py);
}

// Tile of workgroup slot s: lambda (all fractal) or the bounding box
// (identity over nb x nb blocks, kept iff the block is a fractal block).
template <int M, bool LAMBDA>
__device__ __forceinline__ bool frac_tile(const FracArgs &f, uint64_t t, uint64_t ntiles, int rb,
                                          uint32_t nb, uint32_t &bx, uint32_t &by) {
  if (t >= ntiles) return false;
  if constexpr (LAMBDA) {
    frac_decode_levels<M>(f, (uint32_t)t, rb, bx, by);
    return true;
  } else {
    // t < nb^2 <= 2^36: quotient by a double division, then one correction
    uint64_t q = (uint64_t)((double)t / (double)nb);
    int64_t rem = (int64_t)(t - q * nb);
    if (rem < 0) {
      --q;
      rem += nb;
    } else if (rem >= (int64_t)nb) {
      ++q;
      rem -= nb;
    }
    by = (uint32_t)q;
    bx = (uint32_t)rem;
    return kept_digits<M>(f, bx, by, rb);
  }
}

struct FracPass {
  int r, q, rb;       // n = M^r, rho = M^q, rb = r - q
  uint32_t n, rho, nb;
  int tpg;            // tiles per workgroup
  uint64_t ntiles;
};

// In-tile membership as bit rows: bit tx of word wd of row ty (tx = 32 wd +
// bit) is set iff cell (tx, ty) of a fractal tile is on the fractal.  Built
// once per workgroup from level masks: L[j][d] holds the columns whose level-j
// digit forms a kept offset with row digit d, and row ty is the AND over the
// levels j of L[j][digit_j(ty)] (membership is a product over levels).
constexpr int kMaskWords = (SG_FRAC_MAX_RHO + 31) / 32;
// Tiles at least this wide are written a word at a time (the bit rows pay for
// themselves); smaller ones a cell at a time.
constexpr uint32_t kWordTileMin = 64;

// Level masks: L[j][d] (kMaskWords words) holds the tile columns whose
// level-j digit forms a kept offset with row digit d.  A thread builds one
// word, walking its 32 columns with a running digit (the level-j digit of
// column c steps every m^j columns).
template <int M, int NT = kFracThreads>
__device__ __forceinline__ void build_level_masks(const FracArgs &f, int q, uint32_t rho,
                                                  uint32_t *L) {
  const int nw = (int)(rho + 31) / 32;  // words a row needs
  for (int e = threadIdx.x; e < q * M * nw; e += NT) {
    const int wd = e % nw, d = (e / nw) % M, j = e / (nw * M);
    uint32_t span = 1;  // columns per level-j digit
    for (int l = 0; l < j; ++l) span *= M;
    const uint32_t c0 = 32u * (uint32_t)wd;
    uint32_t dig = (c0 / span) % M, rem = c0 % span;
    const int bits = (int)rho - (int)c0 < 32 ? (int)rho - (int)c0 : 32;
    uint32_t w = 0;
    for (int b = 0; b < bits; ++b) {
      w |= ((f.kept >> (dig + M * d)) & 1u) << b;
      if (++rem == span) {
        rem = 0;
        dig = dig + 1 == (uint32_t)M ? 0u : dig + 1;
      }
    }
    L[(j * M + d) * kMaskWords + wd] = w;
  }
}

// Membership bits of tile row ty, word wd: the AND over levels j of
// L[j][digit_j(ty)].
template <int M>
__device__ __forceinline__ uint32_t row_mask_word(const uint32_t *L, int q, uint32_t ty,
                                                  uint32_t wd) {
  uint32_t w = ~0u, v = ty;
  for (int j = 0; j < q; ++j) {
    const uint32_t d = v % M;
    v /= M;
    w &= L[(j * M + d) * kMaskWords + wd];
  }
  return w;
}

template <int M>
__device__ __forceinline__ void build_row_masks(const FracArgs &f, int q, uint32_t rho,
                                                uint32_t *L, uint32_t *rows) {
  const int nw = (int)(rho + 31) / 32;
  build_level_masks<M>(f, q, rho, L);
  __syncthreads();
  for (int e = threadIdx.x; e < (int)rho * kMaskWords; e += kFracThreads) {
    const uint32_t ty = e / kMaskWords, wd = e - ty * kMaskWords;
    rows[e] = (int)wd < nw ? row_mask_word<M>(L, q, ty, wd) : 0u;
  }
}

// Bits [b, b + 4) of a bit row (b may be negative or run past the row: those
// bits read as 0).
__device__ __forceinline__ uint32_t row_bits4(const uint32_t *row, int b) {
  const int b0 = b + 32;  // the row is read with one zero word before it
  const uint32_t wi = (uint32_t)b0 >> 5, sh = (uint32_t)b0 & 31u;
  const uint32_t lo = wi >= 1 && wi <= (uint32_t)kMaskWords ? row[wi - 1] : 0u;
  const uint32_t hi = wi + 1 >= 1 && wi < (uint32_t)kMaskWords ? row[wi] : 0u;
  return __builtin_amdgcn_alignbit(hi, lo, sh) & 15u;
}

// Small tiles: one thread per cell, membership from the local digits.
template <int M, bool LAMBDA>
__global__ __launch_bounds__(kFracThreads) void k_frac_write_cells(FracArgs f, FracPass p,
                                                                   uint64_t tile_base,
                                                                   uint8_t *__restrict__ a,
                                                                   uint32_t value) {
  __shared__ uint32_t sbx[kFracThreads], sby[kFracThreads];
  __shared__ uint8_t sok[kFracThreads];
  const int tid = threadIdx.x;
  const uint64_t t0 = tile_base + (uint64_t)logical_group() * p.tpg;
  if (tid < p.tpg) {
    uint32_t bx = 0, by = 0;
    sok[tid] = frac_tile<M, LAMBDA>(f, t0 + tid, p.ntiles, p.rb, p.nb, bx, by);
    sbx[tid] = bx;
    sby[tid] = by;
  }
  __syncthreads();
  const uint32_t cells = p.rho * p.rho;
  for (uint32_t e = tid; e < (uint32_t)p.tpg * cells; e += kFracThreads) {
    const uint32_t s = e / cells, c = e - s * cells;
    if (!sok[s]) continue;
    const uint32_t ty = c / p.rho, tx = c - ty * p.rho;
    const size_t y = (size_t)sby[s] * p.rho + ty, x = (size_t)sbx[s] * p.rho + tx;
    a[y * p.n + x] = kept_digits<M>(f, tx, ty, p.q) ? (uint8_t)value : (uint8_t)0;
  }
}

// Tiles of kWordTileMin cells a side or more: one thread per 4-byte-aligned
// word of a tile row: whole words are stored as
// one 32-bit store, the words at the row's two ends byte by byte.
template <int M, bool LAMBDA>
__global__ __launch_bounds__(kFracThreads) void k_frac_write(FracArgs f, FracPass p,
                                                             uint64_t tile_base,
                                                             uint8_t *__restrict__ a,
                                                             uint32_t value) {
  __shared__ uint32_t sbx[kFracThreads], sby[kFracThreads];
  __shared__ uint8_t sok[kFracThreads];
  __shared__ uint32_t L[160];  // levels x m x words: at most 7 x 2, 5 x 3 or 3 x 4 x 8
  __shared__ uint32_t rows[SG_FRAC_MAX_RHO * kMaskWords];
  const int tid = threadIdx.x;
  const uint64_t t0 = tile_base + (uint64_t)logical_group() * p.tpg;
  if (tid < p.tpg) {
    uint32_t bx = 0, by = 0;
    sok[tid] = frac_tile<M, LAMBDA>(f, t0 + tid, p.ntiles, p.rb, p.nb, bx, by);
    sbx[tid] = bx;
    sby[tid] = by;
  }
  build_row_masks<M>(f, p.q, p.rho, L, rows);
  __syncthreads();
  const uint32_t wpr = (p.rho + 3) / 4 + 1;  // aligned words a tile row can touch
  const uint32_t per_tile = p.rho * wpr;
  for (uint32_t e = tid; e < (uint32_t)p.tpg * per_tile; e += kFracThreads) {
    const uint32_t s = e / per_tile, c = e - s * per_tile;
    if (!sok[s]) continue;
    const uint32_t ty = c / wpr, k = c - ty * wpr;
    const size_t y = (size_t)sby[s] * p.rho + ty;
    uint8_t *row0 = a + y * p.n + (size_t)sbx[s] * p.rho;  // the tile row's first cell
    // k-th 4-byte-aligned word touching the tile row, and the tile column of
    // its first byte (-3..rho)
    uint8_t *dst = reinterpret_cast<uint8_t *>(((uintptr_t)row0 & ~(uintptr_t)3) + 4 * k);
    const int tx0 = (int)(dst - row0);
    if (tx0 >= (int)p.rho) continue;
    const uint32_t bits = row_bits4(rows + ty * kMaskWords, tx0);
    const uint32_t bytes = ((bits * 0x00204081u) & 0x01010101u) * value;
    if (tx0 >= 0 && tx0 + 4 <= (int)p.rho) {
      *reinterpret_cast<uint32_t *>(dst) = bytes;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (tx0 + i >= 0 && tx0 + i < (int)p.rho) dst[i] = (uint8_t)(bytes >> (8 * i));
    }
  }
}

template <int M, bool LAMBDA>
__global__ __launch_bounds__(kFracThreads) void k_frac_life(FracArgs f, FracPass p,
                                                            uint64_t tile_base,
                                                            const uint8_t *__restrict__ in,
                                                            uint8_t *__restrict__ out) {
  extern __shared__ uint8_t reg[];  // tpg regions of (rho + 2)^2 cells
  __shared__ uint32_t sbx[kFracThreads], sby[kFracThreads];
  __shared__ uint8_t sok[kFracThreads];
  const int tid = threadIdx.x;
  const uint64_t t0 = tile_base + (uint64_t)logical_group() * p.tpg;
  if (tid < p.tpg) {
    uint32_t bx = 0, by = 0;
    sok[tid] = frac_tile<M, LAMBDA>(f, t0 + tid, p.ntiles, p.rb, p.nb, bx, by);
    sbx[tid] = bx;
    sby[tid] = by;
  }
  __syncthreads();
  // tile plus a one-cell halo; cells off the grid read 0 (cells off the
  // fractal hold 0, so they add nothing to a count)
  const uint32_t side = p.rho + 2, rcells = side * side;
  for (uint32_t e = tid; e < (uint32_t)p.tpg * rcells; e += kFracThreads) {
    const uint32_t s = e / rcells, c = e - s * rcells;
    uint8_t v = 0;
    if (sok[s]) {
      const uint32_t i = c / side, j = c - i * side;
      const int64_t y = (int64_t)sby[s] * p.rho + i - 1, x = (int64_t)sbx[s] * p.rho + j - 1;
      if (y >= 0 && y < p.n && x >= 0 && x < p.n) v = in[(size_t)y * p.n + (size_t)x];
    }
    reg[e] = v;
  }
  __syncthreads();
  const uint32_t cells = p.rho * p.rho;
  for (uint32_t e = tid; e < (uint32_t)p.tpg * cells; e += kFracThreads) {
    const uint32_t s = e / cells, c = e - s * cells;
    if (!sok[s]) continue;
    const uint32_t ty = c / p.rho, tx = c - ty * p.rho;
    const uint8_t *g = reg + s * rcells + (ty + 1) * side + (tx + 1);
    const uint32_t cnt = g[-(int)side - 1] + g[-(int)side] + g[-(int)side + 1] + g[-1] + g[1] +
                         g[side - 1] + g[side] + g[side + 1];
    const bool alive = cnt == 3u || (g[0] != 0 && cnt == 2u);
    const size_t y = (size_t)sby[s] * p.rho + ty, x = (size_t)sbx[s] * p.rho + tx;
    out[y * p.n + x] = (alive && kept_digits<M>(f, tx, ty, p.q)) ? 1 : 0;
  }
}

// Life step on tiles of kWordTileMin cells a side or more (one tile per
// workgroup).  The tile and a one-cell halo are staged in LDS as rows of
// words, word k of a row holding tile columns 4k - 4 .. 4k - 1.  Rows of the
// embedding (n = m^r bytes) start at every alignment mod 4, so a region row
// is read as 4-byte-aligned words, lane k of a row's lane group holding the
// k-th one and taking the next lane's through a wave shift to realign them
// (tiles at the grid's edge read bytes, with bounds checks).  Then lane k of
// an output row's lane group takes tile columns 4k .. 4k + 3 as one word
// from three LDS rows (SWAR on bytes: 3-row column sums, neighbour bytes by
// funnel shifts, B3/S23 as (count | self) == 3), masks them with the in-tile
// membership bits and realigns the results the other way into aligned output
// words: whole words inside the tile are one store, the words at its two
// ends are written byte by byte.
__host__ __device__ constexpr uint32_t life_row_words(uint32_t rho) {
  return (rho + 3u) / 4u + 2u;  // tile words + a halo word each side
}

static_assert(life_row_words(SG_FRAC_MAX_RHO) + 1 <= 64, "a region row's lane group fits a wave");

__device__ __forceinline__ uint32_t lane_next(uint32_t v) {  // lane i <- lane i + 1
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t lane_prev(uint32_t v) {  // lane i <- lane i - 1
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
}

template <int M, bool LAMBDA, int NT>
__global__ __launch_bounds__(NT) void k_frac_life_words(FracArgs f, FracPass p,
                                                                  uint64_t tile_base,
                                                                  const uint8_t *__restrict__ in,
                                                                  uint8_t *__restrict__ out) {
  extern __shared__ __align__(16) uint32_t regw[];  // rho + 2 rows of life_row_words words
  __shared__ uint32_t L[160];
  __shared__ uint32_t tile_xy[2];
  __shared__ uint8_t tile_ok;
  constexpr int NW = NT / 64;  // waves per workgroup
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = __lane_id();
  const uint64_t t = tile_base + logical_group();
  if (tid == 0) {
    uint32_t bx = 0, by = 0;
    tile_ok = frac_tile<M, LAMBDA>(f, t, p.ntiles, p.rb, p.nb, bx, by);
    tile_xy[0] = bx;
    tile_xy[1] = by;
  }
  build_level_masks<M, NT>(f, p.q, p.rho, L);
  __syncthreads();
  if (!tile_ok) return;
  const uint32_t rho = p.rho, n = p.n;
  const uint32_t SW = life_row_words(rho), wpr = (rho + 3u) / 4u;
  const int64_t X0 = (int64_t)tile_xy[0] * rho, Y0 = (int64_t)tile_xy[1] * rho;

  // 1. stage region rows i = 0 .. rho + 1 (y = Y0 - 1 + i): lane group g of
  //    a wave takes rows, lane k of it LDS word k (the group's last lane only
  //    supplies its aligned word to the one before it)
  {
    const uint32_t GL = SW + 1u, GPW = 64u / GL;  // lanes per group, groups per wave
    const uint32_t g = (uint32_t)lane / GL, k = (uint32_t)lane - g * GL;
    const bool interior = X0 >= 8 && X0 + 4 * (int64_t)SW + 4 <= (int64_t)n && Y0 >= 1 &&
                          Y0 + rho + 1 <= (int64_t)n;
    const uint32_t rows_per_round = GPW * NW;
    if (interior) {
      // kBatch rows per lane in flight at once: their aligned words loaded
      // first, then realigned (wave shift + funnel shift) and stored
      constexpr int kBatch = 8;
      for (uint32_t i0 = 0; i0 < rho + 2u; i0 += kBatch * rows_per_round) {
        uint32_t v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const uint32_t i = i0 + (uint32_t)u * rows_per_round + (uint32_t)wave * GPW + g;
          const bool mine = g < GPW && i < rho + 2u;
          // aligned word k of the row from the byte of tile column -4 on
          const uint64_t base = (uint64_t)(Y0 - 1 + (int64_t)i) * n + (uint64_t)(X0 - 4);
          v[u] = mine ? *reinterpret_cast<const uint32_t *>(in + (base & ~3ull) + 4ull * k) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const uint32_t i = i0 + (uint32_t)u * rows_per_round + (uint32_t)wave * GPW + g;
          const bool mine = g < GPW && i < rho + 2u;
          const uint64_t base = (uint64_t)(Y0 - 1 + (int64_t)i) * n + (uint64_t)(X0 - 4);
          const uint32_t word =
              __builtin_amdgcn_alignbit(lane_next(v[u]), v[u], (uint32_t)(base & 3u) * 8u);
          if (mine && k < SW) regw[i * SW + k] = word;
        }
      }
    } else {
      for (uint32_t i0 = 0; i0 < rho + 2u; i0 += rows_per_round) {
        const uint32_t i = i0 + (uint32_t)wave * GPW + g;
        const int64_t y = Y0 - 1 + (int64_t)i;
        if (!(g < GPW && i < rho + 2u && k < SW)) continue;
        uint32_t word = 0u;
        if (y >= 0 && y < (int64_t)n) {
          const int64_t x0 = X0 - 4 + 4 * (int64_t)k;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t x = x0 + b;
            if (x >= 0 && x < (int64_t)n)
              word |= (uint32_t)in[(uint64_t)y * n + (uint64_t)x] << (8 * b);
          }
        }
        regw[i * SW + k] = word;
      }
    }
  }
  __syncthreads();

  // 2. tile rows ty: lane k of a group takes tile columns 4k .. 4k + 3 (k <
  //    wpr), and output word k of the row (k <= wpr)
  const uint32_t GL = wpr + 1u, GPW = 64u / GL;
  const uint32_t g = (uint32_t)lane / GL, k = (uint32_t)lane - g * GL;
  const uint32_t rows_per_round = GPW * NW;
  for (uint32_t t0 = 0; t0 < rho; t0 += rows_per_round) {
    const uint32_t ty = t0 + (uint32_t)wave * GPW + g;
    const bool mine = g < GPW && ty < rho;
    uint32_t alive = 0u;
    if (mine && k < wpr) {
      const uint32_t *r0 = regw + ty * SW + k + 1u;  // row above; word k + 1 = columns 4k ..
      const uint32_t *r1 = r0 + SW, *r2 = r1 + SW;
      const uint32_t C = r1[0];
      const uint32_t V = r0[0] + C + r2[0];
      const uint32_t Vp = r0[-1] + r1[-1] + r2[-1];
      const uint32_t Vn = r0[1] + r1[1] + r2[1];
      const uint32_t Lb = __builtin_amdgcn_alignbit(V, Vp, 24);  // byte i <- column 4k + i - 1
      const uint32_t Rb = __builtin_amdgcn_alignbit(Vn, V, 8);   // byte i <- column 4k + i + 1
      const uint32_t cnt = Lb + V + Rb - C;                      // live neighbours, per byte
      const uint32_t x = (cnt | C) ^ 0x03030303u;
      uint32_t z = x | (x >> 1);
      z |= z >> 2;
      const uint32_t m = row_mask_word<M>(L, p.q, ty, (4u * k) >> 5);
      const uint32_t bits = (m >> ((4u * k) & 31u)) & 15u;
      alive = ~z & ((bits * 0x00204081u) & 0x01010101u);
    }
    // output word k covers tile columns 4k - d .. 4k - d + 3, d the row's
    // first cell's offset in its aligned word
    const uint64_t row0 = (uint64_t)(Y0 + ty) * n + (uint64_t)X0;
    const uint32_t d = (uint32_t)(row0 & 3u);
    const uint32_t before = lane_prev(alive);  // all lanes
    if (!mine) continue;
    const uint32_t w = d == 0u ? alive : __builtin_amdgcn_alignbit(alive, before, 32u - 8u * d);
    const int tx0 = 4 * (int)k - (int)d;
    uint8_t *dst = out + (row0 & ~3ull) + 4ull * k;
    if (tx0 >= 0 && tx0 + 4 <= (int)rho) {
      *reinterpret_cast<uint32_t *>(dst) = w;
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (tx0 + b >= 0 && tx0 + b < (int)rho) dst[b] = (uint8_t)(w >> (8 * b));
    }
  }
}

// Life tiles this wide run 512 threads: their region (about 62 KB of LDS at
// rho = 243) leaves room for two workgroups per CU.
#ifndef SG_FRAC_WIDE_LIFE_TILE
#define SG_FRAC_WIDE_LIFE_TILE 128
#endif
constexpr uint32_t kWideLifeTile = SG_FRAC_WIDE_LIFE_TILE;

constexpr uint64_t kFracMaxGroups = 1ull << 22;

template <int M, bool LAMBDA, bool LIFE>
hipError_t frac_pass_m(const FracArgs &f, const FracPass &p, hipStream_t s, uint8_t *a,
                       const uint8_t *in, uint32_t value) {
  const uint64_t groups = (p.ntiles + p.tpg - 1) / p.tpg;
  const bool words = p.rho >= kWordTileMin;
  const size_t lds = !LIFE ? 0
                     : words ? (size_t)(p.rho + 2) * life_row_words(p.rho) * sizeof(uint32_t)
                             : (size_t)p.tpg * (p.rho + 2) * (p.rho + 2);
  for (uint64_t g0 = 0; g0 < groups; g0 += kFracMaxGroups) {
    const uint64_t g = groups - g0 < kFracMaxGroups ? groups - g0 : kFracMaxGroups;
    if (LIFE && words && p.rho >= kWideLifeTile)
      hipLaunchKernelGGL((k_frac_life_words<M, LAMBDA, 2 * kFracThreads>), dim3((unsigned)g),
                         dim3(2 * kFracThreads), lds, s, f, p, g0 * (uint64_t)p.tpg, in, a);
    else if (LIFE && words)
      hipLaunchKernelGGL((k_frac_life_words<M, LAMBDA, kFracThreads>), dim3((unsigned)g),
                         dim3(kFracThreads), lds, s, f, p, g0 * (uint64_t)p.tpg, in, a);
    else if (LIFE)
      hipLaunchKernelGGL((k_frac_life<M, LAMBDA>), dim3((unsigned)g), dim3(kFracThreads), lds, s,
                         f, p, g0 * (uint64_t)p.tpg, in, a);
    else if (p.rho >= kWordTileMin)
      hipLaunchKernelGGL((k_frac_write<M, LAMBDA>), dim3((unsigned)g), dim3(kFracThreads), 0, s,
                         f, p, g0 * (uint64_t)p.tpg, a, value);
    else
      hipLaunchKernelGGL((k_frac_write_cells<M, LAMBDA>), dim3((unsigned)g), dim3(kFracThreads),
                         0, s, f, p, g0 * (uint64_t)p.tpg, a, value);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool LIFE>
hipError_t frac_pass(int m, bool lambda, const FracArgs &f, const FracPass &p, hipStream_t s,
                     uint8_t *a, const uint8_t *in, uint32_t value) {
  switch (m) {
    case 2: return lambda ? frac_pass_m<2, true, LIFE>(f, p, s, a, in, value)
                          : frac_pass_m<2, false, LIFE>(f, p, s, a, in, value);
    case 3: return lambda ? frac_pass_m<3, true, LIFE>(f, p, s, a, in, value)
                          : frac_pass_m<3, false, LIFE>(f, p, s, a, in, value);
    case 4: return lambda ? frac_pass_m<4, true, LIFE>(f, p, s, a, in, value)
                          : frac_pass_m<4, false, LIFE>(f, p, s, a, in, value);
    default: return hipErrorInvalidValue;
  }
}

uint64_t ipow(uint64_t b, int e) {
  uint64_t v = 1;
  while (e-- > 0) v *= b;
  return v;
}

// Validates the motif; fills the kernel arguments.
int frac_args(const sg_fractal *fr, FracArgs &f) {
  if (!fr || fr->m < 2 || fr->m > SG_FRAC_MAX_M || fr->k < 1 || fr->k > fr->m * fr->m ||
      fr->k > SG_FRAC_MAX_K)
    return SG_EINVAL;
  f = FracArgs{(uint32_t)fr->k, 0u, 0u, 0u};
  for (int i = 0; i < fr->k; ++i) {
    if (fr->dx[i] >= fr->m || fr->dy[i] >= fr->m) return SG_EINVAL;
    const uint32_t bit = 1u << (fr->dx[i] + fr->m * fr->dy[i]);
    if (f.kept & bit) return SG_EINVAL;  // repeated offset
    f.kept |= bit;
    f.dxw |= (uint32_t)fr->dx[i] << (2 * i);
    f.dyw |= (uint32_t)fr->dy[i] << (2 * i);
  }
  return SG_OK;
}

// Validates (r, rho, map) for a fractal of subdivision m and fills the pass.
int frac_pass_args(const sg_fractal *fr, int map, int r, int rho, FracPass &p) {
  if (map != SG_MAP_LAMBDA && map != SG_MAP_BBOX) return SG_EINVAL;
  const int m = fr->m;
  if (r < 0 || r > 18 || ipow(m, r) > SG_FRAC_MAX_N) return SG_EINVAL;
  int q = 0;
  uint64_t side = 1;
  while (side < (uint64_t)rho && q <= r) {
    side *= m;
    ++q;
  }
  if (rho < 1 || side != (uint64_t)rho || q > r || rho > SG_FRAC_MAX_RHO) return SG_EINVAL;
  p.r = r;
  p.q = q;
  p.rb = r - q;
  p.n = (uint32_t)ipow(m, r);
  p.rho = (uint32_t)rho;
  p.nb = (uint32_t)ipow(m, p.rb);
  const uint64_t cells = (uint64_t)rho * rho;
  p.tpg = cells >= kFracThreads ? 1 : (int)(kFracThreads / cells);
  p.ntiles = map == SG_MAP_LAMBDA ? ipow(fr->k, p.rb) : (uint64_t)p.nb * p.nb;
  if (map == SG_MAP_LAMBDA && p.ntiles > 0xffffffffull) return SG_EINVAL;  // 32-bit decode
  return SG_OK;
}

}  // namespace
}  // namespace sg

extern "C" {

SG_API int sg_frac_block_count(const sg_fractal *fr, int map, int r, int rho, uint64_t *blocks) {
  sg::FracArgs f;
  sg::FracPass p;
  if (!blocks || sg::frac_args(fr, f) != SG_OK) return SG_EINVAL;
  if (sg::frac_pass_args(fr, map, r, rho, p) != SG_OK) return SG_EINVAL;
  *blocks = p.ntiles;
  return SG_OK;
}

SG_API int sg_frac_map(const sg_fractal *fr, int r, int rho, uint32_t *d_bxy, void *stream) {
  sg::FracArgs f;
  sg::FracPass p;
  if (!d_bxy || ((uintptr_t)d_bxy & 7u) || sg::frac_args(fr, f) != SG_OK) return SG_EINVAL;
  if (sg::frac_pass_args(fr, SG_MAP_LAMBDA, r, rho, p) != SG_OK) return SG_EINVAL;
  if (p.ntiles > 0x7fffffffull) return SG_EINVAL;
  if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
  const uint32_t count = (uint32_t)p.ntiles;
  const uint32_t W = (uint32_t)sg::ipow(fr->k, p.rb / 2);
  const dim3 grid((count + sg::kWG - 1) / sg::kWG);
  hipStream_t s = (hipStream_t)stream;
  switch (fr->m) {
    case 2: hipLaunchKernelGGL(sg::k_frac_map<2>, grid, dim3(sg::kWG), 0, s, f, p.rb, W, count, (uint2 *)d_bxy); break;
    case 3: hipLaunchKernelGGL(sg::k_frac_map<3>, grid, dim3(sg::kWG), 0, s, f, p.rb, W, count, (uint2 *)d_bxy); break;
    default: hipLaunchKernelGGL(sg::k_frac_map<4>, grid, dim3(sg::kWG), 0, s, f, p.rb, W, count, (uint2 *)d_bxy); break;
  }
  return sg::status_of(hipGetLastError());
}

SG_API int sg_frac_write(const sg_fractal *fr, int map, int r, int rho, uint8_t *d_a,
                         uint8_t value, void *stream) {
  sg::FracArgs f;
  sg::FracPass p;
  if (!d_a || sg::frac_args(fr, f) != SG_OK) return SG_EINVAL;
  if (sg::frac_pass_args(fr, map, r, rho, p) != SG_OK) return SG_EINVAL;
  if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
  return sg::status_of(sg::frac_pass<false>(fr->m, map == SG_MAP_LAMBDA, f, p,
                                            (hipStream_t)stream, d_a, nullptr, value));
}

SG_API int sg_frac_life_step(const sg_fractal *fr, int map, int r, int rho,
                             const uint8_t *d_in, uint8_t *d_out, void *stream) {
  sg::FracArgs f;
  sg::FracPass p;
  if (!d_in || !d_out || sg::frac_args(fr, f) != SG_OK) return SG_EINVAL;
  if (sg::frac_pass_args(fr, map, r, rho, p) != SG_OK) return SG_EINVAL;
  const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
  const uintptr_t bytes = (uintptr_t)p.n * p.n;
  if (a < b + bytes && b < a + bytes) return SG_EALIAS;
  if (sg::inject_hip_error()) return sg::status_of(hipErrorLaunchFailure);
  return sg::status_of(sg::frac_pass<true>(fr->m, map == SG_MAP_LAMBDA, f, p,
                                           (hipStream_t)stream, d_out, d_in, 0u));
}

}  // extern "C"
