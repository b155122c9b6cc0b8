// Temporally blocked B3/S23 life on the gasket (gfx950).
//
// One workgroup owns one rho x rho tile of the map (lambda or bounding box)
// and advances it by T generations per pass (T <= 32), so HBM is read and
// written once per T steps instead of once per step.
//
//  1. Load the tile plus a halo of T rows above/below and T cells left/right
//     (one or two 16-byte chunks) from HBM, skipping chunks with no gasket
//     cell, and bit-pack each 16-byte chunk of 0/1 bytes into 16 bits of an
//     LDS plane (one bit per cell, 32 cells per word, the words aligned to
//     multiples of 32 cells).
//  2. List, once, the vertical segments (one 32-cell word column, kSegRows
//     rows) that hold a gasket cell (wavefront ballot + prefix count), and
//     the gasket pattern of every region row (bounding sub-box test
//     x & y == 0 applied to 32 cells at once).
//  3. T times: each listed segment walks down its rows keeping the
//     horizontal 3-cell sums of the rows above, at and below in registers
//     (bit-sliced: lsb and carry planes), so every row's sums are formed once
//     and used for three output rows; the 3 x 3 sum and the B3/S23 rule are
//     evaluated on the bit planes, one v_bitop3 per three-input function,
//     and masked to the gasket.
//     One plane is updated in place: every segment computes its rows into
//     registers, a barrier, then stores them, a barrier (one plane instead of
//     two lets 8 workgroups share a compute unit at rho = 256, so nearly all
//     32 of its wave slots run segments).  Cells outside the region are taken
//     as dead; the wrong values this makes at the region's cut edges move
//     inward one cell per generation and never reach the tile in T
//     generations.
//  4. Unpack the tile and store every 64-byte granule that holds a gasket
//     cell in full.
//
// Between the passes of a multi-pass run the state is bit-packed tiles
// (bit_tile_words): the passes after the first read those words straight
// into the plane instead of step 1's bytes, and the passes before the last
// store the plane's tile words instead of step 4's bytes (k_life_tb_bits,
// k_life_tb_compact_bits).
#include "sg_device.h"
#include "sg_launch.h"

namespace sg {

namespace {

// Workgroup shape; the defaults are the measured best on MI355X and can be
// overridden at build time.
#ifndef SG_TB_THREADS
#define SG_TB_THREADS 0  // 0: 256 threads
#endif
#ifndef SG_TB_SEG_ROWS
#define SG_TB_SEG_ROWS 5
#endif
template <int RHO>
constexpr int tb_threads() {
  return SG_TB_THREADS > 0 ? SG_TB_THREADS : 256;
}
constexpr int kSegRows = SG_TB_SEG_ROWS;      // rows per vertical segment of a generation
// Waves per SIMD the dense, bit and compact tile passes are compiled for
// (at most 64 VGPRs): 8 workgroups of 256 threads per compute unit.
constexpr int kTbWavesPerSimd = 8;

// Plane pitch (words per plane row) for a region W words wide.  Threads that
// run consecutive segments of one word column touch rows kSegRows apart; a
// pitch P with kSegRows * P = 1 (mod 32) puts those words in consecutive LDS
// banks (32 banks of 4 bytes), so a wave's reads are conflict free.
constexpr int plane_pitch(int W) {
  for (int p = W + 2; p < W + 2 + 32; ++p)
    if ((kSegRows * p) % 32 == 1) return p;
  return W + 2;  // no such pitch (even kSegRows): plain row-major
}

constexpr int rho_log2_const(int rho) { return rho <= 1 ? 0 : 1 + rho_log2_const(rho / 2); }

// e / d for d >= 4 and e (d - 1) < 2^20, given m = ceil(2^20 / d): e * m then
// fits 32 bits (and 24-bit operands), and e * m / 2^20 exceeds e / d by at
// most e (d - 1) / (d 2^20) < 1 / d, which never carries it past the next
// integer.
__host__ __device__ constexpr uint32_t div_small_magic(uint32_t d) {
  return ((1u << 20) + d - 1u) / d;
}
__device__ __forceinline__ int div_small(int e, uint32_t m) {
  return (int)(__umul24((uint32_t)e, m) >> 20);
}

// 16 bytes holding 0/1 -> 16 bits (bit i = byte i): each 4-byte word is a
// dot product of its bytes with the weights 1, 2, 4, 8 (or 16..128 for the
// upper nibble of a byte), one v_dot4_u32_u8 each, accumulated in pairs.
__device__ __forceinline__ uint32_t pack16(const uint4 v) {
  const uint32_t lo = __builtin_amdgcn_udot4(
      v.y, 0x80402010u, __builtin_amdgcn_udot4(v.x, 0x08040201u, 0u, false), false);
  const uint32_t hi = __builtin_amdgcn_udot4(
      v.w, 0x80402010u, __builtin_amdgcn_udot4(v.z, 0x08040201u, 0u, false), false);
  return lo | (hi << 8);
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

// Three-input bitwise functions as one v_bitop3 each.  The 8-bit truth table
// of f(a, b, c) is f applied to the constant columns kA, kB, kC (bit
// 4a + 2b + c of the table is f(a, b, c)).
constexpr uint32_t kA = 0xF0u, kB = 0xCCu, kC = 0xAAu;
constexpr uint32_t kXor3 = kA ^ kB ^ kC;
constexpr uint32_t kMaj3 = (kA & kB) | (kA & kC) | (kB & kC);
template <uint32_t F>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, F & 0xFFu);
}

// Horizontal 3-cell sums (west + centre + east) of a row word, as bit planes
// (h0 + 2 * h1), from the word and its west and east neighbour words.
struct RowSums {
  uint32_t h0, h1;
  uint32_t self;  // the centre cells
};

__device__ __forceinline__ RowSums row_sums(uint32_t left, uint32_t mid, uint32_t right) {
  const uint32_t w = __builtin_amdgcn_alignbit(mid, left, 31);  // bit i <- cell x-1
  const uint32_t e = __builtin_amdgcn_alignbit(right, mid, 1);  // bit i <- cell x+1
  return RowSums{bop3<kXor3>(w, mid, e), bop3<kMaj3>(w, mid, e), mid};
}

// B3/S23 for 32 cells from the sums of the rows above (u), at (m) and below
// (d), masked to the gasket cells `mask`.  With S the 3 x 3 sum
// (centre included) a cell lives next iff S == 3, or S == 4 and it is alive.
// Writing S = s0 + 2 (a + k) + 4 b, where (s0, k) are the sum and carry of
// the three lsb planes and (a, b) those of the three msb planes:
//   S == 3  iff  s0 and not b and (a xor k),
//   S == 4  iff  not s0 and ((not b, a, k) or (b, not a, not k)).
__device__ __forceinline__ uint32_t life_rule(const RowSums &u, const RowSums &m,
                                              const RowSums &d, uint32_t mask) {
  const uint32_t s0 = bop3<kXor3>(u.h0, m.h0, d.h0);
  const uint32_t k = bop3<kMaj3>(u.h0, m.h0, d.h0);
  const uint32_t a = bop3<kXor3>(u.h1, m.h1, d.h1);
  const uint32_t b = bop3<kMaj3>(u.h1, m.h1, d.h1);
  const uint32_t e3 = bop3<~kA & (kB ^ kC)>(b, a, k);                         // rest of S == 3
  const uint32_t e4 = bop3<(~kA & kB & kC) | (kA & ~kB & ~kC)>(b, a, k);      // rest of S == 4
  const uint32_t f = bop3<(kA & kB) | (~kA & kC)>(s0, e3, e4);                // s0 ? e3 : e4
  return bop3<kA & (kB | kC)>(f, s0, m.self) & mask;                          // f & (s0 | self)
}

// Work units of a tile pass's region load and store, fixed per tile side.
//
// Inside any block of the gasket's block grid that holds gasket cells, the
// 16-byte chunk c (cells 16c..16c+15 of a row) of the 16-row band q (rows
// 16q..16q+15) holds gasket cells iff (c & q) == 0, in every row of the
// band: x & y = (block bits) | (16c & y) | (lower bits), and 16c & y only
// sees bits 4.. of the row.  A load unit is 64 lanes: 16 rows of one band of
// one of the 3 x 3 blocks around the tile times 4 slots, each slot a live
// (band, chunk) pair of that block inside the pass's region (the tile, its
// halo rows of up to 32 above and below, its halo word each side); so only
// chunks that hold gasket cells are loaded and packed.  A store unit is a
// 64-byte granule g (4 chunks) of a tile band q, live iff (g & (q >> 2)) == 0,
// as 16 rows x 4 chunks.  Whether a neighbour block holds gasket cells, and
// which halo rows a pass of T generations needs, are decided when the pass
// runs.
constexpr int kMaxUnits = 64;
constexpr uint32_t kNoPair = 0xFFu;  // an empty slot (band 15, chunk 15: never live)

struct TileUnits {
  int nload = 0, nstore = 0;
  uint32_t load_pairs[kMaxUnits] = {};  // 4 slots of 8 bits: band << 4 | chunk
  uint32_t load_block[kMaxUnits] = {};  // (dbx + 1) + 3 (dby + 1)
  uint32_t store_pairs[kMaxUnits] = {}; // band << 4 | granule
};

template <int RHO>
constexpr TileUnits make_tile_units() {
  TileUnits t{};
  constexpr int NC = RHO / 16;  // chunk columns and bands per block
  // the tile first, then the halo blocks
  const int order[9][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1},
                           {-1, -1}, {1, -1}, {-1, 1}, {1, 1}};
  for (const auto &o : order) {
    const int dbx = o[0], dby = o[1];
    const int q0 = dby < 0 ? NC - 2 : 0, q1 = dby > 0 ? 2 : NC;  // the region's bands
    const int c0 = dbx < 0 ? NC - 2 : 0, c1 = dbx > 0 ? 2 : NC;  // and chunk columns
    int slot = 0;
    uint32_t word = 0;
    for (int q = q0; q < q1; ++q)
      for (int c = c0; c < c1; ++c) {
        if ((q & c) != 0) continue;
        word |= (uint32_t)((q << 4) | c) << (8 * slot);
        if (++slot == 4) {
          t.load_pairs[t.nload] = word;
          t.load_block[t.nload++] = (uint32_t)((dbx + 1) + 3 * (dby + 1));
          slot = 0;
          word = 0;
        }
      }
    if (slot) {
      for (; slot < 4; ++slot) word |= kNoPair << (8 * slot);
      t.load_pairs[t.nload] = word;
      t.load_block[t.nload++] = (uint32_t)((dbx + 1) + 3 * (dby + 1));
    }
  }
  for (int q = 0; q < NC; ++q)
    for (int g = 0; g < RHO / 64; ++g)
      if ((g & (q >> 2)) == 0) t.store_pairs[t.nstore++] = (uint32_t)((q << 4) | g);
  return t;
}

template <int RHO>
struct TileUnitTable {
  static constexpr TileUnits units = make_tile_units<RHO>();
};
template <int RHO>
__constant__ TileUnits kTileUnits = TileUnitTable<RHO>::units;

// The omegas (lambda_encode) of the 3 x 3 blocks around block (tbx, tby),
// -1 for a block off the grid or off the gasket: threads 0..8 write
// nbr[3 (dy + 1) + dx + 1]; the caller synchronises before reading them.
__device__ __forceinline__ void neighbour_omegas(int tid, uint32_t tbx, uint32_t tby, int rb,
                                                 int32_t *nbr) {
  if (tid < 9) {
    const int x = (int)tbx + tid % 3 - 1, y = (int)tby + tid / 3 - 1;
    const int nb = 1 << rb;
    int32_t w = -1;
    if (x >= 0 && y >= 0 && x < nb && y < nb && (x & y) == 0)
      w = (int32_t)lambda_encode((uint32_t)x, (uint32_t)y, rb);
    nbr[tid] = w;
  }
}

// Where a tile pass reads and writes cells.
//
// DenseMem: the 2^lgn x 2^lgn embedding itself (row y at y << lgn; callers
// pass cells inside the grid).
struct DenseMem {
  const uint8_t *in;
  uint8_t *out;
  int lgn;
  static constexpr bool kCompact = false;
  static constexpr bool kBits = false;
  __device__ __forceinline__ void prepare(int, uint32_t, uint32_t, int) const {}
  __device__ __forceinline__ size_t off(int y, int x) const {
    return ((size_t)(uint32_t)y << lgn) + (uint32_t)x;
  }
  __device__ __forceinline__ const uint8_t *src(int y, int x) const { return in + off(y, x); }
  __device__ __forceinline__ uint8_t *dst(int y, int x) const { return out + off(y, x); }
};

// CompactMem: only the fractal rho x rho tiles, tile omega stored contiguously
// (row-major, rows of rho bytes) at omega * rho^2.  A pass reads the 3 x 3
// tiles around its own, whose omegas (lambda_encode, or -1 off the gasket)
// are found once per workgroup into `nbr` (9 words of LDS).
template <int RHO>
struct CompactMem {
  const uint8_t *in;
  uint8_t *out;
  int32_t *nbr;
  int bx, by;
  static constexpr bool kCompact = true;
  static constexpr bool kBits = false;
  static constexpr int K = rho_log2_const(RHO);
  __device__ __forceinline__ void prepare(int tid, uint32_t tbx, uint32_t tby, int rb) const {
    neighbour_omegas(tid, tbx, tby, rb, nbr);
  }
  __device__ __forceinline__ size_t tile_off(int y, int x) const {
    const int dy = (y >> K) - by + 1, dx = (x >> K) - bx + 1;
    return (size_t)nbr[dy * 3 + dx] * (RHO * RHO) + (size_t)(y & (RHO - 1)) * RHO + (x & (RHO - 1));
  }
  __device__ __forceinline__ const uint8_t *src(int y, int x) const { return in + tile_off(y, x); }
  __device__ __forceinline__ uint8_t *dst(int y, int x) const { return out + tile_off(y, x); }
};

// The region loads of one tile pass, in flight in registers until packed:
// wave w holds the loads of load units w, w + NW, ... (TileUnits).
template <int RHO, int NT>
struct RegionLoads {
  static constexpr bool kBits = false;
  static constexpr int NW = NT / 64;                            // waves per workgroup
  static constexpr int NU = TileUnitTable<RHO>::units.nload;   // load units
  static constexpr int UPW = (NU + NW - 1) / NW;               // load units per wave
  uint4 v[UPW];
  uint32_t live;  // bit k: this lane's slot of unit w + k NW was loaded
};

// Issues the region loads of the tile at block (bx, by) for a pass of T
// generations.  A unit whose block holds no gasket cell (or lies off the
// grid) is skipped by the whole wave; in the others, a lane loads its chunk
// if that chunk lies in the region (the tile, T rows above and below, and
// the halo chunks within T cells of it).  Nothing waits for the loads here.
template <int RHO, int NT, class Mem>
__device__ __forceinline__ void tb_load(const Mem &mem, int r, uint32_t bx, uint32_t by, int T,
                                        RegionLoads<RHO, NT> &ld) {
  using LD = RegionLoads<RHO, NT>;
  constexpr int NC = RHO / 16;      // chunk columns (and bands) per block
  constexpr int CH = RHO / 16 + 4;  // 16-byte chunks per region row
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = __lane_id();
  const int nbk = 1 << (r - rho_log2_const(RHO));  // blocks per grid side
  const int R = RHO + 2 * T, jlo = T > 16 ? 0 : 1;
  const int yr0 = (int)by * RHO - T;  // row of region row 0
  ld.live = 0u;
#pragma unroll
  for (int k = 0; k < LD::UPW; ++k) {
    const int u = wave + k * LD::NW;
    bool ok = false;
    int y = 0, x = 0;
    if (u < LD::NU) {
      const uint32_t blk = kTileUnits<RHO>.load_block[u];
      const int dbx = (int)(blk % 3u) - 1, dby = (int)(blk / 3u) - 1;
      const int Bx = (int)bx + dbx, By = (int)by + dby;
      if (Bx >= 0 && By >= 0 && Bx < nbk && By < nbk && (Bx & By) == 0) {
        const uint32_t pr = (kTileUnits<RHO>.load_pairs[u] >> (8 * (lane & 3))) & 0xFFu;
        const int q = (int)(pr >> 4), c = (int)(pr & 15u);
        y = By * RHO + 16 * q + (lane >> 2);
        x = Bx * RHO + 16 * c;
        const int i = y - yr0;            // region row
        const int jr = dbx * NC + c + 2;  // region chunk column
        ok = pr != kNoPair && (unsigned)i < (unsigned)R && jr >= jlo && jr < CH - jlo;
      }
    }
    // a defined value either way keeps each load in its own registers, so
    // the wave's loads stay in flight together
    ld.v[k] = ok ? *reinterpret_cast<const uint4 *>(mem.src(y, x)) : make_uint4(0u, 0u, 0u, 0u);
    ld.live |= (ok ? 1u : 0u) << k;
  }
}

// A 16-byte store of a pass's output; `stream`: non-temporal (nothing reads
// the output within the pass, and a working set larger than the cache is
// better left to the region reads, whose halos neighbouring tiles share).
__device__ __forceinline__ void store16(uint8_t *p, const uint4 w, bool stream) {
  if (stream) {
    const u32x4 v = {w.x, w.y, w.z, w.w};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
  } else {
    *reinterpret_cast<uint4 *>(p) = w;
  }
}

// Bit-packed tiles: the state between the passes of a multi-pass run, one
// bit per cell, so a pass that neither starts nor ends the run moves a
// quarter of a byte state's 64-byte granules at most.  Tile omega (the
// lambda_encode of its block) is rho^2 / 32 words at omega * rho^2 / 32; in
// it, word column j (cells 32j .. 32j + 31 of a row, bit i = cell 32j + i)
// is rho words at j * rho, row y at + y.  Column-major, so the west and east
// halo words of a region (one word column of a neighbour tile) are one
// contiguous run each, and so are the T-row halos above and below in every
// column.  Bits of cells off the gasket are 0.
template <int RHO>
constexpr size_t bit_tile_words() {
  return (size_t)RHO * RHO / 32;
}

// The region of a pass read from bit-packed tiles, in flight in registers
// until written to the plane.  With C = ceil(T / 4) and GR = rho / 4 + 2C,
// unit u is 4 rows of region word column u / GR: region rows from
// 4 (u % GR) - 4C + T (those in [0, R) are kept), a 16-byte run of one tile
// column.  Thread tid holds units tid, tid + NT, ...
template <int RHO, int NT>
struct BitLoads {
  static constexpr bool kBits = true;
  static constexpr int W = RHO / 32 + 2;                                   // region words per row
  static constexpr int GMAX = RHO / 4 + 2 * ((kMaxStepsPerPass + 3) / 4);  // row groups at T = 32
  static constexpr int UPT = (W * GMAX + NT - 1) / NT;                    // units per thread
  static_assert(W * GMAX * (GMAX - 1) < (1 << 20), "div_small covers u / GR");
  uint4 v[UPT];
  uint32_t live;  // bit k: unit tid + k NT was loaded
};

// Region word column w and row group g of unit u (BitLoads).
__device__ __forceinline__ void bit_unit(int u, int GR, uint32_t gr_magic, int &w, int &g) {
  w = div_small(u, gr_magic);
  g = u - w * GR;
}

// Issues the region loads of a pass of T generations from bit-packed tiles,
// nbr holding the omegas of the 3 x 3 blocks around the tile (-1: no tile,
// its cells are dead).  The region's words are those of the tile, its T rows
// above and below, and one word column each side.
template <int RHO, int NT>
__device__ __forceinline__ void bits_load(const uint32_t *in, const int32_t *nbr, int T,
                                          BitLoads<RHO, NT> &ld) {
  using LD = BitLoads<RHO, NT>;
  constexpr int WT = RHO / 32, GT = RHO / 4;  // words per tile row, row groups per tile column
  const int C = (T + 3) >> 2, GR = GT + 2 * C;
  const uint32_t magic = div_small_magic((uint32_t)GR);
  ld.live = 0u;
#pragma unroll
  for (int k = 0; k < LD::UPT; ++k) {
    const int u = (int)threadIdx.x + k * NT;
    bool ok = false;
    size_t off = 0;
    if (u < LD::W * GR) {
      int w, g;
      bit_unit(u, GR, magic, w, g);
      const int dbx = w == 0 ? -1 : (w == LD::W - 1 ? 1 : 0);
      const int j = w == 0 ? WT - 1 : (w == LD::W - 1 ? 0 : w - 1);  // column in its tile
      const int dby = g < C ? -1 : (g < C + GT ? 0 : 1);
      const int yb = 4 * (g - C) - dby * RHO;  // first row in its tile: 0 .. rho - 4
      const int32_t om = nbr[3 * (dby + 1) + dbx + 1];
      ok = om >= 0;
      off = (size_t)(uint32_t)om * bit_tile_words<RHO>() + (size_t)(j * RHO + yb);
    }
    ld.v[k] = ok ? *reinterpret_cast<const uint4 *>(in + off) : make_uint4(0u, 0u, 0u, 0u);
    ld.live |= (ok ? 1u : 0u) << k;
  }
}

// A pass's output as bit-packed tiles: the workgroup's own tile is
// nbr[4]'s (read at the store, after the workgroup has synchronised).
struct BitsOut {
  uint32_t *out;
  const int32_t *nbr;
  static constexpr bool kBits = true;
};

// One tile pass: the rho x rho tile at block (bx, by) of the gasket of level
// r advanced by T generations, by NT threads, from its region loads `ld`
// (RegionLoads issued by tb_load from the bytes, a compact Mem prepared; or
// BitLoads issued by bits_load) to mem.dst (a byte Mem) or bit-packed tiles
// (BitsOut).  `lds` holds tb_lds_bytes<RHO>(T) bytes (or more); the caller
// synchronises the workgroup before reusing it.  stream_out: store the
// output non-temporally (life_stream_stores).
template <int RHO, int NT, class Mem, class Loads>
__device__ __forceinline__ void tb_tile(const Mem &mem, int r, uint32_t bx, uint32_t by, int T,
                                        uint32_t *lds, uint32_t *nseg_p, const Loads &ld,
                                        bool stream_out) {
  uint32_t &nseg = *nseg_p;
  constexpr int kTbThreads = NT;
  // Region columns [X0-32, X0+RHO+32): the tile plus one 32-cell word each
  // side (a halo of up to 32 cells), word w starting at X0 - 32 + 32w, so
  // every word starts on a multiple of 32 and holds the gasket pattern of
  // its row whenever its first cell is on the gasket.
  constexpr int W = RHO / 32 + 2;     // region words per row
  constexpr int PW = plane_pitch(W);  // plane pitch (at least one zero guard word each side)
  constexpr int L = kSegRows;
  static_assert(L <= 8, "row bits of a segment are kept in 8 bits");
  static_assert(RHO % 32 == 0, "tile rows are whole 32-cell words");
  constexpr int NBMAX = (RHO + 2 * kMaxStepsPerPass + L - 1) / L;  // segment blocks, T = 32
  static_assert((RHO + 2 + L - 1) / L >= 4 && W * NBMAX * (NBMAX - 1) < (1 << 20),
                "div_small covers the segment list's e / NB");
  constexpr int G = RHO >= 64 ? 64 : RHO;  // store granule: 64 bytes, or the whole row
  const int R = RHO + 2 * T;          // region rows
  const int NB = (R + L - 1) / L;     // segment blocks per word column
  const int RP = NB * L;              // region rows rounded up to whole blocks
  const int PR = RP + 2;              // plane rows (zero guard row above, below)
  const int tid = threadIdx.x;

  // n <= 2^20, so cell coordinates (halo included) fit in 32-bit ints
  const int n = 1 << r;
  const int X0 = (int)bx * RHO, Y0 = (int)by * RHO;
  const int yr0 = Y0 - T;  // row of region row 0

  uint32_t *plane0 = lds;
  uint32_t *rowpat = plane0 + PR * PW;  // RP: gasket pattern of each region row
  uint32_t *segs = rowpat + RP;         // W * NB: listed segments

  {
    // the plane cleared, 16 bytes per store (the region loads are in flight)
    constexpr int kAlign = 4;
    const int words = PR * PW, n4 = words / kAlign;
    uint4 *z = reinterpret_cast<uint4 *>(lds);
    for (int i = tid; i < n4; i += kTbThreads) z[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = kAlign * n4 + tid; i < words; i += kTbThreads) lds[i] = 0u;
  }
  for (int i = tid; i < RP; i += kTbThreads) {
    const int y = yr0 + i;
    rowpat[i] = (i < R && y >= 0 && y < n) ? word_pattern((uint32_t)y) : 0u;
  }
  if (tid == 0) nseg = 0u;
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int lane = __lane_id();
  constexpr int NW = kTbThreads / 64;  // waves per workgroup

  // 1. bit-pack the region loads into plane 0 (each load unit's chunk goes
  //    to its region row and chunk column), or write the loaded words of
  //    bit-packed tiles there (the rows of each unit inside the region).
  if constexpr (Loads::kBits) {
    const int C = (T + 3) >> 2, GR = RHO / 4 + 2 * C;
    const uint32_t magic = div_small_magic((uint32_t)GR);
#pragma unroll
    for (int k = 0; k < Loads::UPT; ++k) {
      if (!((ld.live >> k) & 1u)) continue;
      int w, g;
      bit_unit(tid + k * kTbThreads, GR, magic, w, g);
      const int i = T - 4 * C + 4 * g;  // region row of the unit's first row
      const uint32_t v[4] = {ld.v[k].x, ld.v[k].y, ld.v[k].z, ld.v[k].w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((unsigned)(i + q) < (unsigned)R) plane0[(i + q + 1) * PW + w + 1] = v[q];
    }
  } else {
    uint16_t *p0h = reinterpret_cast<uint16_t *>(plane0);
    using LD = RegionLoads<RHO, NT>;
    constexpr int NC = RHO / 16;
#pragma unroll
    for (int k = 0; k < LD::UPW; ++k) {
      if (!((ld.live >> k) & 1u)) continue;
      const int u = wave + k * LD::NW;
      const uint32_t blk = kTileUnits<RHO>.load_block[u];
      const int dbx = (int)(blk % 3u) - 1, dby = (int)(blk / 3u) - 1;
      const uint32_t pr = (kTileUnits<RHO>.load_pairs[u] >> (8 * (lane & 3))) & 0xFFu;
      const int i = dby * RHO + 16 * (int)(pr >> 4) + (lane >> 2) + T;  // region row
      const int jr = dbx * NC + (int)(pr & 15u) + 2;                    // region chunk column
      p0h[((i + 1) * PW + (jr >> 1) + 1) * 2 + (jr & 1)] = (uint16_t)pack16(ld.v[k]);
    }
  }

  // 2. compact list of the segments (word column w, rows [b*L, b*L+L)) that
  //    hold a gasket cell, listed column by column; each entry keeps the rows
  //    whose word starts on the gasket (then its cells are exactly those of
  //    the row's pattern)
  const uint32_t nb_magic = div_small_magic((uint32_t)NB);
  for (int base = 0; base < W * NB; base += kTbThreads) {
    const int e = base + tid;
    uint32_t rows = 0u, code = 0u;
    if (e < W * NB) {
      const int w = div_small(e, nb_magic), b = e - w * NB;
      const int xw = X0 - 32 + 32 * w;
      if (xw >= 0 && xw < n) {
#pragma unroll
        for (int q = 0; q < L; ++q) {
          const int i = b * L + q;
          if (rowpat[i] != 0u && (xw & (yr0 + i)) == 0) rows |= 1u << q;
        }
      }
      code = (uint32_t)w | ((uint32_t)b << 8) | (rows << 16);
    }
    const uint64_t ball = __ballot(rows != 0u);
    const uint32_t before = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    uint32_t off = 0u;
    if (lane == 0 && ball != 0ull) off = atomicAdd(&nseg, (uint32_t)__popcll(ball));
    off = __shfl(off, 0);
    if (rows != 0u) segs[off + before] = code;
  }
  __syncthreads();
  const int ns = (int)nseg;

  // 3. T generations in LDS.  Thread tid owns segments tid, tid + NT, ... of
  //    the list for the whole pass; their plane index, the gasket mask of each
  //    row (the row's pattern where the word starts on the gasket, else 0) and
  //    the number of generations that need them are found once, into
  //    registers.  Generation s needs the cells that can still reach the tile
  //    in the T-s-1 generations left: region rows [s+1, R-s-1), and the halo
  //    words only while T-s-1 >= 1; so a segment of rows [i0, i0+L) is needed
  //    while s < min(i0 + L - 1, R - 1 - i0, T, or T - 1 for a halo word).
  constexpr int KSEG = (W * NBMAX + kTbThreads - 1) / kTbThreads;  // list slots per thread
  int sidx[KSEG], slim[KSEG];
  uint32_t smask[KSEG][L];
#pragma unroll
  for (int kk = 0; kk < KSEG; ++kk) {
    const int k = tid + kk * kTbThreads;
    sidx[kk] = 0;
    slim[kk] = 0;  // an empty slot is needed by no generation
#pragma unroll
    for (int q = 0; q < L; ++q) smask[kk][q] = 0u;
    if (k < ns) {
      const uint32_t code = segs[k];
      const int w = (int)(code & 0xffu), i0 = (int)((code >> 8) & 0xffu) * L;
      const uint32_t rows = code >> 16;
      sidx[kk] = (i0 + 1) * PW + (w + 1);
      const int span = (w == 0 || w == W - 1) ? T - 1 : T;
      slim[kk] = min(span, min(i0 + L - 1, R - 1 - i0));
#pragma unroll
      for (int q = 0; q < L; ++q) smask[kk][q] = ((rows >> q) & 1u) ? rowpat[i0 + q] : 0u;
    }
  }
  const int wave0 = __builtin_amdgcn_readfirstlane(tid) & ~63;  // the wave's first thread
  for (int s = 0; s < T; ++s) {
    const uint32_t *src = plane0;
    uint32_t outw[KSEG][L];  // the generation's new rows, stored once every read is done
#pragma unroll
    for (int kk = 0; kk < KSEG; ++kk) {
      if (wave0 + kk * kTbThreads >= ns) break;  // this wave holds no segment here
      if (s >= slim[kk]) continue;               // cannot reach the tile any more
      const int idx0 = sidx[kk];
      // all rows the segment reads, their loads issued together
      uint32_t row[L + 2][3];
#pragma unroll
      for (int q = 0; q < L + 2; ++q) {
        const uint32_t *p = src + idx0 + (q - 1) * PW;
        row[q][0] = p[-1];
        row[q][1] = p[0];
        row[q][2] = p[1];
      }
      RowSums up = row_sums(row[0][0], row[0][1], row[0][2]);
      RowSums mid = row_sums(row[1][0], row[1][1], row[1][2]);
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const RowSums dn = row_sums(row[q + 2][0], row[q + 2][1], row[q + 2][2]);
        outw[kk][q] = life_rule(up, mid, dn, smask[kk][q]);
        up = mid;
        mid = dn;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KSEG; ++kk) {
      if (wave0 + kk * kTbThreads >= ns) break;
      if (s >= slim[kk]) continue;
#pragma unroll
      for (int q = 0; q < L; ++q) plane0[sidx[kk] + q * PW] = outw[kk][q];
    }
    __syncthreads();
  }
  const uint16_t *fin = reinterpret_cast<const uint16_t *>(plane0);

  // 4. unpack and store the tile.  In the embedding, a wave takes the store
  //    units w, w + NW, ... (TileUnits): 16 rows of one 64-byte granule that
  //    holds gasket cells, so every granule written is written whole and
  //    granules without a gasket cell are never touched.  A compact tile, and
  //    the 32-byte rows of rho = 32, are rewritten whole: thread tid takes
  //    chunk column tid % TC of tile rows tid / TC, + RPS, ...
  //    Bit-packed output: thread tid takes the 4-row runs tid, tid + NT, ...
  //    of the tile's words, column by column.
  constexpr int TC = RHO / 16;  // 16-byte chunks per tile row
  if constexpr (Mem::kBits) {
    constexpr int GT = RHO / 4;  // 4-row runs per word column
    const uint32_t *fw = plane0;
    uint32_t *o = mem.out + (size_t)(uint32_t)mem.nbr[4] * bit_tile_words<RHO>();
    for (int u = tid; u < (RHO / 32) * GT; u += kTbThreads) {
      const int j = u / GT, g = u % GT;
      const uint32_t *f = fw + (T + 1 + 4 * g) * PW + 2 + j;
      *reinterpret_cast<uint4 *>(o + j * RHO + 4 * g) = make_uint4(f[0], f[PW], f[2 * PW], f[3 * PW]);
    }
  } else if constexpr (!Mem::kCompact && RHO >= 64) {
    constexpr int NS = TileUnitTable<RHO>::units.nstore;
    for (int u = wave; u < NS; u += NW) {
      const uint32_t pr = kTileUnits<RHO>.store_pairs[u];
      const int ty = 16 * (int)(pr >> 4) + (lane >> 2);
      const int j = 4 * (int)(pr & 15u) + (lane & 3);  // tile chunk; region chunk j + 2
      const uint32_t bits = fin[((T + 1 + ty) * PW + 2 + (j >> 1)) * 2 + (j & 1)];
      store16(mem.dst(Y0 + ty, X0 + 16 * j), unpack16(bits), stream_out);
    }
  } else {
    constexpr int RPS = kTbThreads / TC;  // tile rows per round
    static_assert(kTbThreads % TC == 0, "the store rounds cover whole rows");
    const int j = tid % TC, x = X0 + 16 * j;
    const int f0 = ((T + 1) * PW + 2 + (j >> 1)) * 2 + (j & 1);
    for (int ty = tid / TC; ty < RHO; ty += RPS) {
      const int y = Y0 + ty;
      // the embedding keeps rows without a gasket cell untouched (none at
      // rho = 32: every row of a gasket block holds its cell 0)
      if (!Mem::kCompact && ((x & ~(G - 1)) & y) != 0) continue;
      const uint32_t bits = fin[f0 + ty * (2 * PW)];
      store16(mem.dst(y, x), unpack16(bits), stream_out);
    }
  }
}

// Block (bx, by) of tile t of a pass over the lambda map's 3^rb tiles, or
// the bounding box's 4^rb; false for a bounding-box tile off the gasket.
template <bool LAMBDA>
__device__ __forceinline__ bool tile_block(uint64_t t, int rb, uint32_t &bx, uint32_t &by) {
  if constexpr (LAMBDA) {
    pass_decode((uint32_t)t, rb, bx, by);
    return true;
  } else {
    by = (uint32_t)(t >> rb);
    bx = (uint32_t)(t & ((1ull << rb) - 1ull));
    return (bx & by) == 0u;
  }
}

// One workgroup per tile of one gasket.  Its region loads are issued first,
// so they are in flight while the LDS plane is cleared.
template <int RHO, bool LAMBDA, int NT>
__global__ __launch_bounds__(NT, kTbWavesPerSimd) void k_life_tb(const uint8_t *__restrict__ in,
                                                               uint8_t *__restrict__ out, int r,
                                                               int rb, uint64_t tile_base,
                                                               uint64_t ntiles, int T,
                                                               int stream_out) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t nseg;
  const uint64_t t = tile_base + logical_group();
  if (t >= ntiles) return;
  uint32_t bx, by;
  if (!tile_block<LAMBDA>(t, rb, bx, by)) return;
  const DenseMem mem{in, out, r};
  RegionLoads<RHO, NT> ld;
  tb_load<RHO, NT>(mem, r, bx, by, T, ld);
  tb_tile<RHO, NT>(mem, r, bx, by, T, lds, &nseg, ld, stream_out != 0);
}

// A pass with bit-packed tiles on either side (SRC_BITS: the input, DST_BITS:
// the output) and the byte embedding on the other, if any: the passes of a
// multi-pass run after the first read bits, those before the last write
// them.  The 3 x 3 blocks' omegas are found first, into LDS; with a byte
// input its loads are issued before the workgroup waits for them.
template <int RHO, bool LAMBDA, bool SRC_BITS, bool DST_BITS, int NT>
__global__ __launch_bounds__(NT, kTbWavesPerSimd) void k_life_tb_bits(
    const void *__restrict__ in, void *__restrict__ out, int r, int rb, uint64_t tile_base,
    uint64_t ntiles, int T, int stream_out) {
  static_assert(SRC_BITS || DST_BITS, "byte-to-byte passes are k_life_tb");
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t nseg;
  __shared__ int32_t nbr[9];
  const uint64_t t = tile_base + logical_group();
  if (t >= ntiles) return;
  uint32_t bx, by;
  if (!tile_block<LAMBDA>(t, rb, bx, by)) return;
  const int tid = (int)threadIdx.x;
  auto run = [&](const auto &ld) {
    if constexpr (DST_BITS) {
      const BitsOut mem{static_cast<uint32_t *>(out), nbr};
      tb_tile<RHO, NT>(mem, r, bx, by, T, lds, &nseg, ld, false);
    } else {
      const DenseMem mem{nullptr, static_cast<uint8_t *>(out), r};
      tb_tile<RHO, NT>(mem, r, bx, by, T, lds, &nseg, ld, stream_out != 0);
    }
  };
  if constexpr (SRC_BITS) {
    neighbour_omegas(tid, bx, by, rb, nbr);
    __syncthreads();
    BitLoads<RHO, NT> ld;
    bits_load<RHO, NT>(static_cast<const uint32_t *>(in), nbr, T, ld);
    run(ld);
  } else {
    RegionLoads<RHO, NT> ld;
    tb_load<RHO, NT>(DenseMem{static_cast<const uint8_t *>(in), nullptr, r}, r, bx, by, T, ld);
    neighbour_omegas(tid, bx, by, rb, nbr);  // read at the store, after tb_tile's barriers
    run(ld);
  }
}

// One workgroup per tile of a gasket in block-compacted storage (lambda
// order): tile omega is the workgroup's omega.
template <int RHO>
__global__ __launch_bounds__(tb_threads<RHO>(), kTbWavesPerSimd) void k_life_tb_compact(
    const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int r, int rb,
    uint64_t tile_base, uint64_t ntiles, int T, int stream_out) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t nseg;
  __shared__ int32_t nbr[9];
  const uint64_t t = tile_base + logical_group();
  if (t >= ntiles) return;
  uint32_t bx, by;
  lambda_decode((uint32_t)t, rb, bx, by);  // storage order
  const CompactMem<RHO> mem{in, out, nbr, (int)bx, (int)by};
  mem.prepare((int)threadIdx.x, bx, by, rb);
  __syncthreads();  // the neighbour tiles' omegas
  RegionLoads<RHO, tb_threads<RHO>()> ld;
  tb_load<RHO, tb_threads<RHO>()>(mem, r, bx, by, T, ld);
  tb_tile<RHO, tb_threads<RHO>()>(mem, r, bx, by, T, lds, &nseg, ld, stream_out != 0);
}

// A pass over block-compacted storage with bit-packed tiles (the same
// lambda order: tile omega is the workgroup's omega) as its input, its
// output, or both, and compact byte tiles on the other side, if any.
template <int RHO, bool SRC_BITS, bool DST_BITS>
__global__ __launch_bounds__(tb_threads<RHO>(), kTbWavesPerSimd) void k_life_tb_compact_bits(
    const void *__restrict__ in, void *__restrict__ out, int r, int rb, uint64_t tile_base,
    uint64_t ntiles, int T, int stream_out) {
  static_assert(SRC_BITS || DST_BITS, "byte-to-byte passes are k_life_tb_compact");
  constexpr int NT = tb_threads<RHO>();
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t nseg;
  __shared__ int32_t nbr[9];
  const uint64_t t = tile_base + logical_group();
  if (t >= ntiles) return;
  uint32_t bx, by;
  lambda_decode((uint32_t)t, rb, bx, by);  // storage order
  neighbour_omegas((int)threadIdx.x, bx, by, rb, nbr);
  __syncthreads();  // the neighbour tiles' omegas, for either side
  auto run = [&](const auto &ld) {
    if constexpr (DST_BITS) {
      const BitsOut mem{static_cast<uint32_t *>(out), nbr};
      tb_tile<RHO, NT>(mem, r, bx, by, T, lds, &nseg, ld, false);
    } else {
      const CompactMem<RHO> mem{nullptr, static_cast<uint8_t *>(out), nbr, (int)bx, (int)by};
      tb_tile<RHO, NT>(mem, r, bx, by, T, lds, &nseg, ld, stream_out != 0);
    }
  };
  if constexpr (SRC_BITS) {
    BitLoads<RHO, NT> ld;
    bits_load<RHO, NT>(static_cast<const uint32_t *>(in), nbr, T, ld);
    run(ld);
  } else {
    const CompactMem<RHO> src{static_cast<const uint8_t *>(in), nullptr, nbr, (int)bx, (int)by};
    RegionLoads<RHO, NT> ld;
    tb_load<RHO, NT>(src, r, bx, by, T, ld);
    run(ld);
  }
}

// One tile of a batched pass: its region loads, then the tile pass.
template <int RHO, int NT>
__device__ __forceinline__ void batch_tile(const DenseMem &mem, int r, uint32_t bx, uint32_t by,
                                           int T, uint32_t *lds, uint32_t *nseg, bool stream_out) {
  RegionLoads<RHO, NT> ld;
  tb_load<RHO, NT>(mem, r, bx, by, T, ld);
  tb_tile<RHO, NT>(mem, r, bx, by, T, lds, nseg, ld, stream_out);
}

// Many gaskets in one persistent launch: workgroups stride over the global
// tile index of all items (each item's lambda tiles numbered from its
// tile_begin, items sorted by tile_begin), find the item by a binary search
// (uniform per workgroup, so it runs on the scalar unit) and run the tile
// pass on that item's buffers, with that item's tile side (up to MAXRHO) and
// generation count.
template <int MAXRHO, int NT>
__global__ __launch_bounds__(NT, kTbWavesPerSimd) void k_life_tb_batch(const BatchItem *__restrict__ items,
                                                      int count, uint64_t total_tiles,
                                                      int stream_out) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t nseg;
  for (uint64_t g = blockIdx.x; g < total_tiles; g += gridDim.x) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= g) lo = mid; else hi = mid - 1;
    }
    const BatchItem it = items[lo];
    uint32_t bx, by;
    pass_decode((uint32_t)(g - it.tile_begin), it.r - it.k, bx, by);
    const DenseMem mem{it.src, it.dst, it.r};
    if (it.k == 6) {
      batch_tile<64, NT>(mem, it.r, bx, by, it.steps, lds, &nseg, stream_out != 0);
    } else if (MAXRHO >= 128 && it.k == 7) {
      batch_tile<(MAXRHO >= 128 ? 128 : 64), NT>(mem, it.r, bx, by, it.steps, lds, &nseg,
                                                 stream_out != 0);
    } else if (MAXRHO >= 256 && it.k == 8) {
      batch_tile<(MAXRHO >= 256 ? 256 : 64), NT>(mem, it.r, bx, by, it.steps, lds, &nseg,
                                                 stream_out != 0);
    }
    __syncthreads();  // the next tile reuses the LDS plane
  }
}

template <int RHO>
size_t tb_lds_bytes(int T) {
  // the layout of tb_tile: the plane, the row patterns, and a segment list
  // of up to W * NB entries (W = the tile's words plus a halo word each side)
  const int W = RHO / 32 + 2, PW = plane_pitch(W), R = RHO + 2 * T;
  const int NB = (R + kSegRows - 1) / kSegRows, RP = NB * kSegRows, PR = RP + 2;
  return sizeof(uint32_t) * (size_t)(PR * PW + RP + W * NB);
}

// Threads per workgroup of a dense or bit pass.  tb_threads (256: 8
// workgroups share a compute unit, so nearly every wave slot runs segments)
// once the grid fills the chip; 512 at rho = 256 when every gasket tile runs
// at once (at most 256 compute units x 4 workgroups of 512), where a tile's
// latency is the pass's and twice the threads halve the segments per wave.
constexpr uint64_t kWideTileLimit = 1024;
template <int RHO>
bool tb_wide(const PassArgs &a) {
  if (RHO < 256 || tb_threads<RHO>() != 256) return false;
  uint64_t tiles = 1;  // gasket tiles, for either map
  for (int i = 0; i < a.rb && tiles <= kWideTileLimit; ++i) tiles *= 3;
  return tiles <= kWideTileLimit;
}

template <int RHO, int NT>
hipError_t life_tb_launch(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  const size_t lds = tb_lds_bytes<RHO>(T);
  const int stream_out = life_stream_stores(life_touched_bytes(a.r)) ? 1 : 0;
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    if (a.lambda)
      hipLaunchKernelGGL((k_life_tb<RHO, true, NT>), dim3((unsigned)g), dim3(NT), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T, stream_out);
    else
      hipLaunchKernelGGL((k_life_tb<RHO, false, NT>), dim3((unsigned)g), dim3(NT), lds,
                         a.stream, in, out, a.r, a.rb, g0, a.ntiles, T, stream_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO>
hipError_t life_tb_rho(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  if constexpr (RHO >= 256) {
    if (tb_wide<RHO>(a)) return life_tb_launch<RHO, 512>(a, T, in, out);
  }
  return life_tb_launch<RHO, tb_threads<RHO>()>(a, T, in, out);
}

// Bytes of one bit-packed state of tiles of side RHO at block level rb.
template <int RHO>
size_t bit_state_bytes(int rb) {
  uint64_t t = 1;
  for (int i = 0; i < rb; ++i) t *= 3;
  return (size_t)t * bit_tile_words<RHO>() * sizeof(uint32_t);
}

template <int RHO, bool LAMBDA, int NT>
hipError_t life_tb_bits_map(const PassArgs &a, int T, const void *in, bool in_bits, void *out,
                            bool out_bits) {
  const size_t lds = tb_lds_bytes<RHO>(T);
  // a byte output streams when it and the bits read exceed the cache; bits
  // written are read by the next pass
  const uint64_t touched = life_touched_bytes(a.r) / 2 + bit_state_bytes<RHO>(a.rb);
  const int stream_out = !out_bits && life_stream_stores(touched) ? 1 : 0;
  auto k = in_bits ? (out_bits ? k_life_tb_bits<RHO, LAMBDA, true, true, NT>
                               : k_life_tb_bits<RHO, LAMBDA, true, false, NT>)
                   : k_life_tb_bits<RHO, LAMBDA, false, true, NT>;
  if (!in_bits && !out_bits) return hipErrorInvalidValue;
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(NT), lds, a.stream, in, out,
                       a.r, a.rb, g0, a.ntiles, T, stream_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO>
hipError_t life_tb_bits_rho(const PassArgs &a, int T, const void *in, bool in_bits, void *out,
                            bool out_bits) {
  constexpr int NT = tb_threads<RHO>();
  if constexpr (RHO >= 256) {
    if (tb_wide<RHO>(a))
      return a.lambda ? life_tb_bits_map<RHO, true, 512>(a, T, in, in_bits, out, out_bits)
                      : life_tb_bits_map<RHO, false, 512>(a, T, in, in_bits, out, out_bits);
  }
  return a.lambda ? life_tb_bits_map<RHO, true, NT>(a, T, in, in_bits, out, out_bits)
                  : life_tb_bits_map<RHO, false, NT>(a, T, in, in_bits, out, out_bits);
}

template <int RHO>
hipError_t life_tb_compact_rho(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  const size_t lds = tb_lds_bytes<RHO>(T);
  // whole tiles are read and written: 2 states of ntiles * rho^2 bytes
  const int stream_out = life_stream_stores(2 * a.ntiles * RHO * RHO) ? 1 : 0;
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    hipLaunchKernelGGL((k_life_tb_compact<RHO>), dim3((unsigned)g), dim3(tb_threads<RHO>()), lds,
                       a.stream, in, out, a.r, a.rb, g0, a.ntiles, T, stream_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO>
hipError_t life_tb_compact_bits_rho(const PassArgs &a, int T, const void *in, bool in_bits,
                                    void *out, bool out_bits) {
  const size_t lds = tb_lds_bytes<RHO>(T);
  // a compact byte output streams when it and the bits read exceed the cache
  const uint64_t touched = a.ntiles * RHO * RHO + bit_state_bytes<RHO>(a.rb);
  const int stream_out = !out_bits && life_stream_stores(touched) ? 1 : 0;
  if (!in_bits && !out_bits) return hipErrorInvalidValue;
  auto k = in_bits ? (out_bits ? k_life_tb_compact_bits<RHO, true, true>
                               : k_life_tb_compact_bits<RHO, true, false>)
                   : k_life_tb_compact_bits<RHO, false, true>;
  const uint64_t per_launch = 1ull << 22;
  for (uint64_t g0 = 0; g0 < a.ntiles; g0 += per_launch) {
    const uint64_t g = a.ntiles - g0 < per_launch ? a.ntiles - g0 : per_launch;
    hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(tb_threads<RHO>()), lds, a.stream, in, out,
                       a.r, a.rb, g0, a.ntiles, T, stream_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int RHO, int NT>
hipError_t life_tb_batch_rho(const BatchItem *d_items, int count, uint64_t total_tiles,
                             int max_steps, int groups, bool stream_out, hipStream_t stream) {
  // the largest tile side needs the most LDS
  const size_t lds = tb_lds_bytes<RHO>(max_steps);
  const uint64_t g = total_tiles < (uint64_t)groups ? total_tiles : (uint64_t)groups;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL((k_life_tb_batch<RHO, NT>), dim3((unsigned)g), dim3(NT), lds, stream,
                     d_items, count, total_tiles, stream_out ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_life_tb_batch(int max_rho, int threads, const BatchItem *d_items, int count,
                                uint64_t total_tiles, int max_steps, int groups,
                                bool stream_out, hipStream_t stream) {
  if (max_steps < 1 || max_steps > kMaxStepsPerPass || groups < 1) return hipErrorInvalidValue;
  const bool t512 = threads == 512;
  if (threads != 256 && threads != 512) return hipErrorInvalidValue;
  const bool so = stream_out;
  switch (max_rho) {
    case 64: return t512 ? life_tb_batch_rho<64, 512>(d_items, count, total_tiles, max_steps, groups, so, stream)
                         : life_tb_batch_rho<64, 256>(d_items, count, total_tiles, max_steps, groups, so, stream);
    case 128: return t512 ? life_tb_batch_rho<128, 512>(d_items, count, total_tiles, max_steps, groups, so, stream)
                          : life_tb_batch_rho<128, 256>(d_items, count, total_tiles, max_steps, groups, so, stream);
    case 256: return t512 ? life_tb_batch_rho<256, 512>(d_items, count, total_tiles, max_steps, groups, so, stream)
                          : life_tb_batch_rho<256, 256>(d_items, count, total_tiles, max_steps, groups, so, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_life_tb_compact(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  if (T < 1 || T > kMaxStepsPerPass) return hipErrorInvalidValue;
  switch (a.rho) {
    case 64: return life_tb_compact_rho<64>(a, T, in, out);
    case 128: return life_tb_compact_rho<128>(a, T, in, out);
    case 256: return life_tb_compact_rho<256>(a, T, in, out);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_life_tb_compact_bits(const PassArgs &a, int T, const void *in, bool in_bits,
                                       void *out, bool out_bits) {
  if (T < 1 || T > kMaxStepsPerPass || !(in_bits || out_bits)) return hipErrorInvalidValue;
  switch (a.rho) {
    case 64: return life_tb_compact_bits_rho<64>(a, T, in, in_bits, out, out_bits);
    case 128: return life_tb_compact_bits_rho<128>(a, T, in, in_bits, out, out_bits);
    case 256: return life_tb_compact_bits_rho<256>(a, T, in, in_bits, out, out_bits);
    default: return hipErrorInvalidValue;
  }
}

bool life_tb_supported(int rho) { return rho == 64 || rho == 128 || rho == 256; }
bool life_tb_dense_supported(int rho) { return rho == 32 || life_tb_supported(rho); }

size_t life_tb_bit_state_bytes(const PassArgs &a) {
  switch (a.rho) {
    case 32: return bit_state_bytes<32>(a.rb);
    case 64: return bit_state_bytes<64>(a.rb);
    case 128: return bit_state_bytes<128>(a.rb);
    case 256: return bit_state_bytes<256>(a.rb);
    default: return 0;
  }
}

hipError_t launch_life_tb_bits(const PassArgs &a, int T, const void *in, bool in_bits, void *out,
                               bool out_bits) {
  if (T < 1 || T > kMaxStepsPerPass || !(in_bits || out_bits)) return hipErrorInvalidValue;
  switch (a.rho) {
    case 32: return life_tb_bits_rho<32>(a, T, in, in_bits, out, out_bits);
    case 64: return life_tb_bits_rho<64>(a, T, in, in_bits, out, out_bits);
    case 128: return life_tb_bits_rho<128>(a, T, in, in_bits, out, out_bits);
    case 256: return life_tb_bits_rho<256>(a, T, in, in_bits, out, out_bits);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_life_tb(const PassArgs &a, int T, const uint8_t *in, uint8_t *out) {
  if (T < 1 || T > kMaxStepsPerPass) return hipErrorInvalidValue;
  switch (a.rho) {
    case 32: return life_tb_rho<32>(a, T, in, out);
    case 64: return life_tb_rho<64>(a, T, in, out);
    case 128: return life_tb_rho<128>(a, T, in, out);
    case 256: return life_tb_rho<256>(a, T, in, out);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sg
