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

template <int M, bool LAMBDA>
__global__ __launch_bounds__(kFracThreads) void k_frac_write(FracArgs f, FracPass p,
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

constexpr uint64_t kFracMaxGroups = 1ull << 22;

template <int M, bool LAMBDA, bool LIFE>
hipError_t frac_pass_m(const FracArgs &f, const FracPass &p, hipStream_t s, uint8_t *a,
                       const uint8_t *in, uint32_t value) {
  const uint64_t groups = (p.ntiles + p.tpg - 1) / p.tpg;
  const size_t lds = LIFE ? (size_t)p.tpg * (p.rho + 2) * (p.rho + 2) : 0;
  for (uint64_t g0 = 0; g0 < groups; g0 += kFracMaxGroups) {
    const uint64_t g = groups - g0 < kFracMaxGroups ? groups - g0 : kFracMaxGroups;
    if (LIFE)
      hipLaunchKernelGGL((k_frac_life<M, LAMBDA>), dim3((unsigned)g), dim3(kFracThreads), lds, s,
                         f, p, g0 * (uint64_t)p.tpg, in, a);
    else
      hipLaunchKernelGGL((k_frac_write<M, LAMBDA>), dim3((unsigned)g), dim3(kFracThreads), 0, s,
                         f, p, g0 * (uint64_t)p.tpg, a, value);
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
