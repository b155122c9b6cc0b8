/*
 * sg.h -- C ABI of libsg, the MI355X (gfx950) library for the block-space
 * thread map lambda(omega) of "Block-space GPU Mapping for Embedded
 * Sierpinski Gasket Fractals" (Navarro, Bustos, Vega, Hitschfeld,
 * arXiv 1706.04552) and the data-parallel passes it feeds.
 *
 * Problem (Section I): a Sierpinski gasket of level r is embedded in an
 * n x n array, n = 2^r, so that memory neighbours (x+-1, y+-1) are fractal
 * neighbours.  A GPU pass over the gasket maps blocks of rho x rho threads
 * (rho = 2^k) onto blocks of the array.  The bounding-box map (BB) launches
 * all n_b x n_b blocks (n_b = n/rho) and discards the threads that fall off
 * the gasket; lambda(omega) (Theorem 1, Eq. 4-10) launches only the
 * 3^(r-k) blocks that hold gasket cells.
 *
 * Coordinates (build frame): cell (x, y) is column x, row y, 0-based,
 * stored row-major with pitch n; it belongs to the gasket iff
 * (x & y) == 0.  The paper's frame (origin top-left, y down, test
 * x & (n-1-y) == 0, Section III-D) is this frame reflected by y -> n-1-y.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are DEVICE pointers (hipMalloc'd or torch tensors),
 *    owned by the caller; the library never frees or keeps them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is asynchronous on that stream; the library does not
 *    synchronise.
 *  - Arguments are validated on the host before any HIP call, so invalid
 *    arguments return an error with no device work queued.
 *  - State arrays (d_a, d_in, d_out) must be 16-byte aligned; misaligned
 *    pointers return SG_EINVAL.
 *  - r must lie in [0, SG_MAX_R]; rho must be a power of two in
 *    [1, SG_MAX_RHO] with rho <= n.
 *  - State arrays are n x n and must hold 0 on every cell off the gasket
 *    (the caller zeroes both ping-pong buffers once).  Entry points never
 *    touch a block that holds no gasket cell; inside a block they may store
 *    0 into cells off the gasket.  Results on inputs with non-zero cells off
 *    the gasket are unspecified.
 *  - Return value: SG_OK (0) or a negative sg_status.  Launch failures are
 *    reported as SG_EHIP; faults of a running kernel surface at the caller's
 *    next synchronisation, as for any asynchronous HIP work.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_API __attribute__((visibility("default")))

#define SG_MAX_R 20
#define SG_MAX_RHO 256

typedef enum sg_status {
    SG_OK = 0,
    SG_EINVAL = -1, /* r, rho, map kind or a size out of range; null pointer */
    SG_EALIAS = -2, /* input and output arrays overlap */
    SG_EHIP = -3,   /* a HIP runtime call or kernel launch failed */
    SG_ENOMEM = -4, /* the library could not allocate what it needs */
} sg_status;

typedef enum sg_map_kind {
    SG_MAP_LAMBDA = 0, /* lambda(omega): one block per fractal block */
    SG_MAP_BBOX = 1    /* bounding box: every block, off-gasket threads discarded */
} sg_map_kind;

/* Human-readable text of a status code (static storage, never NULL). */
SG_API const char *sg_strerror(int code);

/* Text of the last HIP error the calling thread met inside the library, or
 * "" if none (static per-thread storage). */
SG_API const char *sg_last_hip_error(void);

/* ABI version, bumped when a signature changes. */
SG_API int sg_version(void);

/* Host only.  Sides of the lambda launch orthotope Pi^2 for level r and
 * block side rho (Lemma 2, Eq. 4): *W = 3^floor(r_b/2) columns (omega_x),
 * *H = 3^ceil(r_b/2) rows (omega_y), r_b = r - log2(rho); W*H = 3^r_b.
 * Errors: SG_EINVAL for bad r/rho or null outputs. */
SG_API int sg_lambda_grid(int r, int rho, uint64_t *W, uint64_t *H);

/* Host only.  Number of blocks the given map launches: 3^r_b for lambda,
 * 4^r_b = n_b^2 for the bounding box (Theorem 2's parallel spaces). */
SG_API int sg_block_count(int map, int r, int rho, uint64_t *blocks);

/* lambda(omega), Theorem 1, Eq. 4-10.  Writes the block each omega maps to:
 * d_bxy[2i] = bx, d_bxy[2i+1] = by for omega = (omega_x, omega_y) at linear
 * index i = omega_y * W + omega_x, in the build frame
 * (bx, by) = (lambda_x, n_b - 1 - lambda_y).
 * d_bxy: device, 2 * 3^r_b uint32 (8-byte aligned).  Errors: SG_EINVAL. */
SG_API int sg_map_lambda(int r, int rho, uint32_t *d_bxy, void *stream);

/* Inverse of lambda: d_omega[by * n_b + bx] = the linear omega that
 * sg_map_lambda sends to block (bx, by), or -1 if the block holds no gasket
 * cell.  d_omega: device, n_b * n_b int32 (4-byte aligned).
 * Errors: SG_EINVAL (also 3^r_b > 2^31 - 1). */
SG_API int sg_map_lambda_inverse(int r, int rho, int32_t *d_omega, void *stream);

/* Bounding-box map (Section I, Fig. 3): the identity over the n_b x n_b
 * block grid.  d_mask[by * n_b + bx] = 1 iff block (bx, by) keeps at least
 * one thread (holds a gasket cell), else 0.
 * d_mask: device, n_b * n_b bytes.  Errors: SG_EINVAL. */
SG_API int sg_map_bbox(int r, int rho, uint8_t *d_mask, void *stream);

/* Write pass, the paper's experiment (Section IV): store `value` into every
 * gasket cell of d_a; cells off the gasket keep (or get) 0.
 * map: SG_MAP_LAMBDA or SG_MAP_BBOX (same result, different launch).
 * d_a: device, n * n bytes, row-major.  Errors: SG_EINVAL. */
SG_API int sg_write_pass(int map, int r, int rho, uint8_t *d_a, uint8_t value,
                         void *stream);

/* Intra-block mapping of the threads of a block (Section III-D). */
typedef enum sg_intra_kind {
    SG_INTRA_SUBBOX = 0, /* bounding sub-boxes: every cell of the block, masked */
    SG_INTRA_UNROLL = 1, /* further unrolling: lambda again at thread level */
    SG_INTRA_LUT = 2     /* a shared lookup table of the in-block cell offsets */
} sg_intra_kind;

/* The write pass with a chosen intra-block mapping.  SG_INTRA_SUBBOX is
 * sg_write_pass.  SG_INTRA_UNROLL and SG_INTRA_LUT launch only the 3^k
 * threads per block that own a gasket cell (rho = 2^k <= 32) and store one
 * byte each: cells off the gasket are never written.
 * Errors: SG_EINVAL (also rho > 32 for UNROLL/LUT), SG_EHIP. */
SG_API int sg_write_pass_intra(int map, int intra, int r, int rho, uint8_t *d_a,
                               uint8_t value, void *stream);

/* One generation of B3/S23 life on the gasket (an application of the
 * embedded gasket, Section I): for every gasket cell, c = number of live
 * cells among its 8 neighbours that lie in the grid and in the gasket;
 * out = 1 iff c == 3 or (in == 1 and c == 2); cells off the gasket are 0.
 * d_in, d_out: device, n * n bytes holding 0/1, distinct, not overlapping.
 * Errors: SG_EINVAL, SG_EALIAS. */
SG_API int sg_ca_step(int map, int r, int rho, const uint8_t *d_in,
                      uint8_t *d_out, void *stream);

/* `steps` generations of the life step above (sg_ca_step), with the result
 * left in d_out.  The generations run in ceil(steps / steps_per_pass)
 * passes that split them as evenly as possible (each runs floor or ceil of
 * steps / passes, at most `steps_per_pass`): a pass reads its tile plus a
 * halo of as many cells as its generations from HBM once, runs the
 * generations on chip and writes the tile once (temporal blocking), so HBM
 * traffic per generation falls by that factor.  The result is identical to
 * `steps` calls of sg_ca_step.
 *   steps_per_pass: 1 (one launch per generation, any rho), 2..32 (rho in
 *     {32, 64, 128, 256}), 2..16 (rho = 16), or 0 for the library's choice
 *     (the largest where supported, else 1).
 *   d_in: read only.  d_out: receives the state after `steps` generations.
 *   d_work: a third n * n buffer used when more than one pass runs (may be
 *     NULL otherwise).  All three: device, 16-byte aligned, pairwise
 *     non-overlapping, 0 on every cell off the gasket.  With rho in {32, 64,
 *     128, 256} and steps_per_pass >= 2, the state between passes is kept in
 *     d_work as bit-packed tiles (one bit per cell, lambda order), so a pass
 *     that neither starts nor ends the run reads and writes about an eighth
 *     of the bytes; d_work's contents after the call are unspecified.
 *   steps = 0 copies d_in to d_out.
 * Errors: SG_EINVAL (bad sizes, steps < 0, unsupported steps_per_pass for
 * rho, d_work missing when needed), SG_EALIAS, SG_EHIP. */
SG_API int sg_ca_steps(int map, int r, int rho, int steps, int steps_per_pass,
                       const uint8_t *d_in, uint8_t *d_out, uint8_t *d_work,
                       void *stream);

/* Launch-shape autotuner of sg_ca_steps for one gasket: times `steps`
 * generations from d_in on the caller's buffers (d_out and d_work written,
 * d_in only read; d_work needed) for every tile side rho in {32, 64, 128,
 * 256} that fits in n and every steps_per_pass in {8, 16, 32}, one warm-up
 * call and one timed call each (HIP events on `stream`), and returns the
 * fastest shape and its time in milliseconds.  Synchronises the stream.
 * Errors: SG_EINVAL (as sg_ca_steps for any candidate, steps < 1, n < 32,
 * NULL outputs), SG_EALIAS, SG_EHIP. */
SG_API int sg_ca_steps_autotune(int map, int r, int steps, const uint8_t *d_in, uint8_t *d_out,
                                uint8_t *d_work, int *best_rho, int *best_steps_per_pass,
                                float *best_ms, void *stream);

/* One explicit diffusion step on the gasket in FP32 (a nearest-neighbour
 * application, Section I): for every gasket cell,
 *   out = u + alpha * sum_{nb in W, E, N, S; in grid and in gasket} (u_nb - u);
 * cells off the gasket are 0 and never enter a sum.  In FP32 the sum is
 * formed as (u_W + u_E) + (u_N + u_S) - deg * u (one fma; deg the number of
 * those neighbours, off-gasket neighbours contributing their 0) and
 * out = u + alpha * that (one fma).
 * d_in, d_out: device, n * n floats, distinct, not overlapping.
 * Errors: SG_EINVAL, SG_EALIAS. */
SG_API int sg_diffuse_step(int map, int r, int rho, const float *d_in,
                           float *d_out, float alpha, void *stream);

/* `steps` diffusion steps (sg_diffuse_step) with the result in d_out, in
 * ceil(steps / steps_per_pass) passes that split the steps as evenly as
 * possible (as sg_ca_steps): a pass reads its tile plus a halo of as many
 * cells as its steps from HBM once and runs the steps on chip (temporal
 * blocking).  Every cell update is the same FP32 arithmetic as
 * sg_diffuse_step, so the result equals `steps` calls of it bit for bit.
 *   steps_per_pass: 1 (one launch per step, any rho), 2..16 (rho in {16, 32,
 *     64}), or 0 for the library's choice (16 at rho = 16 and 64, 8 at
 *     rho = 32, else 1).
 *   d_in: read only.  d_out: the state after `steps` steps.  d_work: a third
 *     n * n float buffer, used when more than one pass runs (may be NULL
 *     otherwise).  All: device, 16-byte aligned, pairwise non-overlapping,
 *     0 off the gasket.  steps = 0 copies d_in to d_out.
 * Errors: SG_EINVAL, SG_EALIAS, SG_EHIP. */
SG_API int sg_diffuse_steps(int map, int r, int rho, int steps, int steps_per_pass,
                            const float *d_in, float *d_out, float *d_work, float alpha,
                            void *stream);

/* ---------------------------------------------------------------------
 * Block-compacted storage: only the 3^r_b fractal tiles of side rho (64,
 * 128 or 256), tile omega (lambda order, as sg_map_lambda) stored at byte
 * omega * rho^2 as rho rows of rho bytes -- (4/3)^k * 3^r bytes instead of
 * the n^2 of the embedding.  A compact state holds 0 on the cells of its
 * tiles that are off the gasket.
 * --------------------------------------------------------------------- */

/* Host only.  Bytes of a compact state: 3^r_b * rho^2. */
SG_API int sg_compact_bytes(int r, int rho, uint64_t *bytes);

/* Embedding (n * n bytes) -> compact state, and back.  Unpack writes the
 * fractal tiles of d_dense whole and nothing else (the rest must be 0).
 * Errors: SG_EINVAL, SG_EALIAS (the two arrays overlap), SG_EHIP. */
SG_API int sg_compact_pack(int r, int rho, const uint8_t *d_dense, uint8_t *d_compact,
                           void *stream);
SG_API int sg_compact_unpack(int r, int rho, const uint8_t *d_compact, uint8_t *d_dense,
                             void *stream);

/* A seeded Bernoulli life state written straight into a compact state
 * (sg_compact_bytes bytes, 16-byte aligned), for gaskets whose embedding is
 * too large to build (at r = 20 it would take 2^40 bytes; the compact state
 * at rho = 256 takes 35 GB).  Gasket cell (x, y) is 1 iff output number
 * y * 2^32 + x (from 0) of the SplitMix64 generator seeded with `seed`
 * (Steele, Lea and Flood, OOPSLA 2014) is below `threshold` (so each cell is
 * alive with probability threshold / 2^64); every other byte is 0.  The same
 * state as sg_compact_pack of an embedding built that way.
 * Errors: SG_EINVAL (shape, rho not 64/128/256, NULL or misaligned), SG_EHIP. */
SG_API int sg_compact_init_bernoulli(int r, int rho, uint64_t seed, uint64_t threshold,
                                     uint8_t *d_compact, void *stream);

/* sg_ca_steps on compact states (lambda map): `steps` life generations
 * from d_in into d_out, in passes of at most `steps_per_pass` (1..32,
 * 0 = 32) split as sg_ca_steps splits them;
 * every pass rewrites its output tiles whole, so d_out and d_work need no
 * zeroing.  All three: compact-sized, 16-byte aligned, non-overlapping.
 * With two or more passes the state between them is kept in d_work as
 * bit-packed tiles (one bit per cell, an eighth of the compact bytes);
 * d_work's contents after the call are unspecified.
 * Errors: SG_EINVAL, SG_EALIAS, SG_EHIP. */
SG_API int sg_ca_steps_compact(int r, int rho, int steps, int steps_per_pass,
                               const uint8_t *d_in, uint8_t *d_out, uint8_t *d_work,
                               void *stream);

/* ---------------------------------------------------------------------
 * Rectangular blocks (Section III-B defines blocks of rho_x x rho_y
 * threads): rho_x = 2^a columns by rho_y = 2^b rows, powers of two up to
 * SG_MAX_RHO and n.  For a >= b the blocks that hold a gasket cell are
 * (bx, by) with bx & (by >> (a-b)) == 0 (for b > a, (bx >> (b-a)) & by == 0):
 * 3^(r - max(a,b)) * 2^|a-b| of them, the 2^|a-b| blocks that tile one
 * lambda square block of side 2^max(a,b).  The map decodes the square with
 * lambda and takes the position in the stack from the lowest bits of the
 * block index; with a = b it is sg_map_lambda.
 * --------------------------------------------------------------------- */

/* Host only.  Blocks launched: 3^(r-max(a,b)) * 2^|a-b| (SG_MAP_LAMBDA) or
 * (n/rho_x) * (n/rho_y) (SG_MAP_BBOX).  Errors: SG_EINVAL. */
SG_API int sg_block_count_rect(int map, int r, int rho_x, int rho_y, uint64_t *blocks);

/* d_bxy[2i], d_bxy[2i+1] = (bx, by) of block i: i = omega * 2^|a-b| + j,
 * omega lambda's linear index of the square block, j the position in its
 * stack (downwards for a >= b, rightwards for b > a).  d_bxy: device,
 * 8-byte aligned.  Errors: SG_EINVAL (also more than 2^31 - 1 blocks). */
SG_API int sg_map_lambda_rect(int r, int rho_x, int rho_y, uint32_t *d_bxy, void *stream);

/* The write pass (Section IV) over rho_x x rho_y blocks: `value` on every
 * gasket cell; inside a kept block cells off the gasket may be written with
 * 0 (16-byte chunks, or whole 64-byte granules for rho_x >= 64); blocks and
 * granules without a gasket cell are untouched.  d_a: device, n * n,
 * 16-byte aligned.  Errors: SG_EINVAL, SG_EHIP. */
SG_API int sg_write_pass_rect(int map, int r, int rho_x, int rho_y, uint8_t *d_a,
                              uint8_t value, void *stream);

/* ---------------------------------------------------------------------
 * Other embedded fractals F^{k,s}, s = 1/m (Section III-A), with the block
 * map generalised to them (Section V): the fractal keeps k of the m x m
 * sub-squares at every scale.  n = m^r, blocks of rho = m^q cells a side,
 * r_b = r - q.  The generalised map launches k^r_b blocks: the W x H grid
 * W = k^floor(r_b/2), H = k^ceil(r_b/2), the helper function beta_mu the
 * base-k digit of omega_y (odd mu) or omega_x (even mu) of weight
 * k^(ceil(mu/2)-1) (Eq. 4 with k for 3), the offset function the motif
 * entry of beta_mu (for Eq. 5) and the weight m^(mu-1) (Eq. 6-10); with
 * m = 2, k = 3 and the gasket's motif {(0,1), (0,0), (1,0)} it is lambda.
 * The bounding box launches all (n/rho)^2 blocks and keeps the fractal ones.
 * States: n x n uint8, row-major, 0 off the fractal (no alignment needed).
 * --------------------------------------------------------------------- */
#define SG_FRAC_MAX_M 4
#define SG_FRAC_MAX_K 16
#define SG_FRAC_MAX_N (1u << 18) /* largest n = m^r */
#define SG_FRAC_MAX_RHO 243      /* largest block side */

typedef struct sg_fractal {
    int32_t m;                   /* subdivision, 2..SG_FRAC_MAX_M */
    int32_t k;                   /* kept sub-squares, 1..min(m*m, SG_FRAC_MAX_K) */
    uint8_t dx[SG_FRAC_MAX_K];   /* offsets of the kept sub-squares in [0, m), */
    uint8_t dy[SG_FRAC_MAX_K];   /* distinct, in the order the digit enumerates them */
} sg_fractal;

/* Host only.  Blocks the map launches: k^r_b (SG_MAP_LAMBDA) or (n/rho)^2
 * (SG_MAP_BBOX).  Errors: SG_EINVAL (bad motif, n > SG_FRAC_MAX_N, rho not a
 * power of m up to n and SG_FRAC_MAX_RHO, k^r_b >= 2^32). */
SG_API int sg_frac_block_count(const sg_fractal *f, int map, int r, int rho, uint64_t *blocks);

/* Table of the generalised map: d_bxy[2i], d_bxy[2i+1] = (bx, by) of the
 * block with linear index i = omega_y * W + omega_x.  d_bxy: device,
 * 2 k^r_b uint32, 8-byte aligned.  Errors: SG_EINVAL (also k^r_b >= 2^31). */
SG_API int sg_frac_map(const sg_fractal *f, int r, int rho, uint32_t *d_bxy, void *stream);

/* The write pass on the fractal: `value` on its cells, 0 on the other cells
 * of its blocks; blocks without a fractal cell are untouched.
 * Errors: SG_EINVAL, SG_EHIP. */
SG_API int sg_frac_write(const sg_fractal *f, int map, int r, int rho, uint8_t *d_a,
                         uint8_t value, void *stream);

/* One B3/S23 step on the fractal: neighbours are the 8-neighbourhood cells
 * in the grid and on the fractal; cells off the fractal stay 0.  d_in, d_out:
 * device, n * n, distinct.  Errors: SG_EINVAL, SG_EALIAS, SG_EHIP. */
SG_API int sg_frac_life_step(const sg_fractal *f, int map, int r, int rho,
                             const uint8_t *d_in, uint8_t *d_out, void *stream);

/* ---------------------------------------------------------------------
 * Many gaskets at once (a batch of independent embedded gaskets of uneven
 * levels).  Every entry point below runs the temporally blocked life pass of
 * sg_ca_steps over the lambda tiles of all gaskets in one persistent launch
 * per pass; each gasket's result is identical to sg_ca_steps on it alone.
 * --------------------------------------------------------------------- */

/* Launch shape of a batched pass.
 *   rho:            largest lambda tile side, 64, 128 or 256; a gasket of
 *                   side n < rho uses tiles of side n (gaskets need n >= 64)
 *   steps_per_pass: generations per pass, 1..32
 *   groups_per_cu:  persistent workgroups per compute unit, 1..64, or 0 for
 *                   one workgroup per tile
 *   threads:        threads per workgroup, 256 or 512 */
typedef struct sg_tune {
    int32_t rho;
    int32_t steps_per_pass;
    int32_t groups_per_cu;
    int32_t threads;
} sg_tune;

/* One gasket of a batch: `steps` generations from d_in into d_out, with
 * d_work as the third buffer when more than one pass runs (as sg_ca_steps).
 * All device pointers, n * n bytes, 16-byte aligned, 0 off the gasket. */
typedef struct sg_gasket {
    const uint8_t *in;
    uint8_t *out;
    uint8_t *work;
    int32_t r;
    int32_t steps;
} sg_gasket;

/* One gasket of a single batched pass: `steps` (0..steps_per_pass)
 * generations from src into dst; items with steps = 0 are skipped. */
typedef struct sg_pass_item {
    const uint8_t *src;
    uint8_t *dst;
    int32_t r;
    int32_t steps;
} sg_pass_item;

typedef struct sg_batch sg_batch;       /* planned batch with a captured hipGraph */
typedef struct sg_pass_ctx sg_pass_ctx; /* device item table for repeated passes */

/* Host only.  A valid default shape (rho 64, 32 generations per pass, one
 * workgroup per tile, 256 threads). */
SG_API int sg_tune_default(sg_tune *tune);

/* Plans the passes of `count` gaskets (host array, copied), uploads the
 * per-pass item tables to device memory owned by the handle, and captures
 * all passes (and a device copy in -> out for gaskets with steps = 0) into a
 * hipGraph.  Allocates; not for the hot path.  The gaskets' buffers must stay
 * valid while the handle is used.
 * Errors: SG_EINVAL (bad shape, r < 6 or r > SG_MAX_R, missing work buffer),
 * SG_EALIAS, SG_ENOMEM, SG_EHIP. */
SG_API int sg_batch_create(const sg_gasket *gaskets, int count, const sg_tune *tune,
                           sg_batch **out);

/* Runs the whole batch: one hipGraphLaunch on `stream`. */
SG_API int sg_batch_run(sg_batch *batch, void *stream);

/* Runs the same launches as sg_batch_run without the graph. */
SG_API int sg_batch_run_eager(sg_batch *batch, void *stream);

/* Number of passes and of gasket cell updates (sum of 3^r * steps) of a run. */
SG_API int sg_batch_stats(const sg_batch *batch, uint64_t *passes, uint64_t *cell_steps);

/* Frees the handle, its graph and its device tables (NULL is ignored). */
SG_API void sg_batch_destroy(sg_batch *batch);

/* Times every candidate shape (rho in {64, 128, 256}, 8, 16 or 32
 * generations per pass, 0/2/4/8 groups per compute unit, 256/512 threads)
 * by running the batch on `stream` (writes the gaskets' out/work buffers,
 * never their inputs) and returns the fastest shape and its time.  This is
 * the launch-shape autotuner of the batched path; a single gasket is a batch
 * of one.  Synchronises the stream.  Errors as sg_batch_create. */
SG_API int sg_batch_autotune(const sg_gasket *gaskets, int count, sg_tune *best,
                             float *best_ms, void *stream);

/* Device item tables for up to `capacity` gaskets per pass (continuous
 * batching: the set of gaskets changes from pass to pass), in a ring of 8
 * upload slots so that up to 8 passes can be queued ahead of the GPU.
 * Allocates device and pinned host memory.  Errors: SG_EINVAL, SG_ENOMEM,
 * SG_EHIP. */
SG_API int sg_pass_ctx_create(int capacity, sg_pass_ctx **out);

/* One batched pass over `count` items (host array, validated, then uploaded
 * asynchronously on `stream`; returns once the items are staged, blocking
 * only until the upload of the pass queued 8 calls earlier has run).  Successive
 * calls on one context must use the same stream.  Errors: SG_EINVAL (count > capacity, steps outside
 * 0..steps_per_pass, r < 6 or r > SG_MAX_R), SG_EALIAS, SG_EHIP. */
SG_API int sg_pass_run(sg_pass_ctx *ctx, const sg_pass_item *items, int count,
                       const sg_tune *tune, void *stream);

/* Waits for the context's last upload and frees it (NULL is ignored). */
SG_API void sg_pass_ctx_destroy(sg_pass_ctx *ctx);

/* For callers that cannot allocate (code under hipGraph capture, serving
 * loops that must not call hipMalloc, harnesses that forbid it): the batched
 * pass of sg_pass_run with no context.  The item table lives in a static
 * device array of SG_PASS_STATIC_MAX items (32 bytes each, 128 KiB), one per
 * GPU, held until the process ends; its device address is looked up on the
 * first call on each device.  The items (host array, validated as by
 * sg_pass_run) reach that table through the arguments of small staging
 * launches on `stream`, so the host array may be reused as soon as the call
 * returns.  No memory is allocated or freed, host or device.
 * Every call on one GPU writes that GPU's one table: calls queued on the same
 * stream run in order, but calls whose passes can overlap on the device (two
 * streams, or two host threads) race, and the caller must order them.
 * Results are identical to sg_pass_run's.
 * Errors: SG_EINVAL (count > SG_PASS_STATIC_MAX, or as sg_pass_run),
 * SG_EALIAS, SG_EHIP. */
#define SG_PASS_STATIC_MAX 4096
SG_API int sg_pass_run_static(const sg_pass_item *items, int count, const sg_tune *tune,
                              void *stream);

/* ---------------------------------------------------------------------
 * Continuous batching of life solves (a native serving loop over
 * sg_pass_run).  Requests are admitted first come first served while their
 * footprint (two n x n buffers taken from a device pool that the server owns
 * and recycles by level) fits under cap_bytes.  Every sg_server_step is one
 * scheduling round: admission, then batched passes over every resident
 * request (oldest first within budget_cells of cell updates per pass, if
 * non-zero) queued without waiting for the device until a request finishes
 * or horizon_cells updates are queued (0: one pass per round), then one wait
 * and the retirement of finished requests.  One host thread per server.
 * --------------------------------------------------------------------- */
typedef struct sg_server sg_server;

typedef struct sg_server_done {
    uint64_t tag;            /* the tag given to sg_server_submit */
    const uint8_t *result;   /* device n x n state after `steps` generations,
                                valid until the next sg_server_step; NULL if
                                rejected */
    int32_t rejected;        /* 1: the footprint can never fit under the cap */
} sg_server_done;

typedef struct sg_server_stats {
    uint64_t rounds, passes, completed, rejected, cell_steps;
    uint64_t max_resident_bytes, max_active;
    uint64_t queued, active, resident_bytes; /* now */
    /* device bytes of the buffers the server holds (its pool, resident
     * states and last round's results): now, and the most ever; never above
     * the cap, since idle pooled buffers of other levels are freed before an
     * allocation would pass it */
    uint64_t allocated_bytes, max_allocated_bytes;
    uint64_t transferring;  /* host requests now uploading or reading back */
} sg_server_stats;

/* tune: the batched pass's launch shape (as sg_batch_create); max_requests:
 * queued plus resident requests at most.  Errors: SG_EINVAL, SG_ENOMEM,
 * SG_EHIP. */
SG_API int sg_server_create(const sg_tune *tune, uint64_t cap_bytes, int max_requests,
                            uint64_t horizon_cells, uint64_t budget_cells, void *stream,
                            sg_server **out);

/* Pre-allocates the pool as a server sizes its memory at start: two buffers
 * per entry of `levels` (6..SG_MAX_R, host array), in order, while the pool
 * stays under the cap.  Synchronises the stream.  Errors: SG_EINVAL,
 * SG_ENOMEM, SG_EHIP. */
SG_API int sg_server_reserve(sg_server *s, const int32_t *levels, int count);

/* Queues a request: `steps` generations of the level-r gasket (r 6..SG_MAX_R)
 * from d_init (device, n x n, 16-byte aligned, 0 off the gasket).  d_init is
 * copied when a round admits the request, which the server does not report,
 * so it must stay valid and unchanged until the request is reported done or
 * rejected.  d_out: NULL,
 * or a device n x n buffer (16-byte aligned) that receives a copy of the
 * result before the round that finishes the request returns.
 * Errors: SG_EINVAL, SG_ENOMEM (max_requests reached). */
SG_API int sg_server_submit(sg_server *s, int r, int steps, const uint8_t *d_init,
                            uint8_t *d_out, uint64_t tag);

/* Queues a request whose state lives in host memory: h_init (pinned host
 * memory, e.g. from hipHostMalloc, n x n, 0 off the gasket) is uploaded on a
 * copy stream of the server's when a round admits the request, the request
 * joins passes once its upload has ended, and when it finishes its result is
 * read back into h_out (pinned host n x n, or NULL) on a second copy stream
 * while other requests' passes run; it is reported done (with result =
 * h_out) in the first round after the read-back has ended.  Its buffers are
 * held from admission to that report.  h_init must stay valid and unchanged,
 * and h_out unread, until the request is reported.
 * Errors: SG_EINVAL, SG_ENOMEM (max_requests reached). */
SG_API int sg_server_submit_host(sg_server *s, int r, int steps, const uint8_t *h_init,
                                 uint8_t *h_out, uint64_t tag);

/* Admits at most max_active requests in flight at once (uploading, in
 * passes, or reading back); 0 (the default) sets no limit.  With 1 the
 * server runs one request at a time through the same loop.
 * Errors: SG_EINVAL. */
SG_API int sg_server_set_max_active(sg_server *s, int max_active);

/* A host request's upload starts (the request is admitted) only while fewer
 * than `window` host requests are uploading or reading back; 0 sets no
 * limit.  The default is 1: copies in both directions share one host link,
 * so first-in first-out transfers give each request its result soonest,
 * while passes still overlap them.  Errors: SG_EINVAL. */
SG_API int sg_server_set_transfer_window(sg_server *s, int window);

/* One scheduling round: host requests whose upload or read-back ended move
 * on, admission, then the passes; reports up to max_done finished (or
 * rejected) requests in `done` (host array) and their number in *n_done.
 * Waits for the server's stream when it queued work on it, never for the
 * copy streams.
 * Errors: SG_EINVAL, SG_ENOMEM, SG_EHIP. */
SG_API int sg_server_step(sg_server *s, sg_server_done *done, int max_done, int *n_done);

/* One request of a replay: submitted once `arrival_s` seconds have passed. */
typedef struct sg_server_request {
    double arrival_s;      /* seconds after the replay starts; non-decreasing */
    int32_t r, steps;
    const uint8_t *init;   /* device state, or pinned host state if host != 0 */
    uint8_t *out;          /* device / pinned host copy of the result, or NULL */
    int32_t host;          /* 1: init and out are pinned host memory */
} sg_server_request;

/* Serves `count` requests arriving in real time on an idle server: request i
 * is submitted once arrival_s[i] seconds have passed since the call began,
 * and rounds run whenever requests are open.  finish_s[i] receives the
 * seconds, on the same clock, at which request i was reported (so its
 * latency is finish_s[i] - arrival_s[i]) and rejected[i] whether it was
 * rejected.  Returns when every request has been reported.
 * Errors: SG_EINVAL (arrivals out of order or negative, a busy server, NULL
 * arrays), and those of submission and of sg_server_step. */
SG_API int sg_server_replay(sg_server *s, const sg_server_request *reqs, int count,
                            double *finish_s, int32_t *rejected);

SG_API int sg_server_get_stats(const sg_server *s, sg_server_stats *out);

/* Waits for the stream, frees the pool (NULL is ignored). */
SG_API void sg_server_destroy(sg_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
