/*
 * CPU oracle for "Block-space GPU Mapping for Embedded Sierpinski Gasket
 * Fractals" (Navarro, Bustos, Vega, Hitschfeld, arXiv 1706.04552).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library, and the HIP library
 * never calls it.
 *
 * Conventions (the readings are listed in the design notes):
 *  - n = 2^r is the side of the embedding array, stored row-major with pitch
 *    n; cell (x, y) is column x, row y, both 0-based.
 *  - Build frame: cell (x, y) belongs to the gasket iff (x & y) == 0.  The
 *    paper's own frame (Section III-D, "Bounding Sub-boxes") is
 *    x & (n-1-y) == 0, with the origin at the top-left and y growing
 *    downwards (Section III-B); the two frames differ by the reflection
 *    y -> n-1-y.
 *  - rho = 2^k is the block side, n_b = n / rho, r_b = r - k.
 *
 * Every routine loops over the whole array in the order of its definition,
 * except the gasket-only forms (sgo_life_step_sparse, the gasket graph and
 * its diffusion step), which visit only the 3^r gasket cells and are pinned
 * to the whole-array definitions cell for cell; they make full-size
 * references (r = 16 life, 500 diffusion steps at r = 14) take seconds.
 * Row loops carry an OpenMP pragma: rows are independent, so this changes no
 * result, only the wall time of the CPU baseline.
 *
 * Parity status of each function is stated in its comment; every function
 * here is pinned by an independent test (closed forms, exhaustive
 * enumeration, textbook patterns, hand-derived worked examples, an
 * independent sparse-matrix formulation).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* helpers                                                             */
/* ------------------------------------------------------------------ */

static int64_t pow3(int e)
{
    int64_t v = 1;
    for (int i = 0; i < e; ++i) v *= 3;
    return v;
}

/* ------------------------------------------------------------------ */
/* membership (Section I, Fig. 1-2; Section III-D)                    */
/* ------------------------------------------------------------------ */

/* Build frame.  Pinned by: the cell count equals 3^r (Eq. 2, Lemma 1) and
 * the mask equals the recursive three-copies construction (Section I). */
int sgo_member(int64_t x, int64_t y)
{
    return (x & y) == 0;
}

/* Paper frame, the bounding sub-box test of Section III-D with global
 * coordinates. */
int sgo_member_paper(int64_t n, int64_t x, int64_t y)
{
    return (x & (n - 1 - y)) == 0;
}

/* Number of gasket cells in the n x n array, by scanning every cell. */
int64_t sgo_count_cells(int r)
{
    int64_t n = (int64_t)1 << r, c = 0;
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            c += sgo_member(x, y);
    return c;
}

/* ------------------------------------------------------------------ */
/* lambda(omega), Theorem 1, Eq. 4-10                                  */
/* ------------------------------------------------------------------ */

/* Launch orthotope Pi^2 for block level r_b.  Eq. 4 reads the odd scale
 * levels mu = 1, 3, 5, ... from omega_y and the even ones from omega_x, so
 * omega_y needs ceil(r_b/2) ternary digits and omega_x floor(r_b/2):
 * W = 3^floor(r_b/2) columns, H = 3^ceil(r_b/2) rows (W*H = 3^r_b, the
 * packing of Lemma 2). */
void sgo_lambda_grid(int rb, int64_t *W, int64_t *H)
{
    *W = pow3(rb / 2);
    *H = pow3(rb - rb / 2);
}

/* Eq. 4: the region (0 top, 1 middle, 2 right) that block omega falls in at
 * scale level mu; integer floor division. */
static int64_t sgo_beta(int mu, int64_t wx, int64_t wy)
{
    int64_t v = wx * ((mu + 1) % 2) + wy * (mu % 2);
    int64_t den = pow3((mu + 1) / 2 - 1); /* 3^(ceil(mu/2) - 1) */
    return (v / den) % 3;
}

/* Eq. 5-10 in the paper frame: lambda_x = sum_mu Delta^x_mu 2^(mu-1),
 * lambda_y = sum_mu Delta^y_mu 2^(mu-1), mu = 1..r_b. */
void sgo_lambda(int rb, int64_t wx, int64_t wy, int64_t *lx, int64_t *ly)
{
    int64_t sx = 0, sy = 0;
    for (int mu = 1; mu <= rb; ++mu) {
        int64_t b = sgo_beta(mu, wx, wy);
        int64_t dx = b / 2;             /* Eq. 5, Delta^x */
        int64_t dy = b - b / 2;         /* Eq. 5, Delta^y */
        int64_t off = (int64_t)1 << (mu - 1);
        sx += dx * off;                 /* Eq. 6 and Eq. 9 */
        sy += dy * off;                 /* Eq. 7 and Eq. 10 */
    }
    *lx = sx;
    *ly = sy;
}

/* Table of lambda in the build frame: for omega = (wx, wy) at linear index
 * wy*W + wx, out[2i] = bx = lambda_x and out[2i+1] = by = n_b-1-lambda_y.
 * Pinned by: exhaustive bijection onto {bx & by == 0}, hand-derived worked
 * tables for r_b = 1, 2, 3. */
void sgo_map_lambda(int rb, uint32_t *out)
{
    int64_t W, H, nb = (int64_t)1 << rb;
    sgo_lambda_grid(rb, &W, &H);
    for (int64_t wy = 0; wy < H; ++wy)
        for (int64_t wx = 0; wx < W; ++wx) {
            int64_t lx, ly, i = wy * W + wx;
            sgo_lambda(rb, wx, wy, &lx, &ly);
            out[2 * i] = (uint32_t)lx;
            out[2 * i + 1] = (uint32_t)(nb - 1 - ly);
        }
}

/* ------------------------------------------------------------------ */
/* bounding-box map (Section I, Fig. 3)                                */
/* ------------------------------------------------------------------ */

/* mask[by*n_b + bx] = 1 iff block (bx, by) of the n_b x n_b bounding box
 * holds at least one gasket cell, i.e. iff the identity map keeps at least
 * one of its threads.  Found by scanning every cell of every block. */
void sgo_map_bbox(int r, int rho, uint8_t *mask)
{
    int64_t n = (int64_t)1 << r, nb = n / rho;
#pragma omp parallel for schedule(static)
    for (int64_t by = 0; by < nb; ++by)
        for (int64_t bx = 0; bx < nb; ++bx) {
            int keep = 0;
            for (int64_t ty = 0; ty < rho; ++ty)
                for (int64_t tx = 0; tx < rho; ++tx)
                    keep |= sgo_member(bx * rho + tx, by * rho + ty);
            mask[by * nb + bx] = (uint8_t)keep;
        }
}

/* ------------------------------------------------------------------ */
/* write pass (Section IV): a constant on every gasket element          */
/* ------------------------------------------------------------------ */

/* a[y][x] = value on gasket cells and 0 elsewhere. */
void sgo_write_pass(int r, uint8_t value, uint8_t *a)
{
    int64_t n = (int64_t)1 << r;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            a[y * n + x] = sgo_member(x, y) ? value : 0;
}

/* ------------------------------------------------------------------ */
/* B3/S23 life on the gasket                                           */
/* ------------------------------------------------------------------ */

/* Plain B3/S23 on a w x h grid, all cells live, cells outside the grid dead.
 * Pinned by textbook patterns (still lifes, oscillators, glider). */
void sgo_life_step_plain(int64_t w, int64_t h, const uint8_t *in, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            int c = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t xx = x + dx, yy = y + dy;
                    if ((dx || dy) && xx >= 0 && xx < w && yy >= 0 && yy < h)
                        c += in[yy * w + xx] != 0;
                }
            int self = in[y * w + x] != 0;
            out[y * w + x] = (uint8_t)(c == 3 || (self && c == 2));
        }
}

/* One B3/S23 step on the gasket: neighbours are the 8-neighbourhood cells
 * that lie in the grid and in the gasket; cells off the gasket stay 0.
 * Pinned by: hand-derived worked steps at r = 2, equality with the plain
 * rule masked by membership, an independent neighbour-list formulation. */
void sgo_life_step(int r, const uint8_t *in, uint8_t *out)
{
    int64_t n = (int64_t)1 << r;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x) {
            if (!sgo_member(x, y)) {
                out[y * n + x] = 0;
                continue;
            }
            int c = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t xx = x + dx, yy = y + dy;
                    if ((dx || dy) && xx >= 0 && xx < n && yy >= 0 && yy < n &&
                        sgo_member(xx, yy))
                        c += in[yy * n + xx] != 0;
                }
            int self = in[y * n + x] != 0;
            out[y * n + x] = (uint8_t)(c == 3 || (self && c == 2));
        }
}

/* The same step visiting the gasket's cells only.  Row y of the gasket holds
 * exactly the cells whose column x shares no bit with y, i.e. the submasks of
 * m = ~y & (n-1); they are enumerated in increasing order by x <- (x - m) & m
 * (subtracting m adds one in the positions m keeps and lets the carry jump
 * the others).  Each gasket cell counts its 8 neighbours as in
 * sgo_life_step.  Cells off the gasket of `out` are not written: the caller
 * keeps them 0.  3^r cells per step instead of 4^r.
 * Pinned by: equality with sgo_life_step on every state at r = 2 and on
 * random states up to r = 10. */
void sgo_life_step_sparse(int r, const uint8_t *in, uint8_t *out)
{
    int64_t n = (int64_t)1 << r;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t y = 0; y < n; ++y) {
        const int64_t m = ~y & (n - 1);
        for (int64_t x = 0;; x = (x - m) & m) {
            int c = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t xx = x + dx, yy = y + dy;
                    if ((dx || dy) && xx >= 0 && xx < n && yy >= 0 && yy < n &&
                        sgo_member(xx, yy))
                        c += in[yy * n + xx] != 0;
                }
            int self = in[y * n + x] != 0;
            out[y * n + x] = (uint8_t)(c == 3 || (self && c == 2));
            if (x == m) break;
        }
    }
}

/* `steps` gasket life steps applied to a region of the grid: the gw x gh
 * cells whose top-left cell is (gx0, gy0), held row-major in `a` and updated
 * in place, with every cell outside the region taken as dead.  The region
 * must lie inside the grid (its edges there are the grid's real boundary);
 * where it is cut short of the grid's edge, the cells within Chebyshev
 * distance `steps` of the cut come out wrong. */
void sgo_life_region(int64_t gx0, int64_t gy0, int64_t gw, int64_t gh, int steps, uint8_t *a)
{
    uint8_t *b = (uint8_t *)malloc((size_t)(gw * gh));
    uint8_t *cur = a, *nxt = b;
    for (int t = 0; t < steps; ++t) {
        for (int64_t y = 0; y < gh; ++y)
            for (int64_t x = 0; x < gw; ++x) {
                int64_t X = gx0 + x, Y = gy0 + y;
                if (!sgo_member(X, Y)) {
                    nxt[y * gw + x] = 0;
                    continue;
                }
                int c = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t xx = x + dx, yy = y + dy;
                        if ((dx || dy) && xx >= 0 && xx < gw && yy >= 0 && yy < gh &&
                            sgo_member(gx0 + xx, gy0 + yy))
                            c += cur[yy * gw + xx] != 0;
                    }
                int self = cur[y * gw + x] != 0;
                nxt[y * gw + x] = (uint8_t)(c == 3 || (self && c == 2));
            }
        uint8_t *s = cur; cur = nxt; nxt = s;
    }
    if (cur != a)
        memcpy(a, cur, (size_t)(gw * gh));
    free(b);
}

/* `steps` gasket life steps evaluated on the window [x0, x0+w) x [y0, y0+h)
 * of a full n x n state.  A cell after t steps depends only on cells within
 * Chebyshev distance t, so the window grown by `steps` on every side (and
 * clipped to the grid, whose edges are real boundaries) holds everything the
 * result depends on; the rule is applied to that region with cells outside
 * it taken as dead, and the wrong values this makes at the region's cut
 * edges travel inward one cell per step, never reaching the window. */
void sgo_life_window(int r, const uint8_t *in, int64_t x0, int64_t y0,
                     int64_t w, int64_t h, int steps, uint8_t *out)
{
    int64_t n = (int64_t)1 << r;
    int64_t gx0 = x0 - steps < 0 ? 0 : x0 - steps;
    int64_t gy0 = y0 - steps < 0 ? 0 : y0 - steps;
    int64_t gx1 = x0 + w + steps > n ? n : x0 + w + steps;
    int64_t gy1 = y0 + h + steps > n ? n : y0 + h + steps;
    int64_t gw = gx1 - gx0, gh = gy1 - gy0;
    uint8_t *a = (uint8_t *)malloc((size_t)(gw * gh));
    for (int64_t y = 0; y < gh; ++y)
        memcpy(a + y * gw, in + (gy0 + y) * n + gx0, (size_t)gw);
    sgo_life_region(gx0, gy0, gw, gh, steps, a);
    for (int64_t y = 0; y < h; ++y)
        memcpy(out + y * w, a + (y0 - gy0 + y) * gw + (x0 - gx0), (size_t)w);
    free(a);
}

/* Per-row checksums of a u8 state: xr[y] = XOR over the row, pop[y] = sum of
 * the popcounts of the row's bytes. */
void sgo_row_checksums(int r, const uint8_t *a, uint8_t *xr, uint32_t *pop)
{
    int64_t n = (int64_t)1 << r;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y) {
        uint8_t x8 = 0;
        uint32_t p = 0;
        for (int64_t x = 0; x < n; ++x) {
            uint8_t v = a[y * n + x];
            x8 ^= v;
            for (int b = 0; b < 8; ++b) p += (v >> b) & 1u;
        }
        xr[y] = x8;
        pop[y] = p;
    }
}

/* ------------------------------------------------------------------ */
/* explicit diffusion on the gasket, FP64                              */
/* ------------------------------------------------------------------ */

/* One step of u' = u + alpha * sum_{nb}(u_nb - u), the sum running over the
 * 4-neighbours W, E, N, S (in that order) that lie in the grid and in the
 * gasket; cells off the gasket are held at 0 and never enter a sum.
 * Pinned by: equality with (I - alpha L)^t u0 for the graph Laplacian L of
 * the gasket's 4-adjacency graph (independent sparse formulation), exact
 * conservation of the total, the maximum principle, constant fields, and a
 * hand-derived two-step example at r = 1. */
void sgo_diffuse_step(int r, const double *in, double *out, double alpha)
{
    int64_t n = (int64_t)1 << r;
    static const int DX[4] = {-1, 1, 0, 0}; /* W, E, N, S */
    static const int DY[4] = {0, 0, -1, 1};
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x) {
            if (!sgo_member(x, y)) {
                out[y * n + x] = 0.0;
                continue;
            }
            double u = in[y * n + x], s = 0.0;
            for (int k = 0; k < 4; ++k) {
                int64_t xx = x + DX[k], yy = y + DY[k];
                if (xx >= 0 && xx < n && yy >= 0 && yy < n && sgo_member(xx, yy))
                    s += in[yy * n + xx] - u;
            }
            out[y * n + x] = u + alpha * s;
        }
}

/* The gasket as a graph.  Its cells numbered in row-major order: row y holds
 * 2^(r - popcount(y)) cells (the submasks of ~y), so the cells of rows
 * before y number rowstart(y) = sum over y' < y of those, and cell (x, y)
 * is number rowstart(y) + the rank of x among the submasks of ~y, which is
 * x's bits at the positions where ~y has ones, packed together.
 * pos[i] = y * n + x of cell number i; nb[4 i + k] = the number of its
 * neighbour k (W, E, N, S) if that neighbour is in the grid and on the
 * gasket, else -1.  pos: 3^r entries, nb: 4 * 3^r.
 * Pinned by: diffusion over this graph equals sgo_diffuse_step bit for bit. */
static int64_t sgo_pack_bits(int64_t x, int64_t m)
{
    int64_t v = 0, bit = 1;
    for (int64_t b = 1; b <= m; b <<= 1)
        if (m & b) {
            if (x & b) v |= bit;
            bit <<= 1;
        }
    return v;
}

void sgo_gasket_graph(int r, int64_t *pos, int32_t *nb)
{
    int64_t n = (int64_t)1 << r;
    int64_t *rowstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    rowstart[0] = 0;
    for (int64_t y = 0; y < n; ++y) {
        int pc = 0;
        for (int b = 0; b < r; ++b) pc += (int)((y >> b) & 1);
        rowstart[y + 1] = rowstart[y] + ((int64_t)1 << (r - pc));
    }
    static const int DX[4] = {-1, 1, 0, 0}; /* W, E, N, S */
    static const int DY[4] = {0, 0, -1, 1};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t y = 0; y < n; ++y) {
        const int64_t m = ~y & (n - 1);
        int64_t i = rowstart[y];
        for (int64_t x = 0;; x = (x - m) & m, ++i) {
            pos[i] = y * n + x;
            for (int k = 0; k < 4; ++k) {
                int64_t xx = x + DX[k], yy = y + DY[k];
                int32_t j = -1;
                if (xx >= 0 && xx < n && yy >= 0 && yy < n && sgo_member(xx, yy))
                    j = (int32_t)(rowstart[yy] + sgo_pack_bits(xx, ~yy & (n - 1)));
                nb[4 * i + k] = j;
            }
            if (x == m) break;
        }
    }
    free(rowstart);
}

/* One FP64 diffusion step over the gasket graph: u'_i = u_i + alpha *
 * sum_k (u_nb(i,k) - u_i) over the neighbours k = W, E, N, S that exist, in
 * that order (the sum of sgo_diffuse_step, term for term).  u, out: the N
 * gasket cells in the graph's numbering. */
void sgo_diffuse_step_graph(int64_t N, const int32_t *nb, const double *in, double *out,
                            double alpha)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double u = in[i], s = 0.0;
        for (int k = 0; k < 4; ++k) {
            int32_t j = nb[4 * i + k];
            if (j >= 0) s += in[j] - u;
        }
        out[i] = u + alpha * s;
    }
}

/* `steps` FP64 diffusion steps on a window of a full FP32 initial state, by
 * the same locality argument as sgo_life_window (the 4-neighbour stencil
 * spreads one cell per step).  The FP32 input is widened exactly. */
void sgo_diffuse_window(int r, const float *in, int64_t x0, int64_t y0,
                        int64_t w, int64_t h, int steps, double alpha,
                        double *out)
{
    int64_t n = (int64_t)1 << r;
    static const int DX[4] = {-1, 1, 0, 0};
    static const int DY[4] = {0, 0, -1, 1};
    int64_t gx0 = x0 - steps < 0 ? 0 : x0 - steps;
    int64_t gy0 = y0 - steps < 0 ? 0 : y0 - steps;
    int64_t gx1 = x0 + w + steps > n ? n : x0 + w + steps;
    int64_t gy1 = y0 + h + steps > n ? n : y0 + h + steps;
    int64_t gw = gx1 - gx0, gh = gy1 - gy0;
    double *a = (double *)malloc(sizeof(double) * (size_t)(gw * gh));
    double *b = (double *)malloc(sizeof(double) * (size_t)(gw * gh));
    for (int64_t y = 0; y < gh; ++y)
        for (int64_t x = 0; x < gw; ++x)
            a[y * gw + x] = (double)in[(gy0 + y) * n + gx0 + x];
    for (int t = 0; t < steps; ++t) {
        for (int64_t y = 0; y < gh; ++y)
            for (int64_t x = 0; x < gw; ++x) {
                if (!sgo_member(gx0 + x, gy0 + y)) {
                    b[y * gw + x] = 0.0;
                    continue;
                }
                double u = a[y * gw + x], s = 0.0;
                for (int k = 0; k < 4; ++k) {
                    int64_t xx = x + DX[k], yy = y + DY[k];
                    if (xx >= 0 && xx < gw && yy >= 0 && yy < gh &&
                        sgo_member(gx0 + xx, gy0 + yy))
                        s += a[yy * gw + xx] - u;
                }
                b[y * gw + x] = u + alpha * s;
            }
        double *s = a; a = b; b = s;
    }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x)
            out[y * w + x] = a[(y0 - gy0 + y) * gw + (x0 - gx0 + x)];
    free(a);
    free(b);
}

/* ------------------------------------------------------------------ */
/* rectangular blocks rho_x x rho_y (Section III-B)                    */
/* ------------------------------------------------------------------ */

/* Blocks of rho_x = 2^a columns by rho_y = 2^b rows.  For a >= b, a block
 * (bx, by) holds a gasket cell iff bx & (by >> (a-b)) == 0: its columns' bits
 * below a are free, so only the bits at and above a must be disjoint; the
 * 2^(a-b) blocks stacked in one 2^a x 2^a square are all kept or all not.
 * The map decodes the square block by lambda at level r - a (linear order
 * omega_sq = wy * W + wx) and the position in the stack as the 2^(a-b)
 * lowest values of omega: omega = omega_sq * 2^(a-b) + j, by = by_sq * 2^(a-b)
 * + j.  For b > a the roles of x and y swap.  With a = b it is lambda.
 * out[2i], out[2i+1] = (bx, by).  Pinned by: exhaustive bijection onto the
 * blocks that hold gasket cells, the count 3^(r - max) 2^|a - b|, equality
 * with sgo_map_lambda for a = b. */
void sgo_map_lambda_rect(int r, int a, int b, uint32_t *out)
{
    int hi = a > b ? a : b, d = a > b ? a - b : b - a;
    int rb = r - hi;
    int64_t W, H, nb = (int64_t)1 << rb, stack = (int64_t)1 << d;
    sgo_lambda_grid(rb, &W, &H);
    for (int64_t wy = 0; wy < H; ++wy)
        for (int64_t wx = 0; wx < W; ++wx) {
            int64_t lx, ly, sq = wy * W + wx;
            sgo_lambda(rb, wx, wy, &lx, &ly);
            int64_t bx = lx, by = nb - 1 - ly;
            for (int64_t j = 0; j < stack; ++j) {
                int64_t i = sq * stack + j;
                out[2 * i] = (uint32_t)(a >= b ? bx : bx * stack + j);
                out[2 * i + 1] = (uint32_t)(a >= b ? by * stack + j : by);
            }
        }
}

/* mask[by * (n/rho_x) + bx] = 1 iff the rho_x x rho_y block holds a gasket
 * cell, found by scanning its cells. */
void sgo_map_bbox_rect(int r, int rho_x, int rho_y, uint8_t *mask)
{
    int64_t n = (int64_t)1 << r, nbx = n / rho_x, nby = n / rho_y;
#pragma omp parallel for schedule(static)
    for (int64_t by = 0; by < nby; ++by)
        for (int64_t bx = 0; bx < nbx; ++bx) {
            int keep = 0;
            for (int64_t ty = 0; ty < rho_y; ++ty)
                for (int64_t tx = 0; tx < rho_x; ++tx)
                    keep |= sgo_member(bx * rho_x + tx, by * rho_y + ty);
            mask[by * nbx + bx] = (uint8_t)keep;
        }
}

/* ------------------------------------------------------------------ */
/* other embedded fractals F^{k,s} (Section III-A; Section V)          */
/* ------------------------------------------------------------------ */

/* A fractal built by replicating k copies of itself at scale s = 1/m
 * (Section III-A): the m x m sub-squares kept at every scale are given by a
 * motif, sub-square i at offset (fdx[i], fdy[i]) in [0, m)^2, all distinct,
 * listed in the order the map's digit enumerates them.  n = m^r.  A cell
 * (x, y) belongs to the level-r fractal iff at every scale the pair of its
 * base-m digits is a kept offset.  The gasket is m = 2, k = 3 with the
 * offsets {(0,0), (1,0), (0,1)} (build frame). */

static int64_t ipow(int64_t b, int e)
{
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

static int sgo_frac_kept(int m, int k, const int *fdx, const int *fdy, int64_t dx, int64_t dy)
{
    (void)m;
    for (int i = 0; i < k; ++i)
        if (fdx[i] == dx && fdy[i] == dy) return 1;
    return 0;
}

/* Membership by digits.  Pinned by: brute-force recursive construction,
 * cell count k^r, the gasket motif against (x & y) == 0, the carpet against
 * its textbook definition. */
int sgo_frac_member(int m, int k, const int *fdx, const int *fdy, int r, int64_t x, int64_t y)
{
    for (int j = 0; j < r; ++j) {
        if (!sgo_frac_kept(m, k, fdx, fdy, x % m, y % m)) return 0;
        x /= m;
        y /= m;
    }
    return 1;
}

/* The generalised block map: the W x H grid W = k^floor(rb/2),
 * H = k^ceil(rb/2) (Eq. 4 with 3 replaced by k); at scale level mu the
 * helper function beta_mu is the base-k digit of omega_y (odd mu) or
 * omega_x (even mu) of weight k^(ceil(mu/2)-1) (Eq. 4), the offset
 * function is the motif entry (Delta^x, Delta^y) = motif[beta_mu] (Eq. 5)
 * and the weight function is m^(mu-1) (Eq. 6-7):
 * lambda = sum_mu Delta_mu m^(mu-1) (Eq. 8-10).  Build frame (the motif is
 * given in it, so no reflection).  Pinned by: the gasket motif reproduces
 * sgo_map_lambda; exhaustive bijection onto the fractal blocks. */
void sgo_frac_lambda(int m, int k, const int *fdx, const int *fdy, int rb, int64_t wx,
                     int64_t wy, int64_t *lx, int64_t *ly)
{
    int64_t sx = 0, sy = 0;
    for (int mu = 1; mu <= rb; ++mu) {
        int64_t v = (mu % 2) ? wy : wx;
        int64_t b = (v / ipow(k, (mu + 1) / 2 - 1)) % k;
        int64_t off = ipow(m, mu - 1);
        sx += fdx[b] * off;
        sy += fdy[b] * off;
    }
    *lx = sx;
    *ly = sy;
}

/* Table of the generalised map: out[2i], out[2i+1] = (bx, by) of the block
 * at linear index i = wy * W + wx. */
void sgo_frac_map(int m, int k, const int *fdx, const int *fdy, int rb, uint32_t *out)
{
    int64_t W = ipow(k, rb / 2), H = ipow(k, rb - rb / 2);
    for (int64_t wy = 0; wy < H; ++wy)
        for (int64_t wx = 0; wx < W; ++wx) {
            int64_t lx, ly, i = wy * W + wx;
            sgo_frac_lambda(m, k, fdx, fdy, rb, wx, wy, &lx, &ly);
            out[2 * i] = (uint32_t)lx;
            out[2 * i + 1] = (uint32_t)ly;
        }
}

/* a[y][x] = value on the fractal's cells, 0 elsewhere (n = m^r). */
void sgo_frac_write(int m, int k, const int *fdx, const int *fdy, int r, uint8_t value,
                    uint8_t *a)
{
    int64_t n = ipow(m, r);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            a[y * n + x] = sgo_frac_member(m, k, fdx, fdy, r, x, y) ? value : 0;
}

/* Rows [y0, y0 + rows) of sgo_frac_write's result, into out (rows x n). */
void sgo_frac_write_rows(int m, int k, const int *fdx, const int *fdy, int r, uint8_t value,
                         int64_t y0, int64_t rows, uint8_t *out)
{
    int64_t n = ipow(m, r);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < rows; ++y)
        for (int64_t x = 0; x < n; ++x)
            out[y * n + x] = sgo_frac_member(m, k, fdx, fdy, r, x, y0 + y) ? value : 0;
}

/* One B3/S23 step on the fractal: neighbours are the 8-neighbourhood cells in
 * the grid and in the fractal; cells off the fractal stay 0.  Pinned by the
 * gasket motif against sgo_life_step and an independent neighbour-list
 * formulation. */
void sgo_frac_life_step(int m, int k, const int *fdx, const int *fdy, int r, const uint8_t *in,
                        uint8_t *out)
{
    int64_t n = ipow(m, r);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x) {
            if (!sgo_frac_member(m, k, fdx, fdy, r, x, y)) {
                out[y * n + x] = 0;
                continue;
            }
            int c = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t xx = x + dx, yy = y + dy;
                    if ((dx || dy) && xx >= 0 && xx < n && yy >= 0 && yy < n &&
                        sgo_frac_member(m, k, fdx, fdy, r, xx, yy))
                        c += in[yy * n + xx] != 0;
                }
            int self = in[y * n + x] != 0;
            out[y * n + x] = (uint8_t)(c == 3 || (self && c == 2));
        }
}

/* `steps` fractal life steps on the window [x0, x0+w) x [y0, y0+h) of a full
 * n x n state, from the window grown by `steps` cells on every side (clipped
 * to the grid): a cell after t steps depends only on cells within Chebyshev
 * distance t, and the wrong values at the region's cut edges travel inward
 * one cell per step.  Membership is taken at the cells' global coordinates.
 * Pinned by equality with full runs. */
void sgo_frac_life_window(int m, int k, const int *fdx, const int *fdy, int r,
                          const uint8_t *in, int64_t x0, int64_t y0, int64_t w, int64_t h,
                          int steps, uint8_t *out)
{
    int64_t n = ipow(m, r);
    int64_t gx0 = x0 - steps < 0 ? 0 : x0 - steps, gy0 = y0 - steps < 0 ? 0 : y0 - steps;
    int64_t gx1 = x0 + w + steps > n ? n : x0 + w + steps;
    int64_t gy1 = y0 + h + steps > n ? n : y0 + h + steps;
    int64_t gw = gx1 - gx0, gh = gy1 - gy0;
    uint8_t *a = (uint8_t *)malloc((size_t)(gw * gh));
    uint8_t *b = (uint8_t *)malloc((size_t)(gw * gh));
    for (int64_t y = 0; y < gh; ++y)
        for (int64_t x = 0; x < gw; ++x)
            a[y * gw + x] = in[(gy0 + y) * n + (gx0 + x)];
    for (int s = 0; s < steps; ++s) {
        for (int64_t y = 0; y < gh; ++y)
            for (int64_t x = 0; x < gw; ++x) {
                int64_t X = gx0 + x, Y = gy0 + y;
                if (!sgo_frac_member(m, k, fdx, fdy, r, X, Y)) {
                    b[y * gw + x] = 0;
                    continue;
                }
                int c = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t xx = x + dx, yy = y + dy;
                        if ((dx || dy) && xx >= 0 && xx < gw && yy >= 0 && yy < gh &&
                            sgo_frac_member(m, k, fdx, fdy, r, gx0 + xx, gy0 + yy))
                            c += a[yy * gw + xx] != 0;
                    }
                int self = a[y * gw + x] != 0;
                b[y * gw + x] = (uint8_t)(c == 3 || (self && c == 2));
            }
        uint8_t *t = a;
        a = b;
        b = t;
    }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x)
            out[y * w + x] = a[(y0 - gy0 + y) * gw + (x0 - gx0 + x)];
    free(a);
    free(b);
}

/* Number of threads the OpenMP row loops above use. */
#ifdef _OPENMP
#include <omp.h>
int sgo_threads(void) { return omp_get_max_threads(); }
/* Sets the number of threads of the row loops (the CPU baseline is timed on
 * one core and on all of them). */
void sgo_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
#else
int sgo_threads(void) { return 1; }
void sgo_set_threads(int t) { (void)t; }
#endif
