/*
 * Plain sequential CPU definition of the displace+render frame.
 *
 * TEST INFRASTRUCTURE: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code. It is deliberately slow
 * and literal: one point at a time, one pixel at a time, no blocking, no
 * fusion. Each function names the passage (of the Mimir paper, or of the
 * Philox paper) that it follows, and every reading taken where the paper is
 * silent is marked "Reading".
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * With -ffp-contract=off each binary32 operation below rounds on its own,
 * so the order written here is the order of roundings.
 */
#include "mm_oracle.h"

#include <math.h>
#include <stddef.h>

/* Philox4x32 round multipliers and Weyl key increments, as given for N=4,
 * W=32 in the SC'11 paper's definition of Philox. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* Reading: counter word 1 tags what a draw is for, so that the streams of
 * the displacement and of the colour hash never overlap. */
#define TAG_DISPLACE 0u
#define TAG_COLOUR 2u

static const uint64_t EMPTY_KEY = 0xFFFFFFFFFFFFFFFFull;

/* Philox-4x32: each round multiplies words 0 and 2 by the round
 * multipliers (full 64-bit products), and the new block is
 * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)). The key
 * is bumped by the Weyl increments between rounds; ten rounds in all. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void oracle_philox4x32_10_many(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n)
{
    for (uint64_t j = 0; j < n; ++j)
        oracle_philox4x32_10(ctr + 4 * j, key + 2 * j, out + 4 * j);
}

/* Reading of the displacement law. The paper moves points by Brownian
 * motion drawn in a CUDA kernel (section "Performance Benchmark"); the
 * workload here draws a uniform offset in [-a, a) per coordinate instead.
 * The top 24 bits k of the word index the grid k * 2^-23 - 1 of [-1, 1),
 * which binary32 holds exactly; the only rounding is the product with a. */
float oracle_offset(uint32_t r, float a)
{
    uint32_t k = r >> 8;
    float t = (float)k * 0x1p-23f - 1.0f;
    return t * a;
}

void oracle_offset_many(const uint32_t* r, uint64_t n, float a, float* out)
{
    for (uint64_t j = 0; j < n; ++j)
        out[j] = oracle_offset(r[j], a);
}

/* Reading: the 2D point box is the periodic square [-1, 1)^2. One fold is
 * enough for |x| < 2, and both folds are exact (Sterbenz). */
float oracle_wrap(float x)
{
    if (x >= 1.0f)
        return x - 2.0f;
    if (x < -1.0f)
        return x + 2.0f;
    return x;
}

/* The per-timestep displacement kernel of section "Performance Benchmark",
 * written as a loop over points: the new position depends only on the old
 * position of the same point and on (seed, index, step). */
void oracle_displace(float* pos, uint64_t n, uint32_t dim, uint64_t seed,
                     uint32_t step, float a, int wrap)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {step, TAG_DISPLACE, (uint32_t)i, (uint32_t)(i >> 32)};
        uint32_t r[4];
        oracle_philox4x32_10(ctr, key, r);
        for (uint32_t c = 0; c < dim; ++c) {
            float x = pos[i * dim + c] + oracle_offset(r[c], a);
            if (wrap)
                x = oracle_wrap(x);
            pos[i * dim + c] = x;
        }
    }
}

/* Reading of the view transform. A view carries a model transform and a
 * camera (section "Views"); here both are folded into one row-major float32
 * matrix m. Clip coordinates are rows 0, 1 and 3 of m times (x, y, z, 1),
 * summed left to right. The near test is w > 0.1; normalised device x, y in
 * [-1, 1] map to the screen with y up, and the pixel row counts down from
 * the top. 2D domain: x, y are already normalised, depth is 0. */
int oracle_project(const float* p, uint32_t dim, const float m[16],
                   uint32_t width, uint32_t height,
                   int32_t* px, int32_t* py, uint32_t* depth_bits)
{
    const float half_w = (float)(width / 2u);
    const float half_h = (float)(height / 2u);
    float sx, sy;
    uint32_t bits = 0u;
    if (dim == 2u) {
        sx = (p[0] + 1.0f) * half_w;
        sy = (p[1] + 1.0f) * half_h;
    } else {
        const float x = p[0], y = p[1], z = p[2];
        float cx = m[0] * x;
        cx = cx + m[1] * y;
        cx = cx + m[2] * z;
        cx = cx + m[3];
        float cy = m[4] * x;
        cy = cy + m[5] * y;
        cy = cy + m[6] * z;
        cy = cy + m[7];
        float cw = m[12] * x;
        cw = cw + m[13] * y;
        cw = cw + m[14] * z;
        cw = cw + m[15];
        if (!(cw > 0.1f))
            return 0;
        const float inv_w = 1.0f / cw;
        sx = (cx * inv_w + 1.0f) * half_w;
        sy = (cy * inv_w + 1.0f) * half_h;
        /* cw > 0, so its bit pattern orders like its value. */
        union {
            float f;
            uint32_t u;
        } pun;
        pun.f = cw;
        bits = pun.u;
    }
    if (!(sx >= 0.0f && sx < (float)width && sy >= 0.0f && sy < (float)height))
        return 0;
    *px = (int32_t)floorf(sx);
    *py = (int32_t)height - 1 - (int32_t)floorf(sy);
    *depth_bits = bits;
    return 1;
}

void oracle_project_many(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                         uint32_t width, uint32_t height, int64_t* pixel)
{
    for (uint64_t i = 0; i < n; ++i) {
        int32_t px, py;
        uint32_t bits;
        pixel[i] = oracle_project(pos + i * dim, dim, m, width, height, &px, &py, &bits)
                       ? (int64_t)py * width + px : -1;
    }
}

/* Markers of one size (section "Performance Benchmark") drawn as a square
 * footprint of 1 or 3 pixels a side. Each covered pixel keeps the smallest
 * (depth, index) key: the nearest point wins, and equal depths go to the
 * smaller index. */
void oracle_splat(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                  uint32_t width, uint32_t height, uint32_t footprint,
                  uint64_t* depth, const uint64_t* order)
{
    const int32_t reach = (int32_t)(footprint / 2u);
    for (uint64_t j = 0; j < n; ++j) {
        const uint64_t i = order ? order[j] : j;
        int32_t px, py;
        uint32_t bits;
        if (!oracle_project(pos + i * dim, dim, m, width, height, &px, &py, &bits))
            continue;
        const uint64_t key = ((uint64_t)bits << 32) | (uint64_t)(uint32_t)i;
        for (int32_t dy = -reach; dy <= reach; ++dy) {
            for (int32_t dx = -reach; dx <= reach; ++dx) {
                const int32_t qx = px + dx, qy = py + dy;
                if (qx < 0 || qy < 0 || qx >= (int32_t)width || qy >= (int32_t)height)
                    continue;
                uint64_t* slot = depth + (uint64_t)qy * width + (uint64_t)qx;
                if (key < *slot)
                    *slot = key;
            }
        }
    }
}

/* Reading: "colour is a 32-bit hash of the point index" is taken as the
 * first Philox word of a counter tagged for colour, with opaque alpha. */
uint32_t oracle_colour(uint32_t index, uint64_t seed)
{
    const uint32_t ctr[4] = {0u, TAG_COLOUR, index, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    return r[0] | 0xFF000000u;
}

void oracle_resolve(uint64_t* depth, uint32_t* colour, uint64_t npix, uint64_t seed)
{
    for (uint64_t q = 0; q < npix; ++q) {
        const uint64_t k = depth[q];
        colour[q] = (k == EMPTY_KEY) ? 0u : oracle_colour((uint32_t)k, seed);
        depth[q] = EMPTY_KEY;
    }
}

void oracle_step_render(float* pos, uint64_t n, uint32_t dim, uint64_t seed,
                        uint32_t step, float a, int wrap, const float m[16],
                        uint32_t width, uint32_t height, uint32_t footprint,
                        uint64_t* depth, uint32_t* colour)
{
    oracle_displace(pos, n, dim, seed, step, a, wrap);
    oracle_splat(pos, n, dim, m, width, height, footprint, depth, NULL);
    oracle_resolve(depth, colour, (uint64_t)width * height, seed);
}


/* Screen position (before the pixel floor) and clip w of a vertex, as the
 * point projection computes them: 2D (x + 1) W/2, (y + 1) H/2 and w = 0; 3D
 * rows 0, 1 and 3 of the camera, each summed left to right, and the same
 * perspective divide. Returns 0 when the near test (w > 0.1) culls it; the
 * screen test is left to each sample of a segment. */
int oracle_screen(const float* p, uint32_t dim, const float m[16], uint32_t width,
                  uint32_t height, float* sx, float* sy, float* w)
{
    const float half_w = (float)(width / 2u);
    const float half_h = (float)(height / 2u);
    if (dim == 2u) {
        *sx = (p[0] + 1.0f) * half_w;
        *sy = (p[1] + 1.0f) * half_h;
        *w = 0.0f;
        return 1;
    }
    const float x = p[0], y = p[1], z = p[2];
    float cx = m[0] * x;
    cx = cx + m[1] * y;
    cx = cx + m[2] * z;
    cx = cx + m[3];
    float cy = m[4] * x;
    cy = cy + m[5] * y;
    cy = cy + m[6] * z;
    cy = cy + m[7];
    float cw = m[12] * x;
    cw = cw + m[13] * y;
    cw = cw + m[14] * z;
    cw = cw + m[15];
    if (!(cw > 0.1f))
        return 0;
    const float inv_w = 1.0f / cw;
    *sx = (cx * inv_w + 1.0f) * half_w;
    *sy = (cy * inv_w + 1.0f) * half_h;
    *w = cw;
    return 1;
}

/* Reading of the edges view (the paper draws segments between indexed
 * positions through the raster pipeline): segment e joins vertices a and b.
 * Both must pass the near test. With dx, dy, dw the screen and depth
 * differences b - a, the segment takes n = ceil(max(|dx|, |dy|)) steps
 * (at most EDGE_MAX_STEPS; none for a point-like segment) and samples
 * t = k / n for k = 0..n: x = ax + t dx, y = ay + t dy, w = aw + t dw, each
 * rounded as written. Each sample on the screen takes the minimum of its
 * pixel's key (bits(w) << 32 | e), as a point does. A vertex index past the
 * vertex count skips the segment. */
#define EDGE_MAX_STEPS 32768u

void oracle_splat_edge(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                       uint32_t width, uint32_t height, uint32_t a, uint32_t b, uint32_t e,
                       uint64_t* depth)
{
    if ((uint64_t)a >= n || (uint64_t)b >= n)
        return;
    float ax, ay, aw, bx, by, bw;
    if (!oracle_screen(pos + (uint64_t)a * dim, dim, m, width, height, &ax, &ay, &aw))
        return;
    if (!oracle_screen(pos + (uint64_t)b * dim, dim, m, width, height, &bx, &by, &bw))
        return;
    const float dx = bx - ax, dy = by - ay, dw = bw - aw;
    const float len = fmaxf(fabsf(dx), fabsf(dy));
    const uint32_t steps = len >= (float)EDGE_MAX_STEPS ? EDGE_MAX_STEPS : (uint32_t)ceilf(len);
    for (uint32_t k = 0; k <= steps; ++k) {
        const float t = steps == 0u ? 0.0f : (float)k / (float)steps;
        const float x = ax + t * dx;
        const float y = ay + t * dy;
        const float w = aw + t * dw;
        if (!(x >= 0.0f && x < (float)width && y >= 0.0f && y < (float)height))
            continue;
        const int32_t px = (int32_t)floorf(x);
        const int32_t py = (int32_t)height - 1 - (int32_t)floorf(y);
        union {
            float f;
            uint32_t u;
        } pun;
        pun.f = w;
        const uint64_t key = ((uint64_t)(dim == 2u ? 0u : pun.u) << 32) | (uint64_t)e;
        uint64_t* slot = depth + (uint64_t)py * width + (uint64_t)px;
        if (key < *slot)
            *slot = key;
    }
}

/* All segments: pairs (prim == 2: edge e is (idx[2e], idx[2e+1])) or
 * triangles (prim == 3: triangle t gives edges 3t + j joining idx[3t + j]
 * and idx[3t + (j + 1) % 3]). */
void oracle_splat_edges(const float* pos, uint64_t n, uint32_t dim, const uint32_t* idx,
                        uint64_t nprim, uint32_t prim, const float m[16], uint32_t width,
                        uint32_t height, uint64_t* depth)
{
    for (uint64_t q = 0; q < nprim; ++q) {
        if (prim == 2u) {
            oracle_splat_edge(pos, n, dim, m, width, height, idx[2 * q], idx[2 * q + 1],
                              (uint32_t)q, depth);
        } else {
            for (uint32_t j = 0; j < 3u; ++j)
                oracle_splat_edge(pos, n, dim, m, width, height, idx[3 * q + j],
                                  idx[3 * q + (j + 1u) % 3u], (uint32_t)(3 * q + j), depth);
        }
    }
}
