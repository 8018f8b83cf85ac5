/*
 * Host-copy comparison path: the way a simulation without device interop
 * draws its data (the paper's introduction and section "Performance
 * Benchmark" compare against it). The positions are copied from the device
 * to host memory each frame and rendered here, on every host core.
 *
 * The frame it draws is the same as the device path's, bit for bit: each
 * thread splats a contiguous share of the points into its own key buffer
 * (key = depth bits << 32 | index, minimum wins), the buffers are merged by
 * minimum per pixel, and the winning index is coloured with the Philox
 * colour hash. Arithmetic is binary32 with no contraction, in the order the
 * frame is defined in.
 *
 * Built with gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#include "hostcopy.h"

#define EMPTY_KEY 0xFFFFFFFFFFFFFFFFull

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
 * 32x32->64 products with the counter words, key bumped between rounds. */
static void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * c[0];
        const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)b;
        c[3] = (uint32_t)a;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

static uint32_t colour_of(uint64_t key, uint64_t seed) {
    if (key == EMPTY_KEY) return 0u;
    uint32_t c[4] = {0u, 2u, (uint32_t)key, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return c[0] | 0xFF000000u;
}

/* Pixel of one point; 0 when culled. */
static int to_pixel(const float* p, int dim, const float* m, uint32_t w, uint32_t h,
                    int32_t* px, int32_t* py, uint32_t* bits) {
    const float hw = (float)(w / 2u), hh = (float)(h / 2u);
    float sx, sy;
    *bits = 0u;
    if (dim == 2) {
        sx = (p[0] + 1.0f) * hw;
        sy = (p[1] + 1.0f) * hh;
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
        float cw = m[8] * x;
        cw = cw + m[9] * y;
        cw = cw + m[10] * z;
        cw = cw + m[11];
        if (!(cw > 0.1f)) return 0;
        const float iw = 1.0f / cw;
        sx = (cx * iw + 1.0f) * hw;
        sy = (cy * iw + 1.0f) * hh;
        memcpy(bits, &cw, 4);
    }
    if (!(sx >= 0.0f && sx < (float)w && sy >= 0.0f && sy < (float)h)) return 0;
    *px = (int32_t)floorf(sx);
    *py = (int32_t)h - 1 - (int32_t)floorf(sy);
    return 1;
}

int hc_render(const float* pos, uint64_t n, int dim, const float view_proj[16], uint32_t width,
              uint32_t height, uint32_t footprint, uint64_t seed, uint32_t* rgba, int threads) {
    if (!pos || !rgba || !view_proj || (dim != 2 && dim != 3) || width < 2 || height < 2 ||
        (footprint != 1 && footprint != 3) || n > 0xFFFFFFFFull)
        return -1;
    if (threads <= 0) threads = omp_get_max_threads();
    const uint64_t npix = (uint64_t)width * height;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * npix * (uint64_t)threads);
    if (!keys) return -2;
    float m[12];
    const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) m[4 * r + c] = view_proj[4 * rows[r] + c];
    const int rad = footprint == 3 ? 1 : 0;

#pragma omp parallel num_threads(threads)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        uint64_t* d = keys + (uint64_t)t * npix;
        for (uint64_t q = 0; q < npix; ++q) d[q] = EMPTY_KEY;
        const uint64_t lo = n * (uint64_t)t / (uint64_t)nt, hi = n * (uint64_t)(t + 1) / (uint64_t)nt;
        for (uint64_t i = lo; i < hi; ++i) {
            int32_t px, py;
            uint32_t bits;
            if (!to_pixel(pos + (uint64_t)dim * i, dim, m, width, height, &px, &py, &bits)) continue;
            const uint64_t key = ((uint64_t)bits << 32) | i;
            for (int dy = -rad; dy <= rad; ++dy) {
                const int32_t y = py + dy;
                if (y < 0 || y >= (int32_t)height) continue;
                for (int dx = -rad; dx <= rad; ++dx) {
                    const int32_t x = px + dx;
                    if (x < 0 || x >= (int32_t)width) continue;
                    uint64_t* slot = d + (uint64_t)y * width + (uint64_t)x;
                    if (key < *slot) *slot = key;
                }
            }
        }
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t q = 0; q < (int64_t)npix; ++q) {
            uint64_t k = keys[q];
            for (int u = 1; u < nt; ++u) {
                const uint64_t v = keys[(uint64_t)u * npix + (uint64_t)q];
                k = v < k ? v : k;
            }
            rgba[q] = colour_of(k, seed);
        }
    }
    free(keys);
    return 0;
}

int hc_max_threads(void) { return omp_get_max_threads(); }
