/*
 * Plain sequential CPU definition of one displace+render frame of the
 * point-cloud benchmark of "Mimir: A real-time interactive visualization
 * library for CUDA programs" (section "Performance Benchmark": random
 * initial points, a displacement kernel at every timestep, and a render of
 * the same memory with every point the same size).
 *
 * TEST INFRASTRUCTURE. This library defines the expected result. Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. The GPU library shares no code, header or constant with it.
 *
 * Arithmetic: IEEE-754 binary32, round-to-nearest-even, no contraction, no
 * flush-to-zero (build: gcc -O2 -ffp-contract=off -fno-fast-math). The paper
 * stores positions as float3 (section "Views", listing "C++ Library usage
 * example"), which fixes the precision at binary32.
 */
#ifndef MM_ORACLE_H
#define MM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block cipher (Salmon, Moraes, Dror, Shaw, "Parallel Random
 * Numbers: As Easy as 1, 2, 3", SC'11, the Philox construction). ctr[4], key[2] in,
 * out[4] out. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* n independent blocks: ctr is n*4 words, key n*2 words, out n*4 words. */
void oracle_philox4x32_10_many(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n);

/* Uniform offset in [-a, a) from one 32-bit word: the top 24 bits select a
 * grid point of [-1, 1) that is then scaled by a with one rounding. */
float oracle_offset(uint32_t r, float a);

/* oracle_offset over n words. */
void oracle_offset_many(const uint32_t* r, uint64_t n, float a, float* out);

/* Periodic wrap of one coordinate into [-1, 1), valid for |x| < 2. */
float oracle_wrap(float x);

/* One displacement timestep over n points of dimension dim (2 or 3), AoS,
 * in place. Point i, step s: r = philox(ctr=(s, 0, lo32(i), hi32(i)),
 * key=(lo32(seed), hi32(seed))); coordinate c moves by offset(r[c], a);
 * wrap (if set) folds it back into [-1, 1). */
void oracle_displace(float* pos, uint64_t n, uint32_t dim, uint64_t seed,
                     uint32_t step, float a, int wrap);

/* Projection of one point to a pixel. 2D: orthographic over [-1,1)^2, depth
 * bits 0. 3D: row-major float32 view-projection m[16]; clip w must exceed
 * 0.1; depth bits = bit pattern of clip w. Returns 1 and writes the pixel
 * (row 0 = top) when the point lands on the W x H screen, else 0. */
int oracle_project(const float* p, uint32_t dim, const float m[16],
                   uint32_t width, uint32_t height,
                   int32_t* px, int32_t* py, uint32_t* depth_bits);

/* oracle_project for points 0..n-1 of an AoS array: pixel index
 * py * width + px of each point that lands on screen, else -1. */
void oracle_project_many(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                         uint32_t width, uint32_t height, int64_t* pixel);

/* Depth-resolved splat. For every point (in the order order[0..n-1] when
 * order is not NULL, else 0..n-1) that projects on screen, every pixel of
 * its footprint (1: the pixel itself; 3: the 3x3 block around it, each
 * clipped to the screen) takes min(current, depth_bits<<32 | lo32(i)).
 * depth has width*height keys, row-major. */
void oracle_splat(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                  uint32_t width, uint32_t height, uint32_t footprint,
                  uint64_t* depth, const uint64_t* order);

/* Colour of point index i: first word of philox(ctr=(0, 2, i, 0), key=seed)
 * with the alpha byte forced to 0xFF. RGBA8 packed little-endian. */
uint32_t oracle_colour(uint32_t index, uint64_t seed);

/* Resolve and clear: colour[p] = 0 for an empty pixel, else
 * oracle_colour(lo32(depth[p]), seed); then depth[p] = all ones. */
void oracle_resolve(uint64_t* depth, uint32_t* colour, uint64_t npix, uint64_t seed);
int oracle_screen(const float* p, uint32_t dim, const float m[16], uint32_t width,
                  uint32_t height, float* sx, float* sy, float* w);
void oracle_splat_edge(const float* pos, uint64_t n, uint32_t dim, const float m[16],
                       uint32_t width, uint32_t height, uint32_t a, uint32_t b, uint32_t e,
                       uint64_t* depth);
void oracle_splat_edges(const float* pos, uint64_t n, uint32_t dim, const uint32_t* idx,
                        uint64_t nprim, uint32_t prim, const float m[16], uint32_t width,
                        uint32_t height, uint64_t* depth);

/* One whole frame: displace with step s, splat, resolve. depth must hold
 * all-ones keys on entry and holds them again on return. */
void oracle_step_render(float* pos, uint64_t n, uint32_t dim, uint64_t seed,
                        uint32_t step, float a, int wrap, const float m[16],
                        uint32_t width, uint32_t height, uint32_t footprint,
                        uint64_t* depth, uint32_t* colour);

#ifdef __cplusplus
}
#endif
#endif
