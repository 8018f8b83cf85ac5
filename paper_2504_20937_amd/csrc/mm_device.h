// Per-point device arithmetic shared by the gfx950 kernels: the Philox
// draw, the displacement, and the projection to a pixel. Every operation is
// binary32 round-to-nearest with no contraction, in the order the frame is
// defined in (displace: p + offset, fold; project: clip rows summed left to
// right, IEEE 1/w, screen map, floor).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mm_internal.h"

#pragma clang fp contract(off)

namespace mm {
namespace dev {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kTagDisplace = 0u;
constexpr uint32_t kTagColour = 2u;

// Philox4x32-10 (Salmon et al., SC'11). Counter and key words that are the
// same for the whole launch (seed, step, tag) stay scalar, so the key
// schedule and the first round's uniform product cost no vector ALU. The two
// three-way XORs of a round are single bitop3 instructions on gfx950.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c0;
        const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Offset in [-a, a): the top 24 bits pick k * 2^-23 - 1 (exact), one
// rounding for the product with a.
__device__ __forceinline__ float offset(uint32_t r, float a) {
    const float t = static_cast<float>(r >> 8) * 0x1p-23f - 1.0f;
    return t * a;
}

__device__ __forceinline__ float fold(float x) {
    if (x >= 1.0f) return x - 2.0f;
    if (x < -1.0f) return x + 2.0f;
    return x;
}

// fold() against a uniform limit, without branches: lim = 1 folds, lim = +inf
// leaves x as it is. The two tests in sequence equal fold()'s either-or:
// after x - 2 with x >= 1, x >= -1 holds.
__device__ __forceinline__ float fold_to(float x, float lim) {
    x = x >= lim ? x - 2.0f : x;
    x = x < -lim ? x + 2.0f : x;
    return x;
}

struct Float3 {
    float x, y, z;
};

// Positions are streamed: read once and written once per frame, so both
// directions use non-temporal accesses, which keep the caches for the tile
// records and table that the tile pass reads right after the bin pass
// (1080p, 2^24 points: 177 -> 155 us per frame; 4K 2^28: bin pass 1.75 -> 1.62 ms).
template <int DIM>
__device__ __forceinline__ void load_point(const float* pos, uint32_t i, float& x, float& y,
                                           float& z) {
    if constexpr (DIM == 2) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        const f2v p = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(pos) + i);
        x = p.x;
        y = p.y;
        z = 0.0f;
    } else {
        typedef float f3v __attribute__((ext_vector_type(3)));
        // a 12-byte load (global_load_dwordx3 nt) of the point's 12-byte slot
        const f3v p = __builtin_nontemporal_load(
            reinterpret_cast<const f3v*>(reinterpret_cast<const char*>(pos) + 12ull * i));
        x = p.x;
        y = p.y;
        z = p.z;
    }
}

template <int DIM>
__device__ __forceinline__ void store_point(float* pos, uint32_t i, float x, float y, float z) {
    if constexpr (DIM == 2) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        f2v v;
        v.x = x;
        v.y = y;
        __builtin_nontemporal_store(v, reinterpret_cast<f2v*>(pos) + i);
    } else {
        typedef float f3v __attribute__((ext_vector_type(3)));
        f3v v;
        v.x = x;
        v.y = y;
        v.z = z;
        // a 12-byte store (global_store_dwordx3 nt) at the point's 12-byte slot
        __builtin_nontemporal_store(v, reinterpret_cast<f3v*>(reinterpret_cast<char*>(pos) + 12ull * i));
    }
}

// One timestep of point i: draw keyed by (seed, i, step), add, fold.
template <int DIM, bool WRAP>
__device__ __forceinline__ void displace(const CloudArgs& a, uint32_t step, uint32_t i, float& x,
                                         float& y, float& z) {
    const uint4 r = philox4x32_10(step, kTagDisplace, i, 0u, a.seed_lo, a.seed_hi);
    x = x + offset(r.x, a.amp);
    y = y + offset(r.y, a.amp);
    if constexpr (DIM == 3) z = z + offset(r.z, a.amp);
    if constexpr (WRAP) {
        x = fold(x);
        y = fold(y);
        if constexpr (DIM == 3) z = fold(z);
    }
}

// Projection to a pixel (row 0 = top). Returns false when culled (behind
// the near plane or off screen); depth bits are those of clip w (3D) or 0.
template <int DIM>
__device__ __forceinline__ bool project(const ViewGeom& a, float x, float y, float z,
                                        int32_t& px, int32_t& py, uint32_t& bits) {
    float sx, sy;
    bits = 0u;
    if constexpr (DIM == 2) {
        sx = (x + 1.0f) * a.half_w;
        sy = (y + 1.0f) * a.half_h;
    } else {
        float cx = a.m[0] * x;
        cx = cx + a.m[1] * y;
        cx = cx + a.m[2] * z;
        cx = cx + a.m[3];
        float cy = a.m[4] * x;
        cy = cy + a.m[5] * y;
        cy = cy + a.m[6] * z;
        cy = cy + a.m[7];
        float cw = a.m[8] * x;
        cw = cw + a.m[9] * y;
        cw = cw + a.m[10] * z;
        cw = cw + a.m[11];
        if (!(cw > 0.1f)) return false;
        const float iw = 1.0f / cw;
        sx = (cx * iw + 1.0f) * a.half_w;
        sy = (cy * iw + 1.0f) * a.half_h;
        bits = __float_as_uint(cw);
    }
    if (!(sx >= 0.0f && sx < a.fwidth && sy >= 0.0f && sy < a.fheight)) return false;
    px = static_cast<int32_t>(floorf(sx));
    py = static_cast<int32_t>(a.height) - 1 - static_cast<int32_t>(floorf(sy));
    return true;
}

// Colour of a resolved key: background 0, else the first Philox word of the
// colour-tagged counter of the winning index, alpha forced opaque.
__device__ __forceinline__ uint32_t colour_of(uint64_t key, uint32_t seed_lo, uint32_t seed_hi) {
    if (key == kEmptyKey) return 0u;
    const uint4 r = philox4x32_10(0u, kTagColour, static_cast<uint32_t>(key), 0u, seed_lo,
                                  seed_hi);
    return r.x | 0xFF000000u;
}

// Colour of a resolved key under the view's palette: the hash colour when it
// has none; else the table entry of the winning point (through its index
// when the palette has an index buffer), 0 past the table's end.
__device__ __forceinline__ uint32_t pixel_colour(uint64_t key, uint32_t seed_lo, uint32_t seed_hi,
                                                 const Palette& p) {
    if (!p.table) return colour_of(key, seed_lo, seed_hi);
    if (key == kEmptyKey) return 0u;
    const uint32_t i = static_cast<uint32_t>(key);
    uint32_t j = i;
    if (p.index) {
        if (p.index_size == 1) j = static_cast<const uint8_t*>(p.index)[i];
        else if (p.index_size == 2) j = static_cast<const uint16_t*>(p.index)[i];
        else j = static_cast<const uint32_t*>(p.index)[i];
    }
    return j < p.size ? p.table[j] : 0u;
}

__device__ __forceinline__ void atomic_min_global(uint64_t* slot, uint64_t key) {
    __hip_atomic_fetch_min(reinterpret_cast<unsigned long long*>(slot),
                           static_cast<unsigned long long>(key), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_min_lds(uint64_t* slot, uint64_t key) {
    __hip_atomic_fetch_min(reinterpret_cast<unsigned long long*>(slot),
                           static_cast<unsigned long long>(key), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Work tables do not change during a launch: reading them through the
// constant address space lets the compiler use scalar loads even after the
// kernel's own global stores, so item, cloud and view fields stay uniform
// (SGPRs) instead of being treated as per-lane values.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized fields");
    using CWord = const __attribute__((address_space(4))) uint32_t;
    CWord* q = (CWord*)(p);
    T out;
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (size_t k = 0; k < sizeof(T) / 4; ++k) o[k] = q[k];
    return out;
}

// Per-tile frame stamps: relaxed atomics at wavefront scope, which compile to
// plain cached loads and stores.
__device__ __forceinline__ void store_flag(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint32_t load_flag(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// A padding entry of a work table: the block skips it.
constexpr uint32_t kPadItem = 0xFFFFFFFFu;

}  // namespace dev
}  // namespace mm
