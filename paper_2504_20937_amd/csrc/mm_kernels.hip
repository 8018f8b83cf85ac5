// gfx950 kernels of the displace+render frame.
//
// point kernel  : one pass over the cloud. Per point: load, Philox draw,
//                 displace (+wrap), store, project with the float32 camera,
//                 and a 64-bit atomicMin of (depth_bits << 32 | index) into
//                 every pixel of the marker footprint.
// resolve kernel: one pass over the screen. Key -> RGBA8 (colour hash of
//                 the winning index), and the key is reset to empty for the
//                 next frame.
//
// Bit-exactness with the CPU definition rests on binary32 round-to-nearest
// with no contraction (this file is built with -ffp-contract=off and the
// pragma below), IEEE division (hipcc's default correctly rounded f32
// divide), denormals kept, and the same operation order.
#include "mm_internal.h"

#pragma clang fp contract(off)

namespace mm {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kTagDisplace = 0u;
constexpr uint32_t kTagColour = 2u;

// Philox4x32-10 (Salmon et al., SC'11). The key and counter words that are
// the same for the whole launch (seed, step, tag) stay scalar, so the key
// schedule and the first round's uniform product cost no vector ALU.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c0;
        const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
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

__device__ __forceinline__ void atomic_min_key(uint64_t* slot, uint64_t key) {
    __hip_atomic_fetch_min(reinterpret_cast<unsigned long long*>(slot),
                           static_cast<unsigned long long>(key), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

struct Float3 {
    float x, y, z;
};

template <int DIM, int FOOT, bool WRAP, int PHASE>
__global__ __launch_bounds__(256) void point_kernel(PointArgs a) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= a.n) return;

    float x, y, z = 0.0f;
    if constexpr (DIM == 2) {
        const float2 p = reinterpret_cast<const float2*>(a.pos)[i];
        x = p.x;
        y = p.y;
    } else {
        const Float3 p = reinterpret_cast<const Float3*>(a.pos)[i];
        x = p.x;
        y = p.y;
        z = p.z;
    }

    if constexpr ((PHASE & kDisplace) != 0) {
        const uint4 r = philox4x32_10(a.step, kTagDisplace, i, 0u, a.seed_lo, a.seed_hi);
        x = x + offset(r.x, a.amp);
        y = y + offset(r.y, a.amp);
        if constexpr (DIM == 3) z = z + offset(r.z, a.amp);
        if constexpr (WRAP) {
            x = fold(x);
            y = fold(y);
            if constexpr (DIM == 3) z = fold(z);
        }
        if constexpr (DIM == 2) {
            reinterpret_cast<float2*>(a.pos)[i] = make_float2(x, y);
        } else {
            reinterpret_cast<Float3*>(a.pos)[i] = Float3{x, y, z};
        }
    }

    if constexpr ((PHASE & kRender) != 0) {
        float sx, sy;
        uint32_t bits = 0u;
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
            if (!(cw > 0.1f)) return;
            const float iw = 1.0f / cw;
            sx = (cx * iw + 1.0f) * a.half_w;
            sy = (cy * iw + 1.0f) * a.half_h;
            bits = __float_as_uint(cw);
        }
        if (!(sx >= 0.0f && sx < a.fwidth && sy >= 0.0f && sy < a.fheight)) return;
        const int32_t px = static_cast<int32_t>(floorf(sx));
        const int32_t py = static_cast<int32_t>(a.height) - 1 - static_cast<int32_t>(floorf(sy));
        const uint64_t key = (static_cast<uint64_t>(bits) << 32) | i;
        if constexpr (FOOT == 1) {
            uint64_t* slot = a.depth + static_cast<uint64_t>(py) * a.width + px;
            if (key < *slot) atomic_min_key(slot, key);
        } else {
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t qy = py + dy;
                if (qy < 0 || qy >= static_cast<int32_t>(a.height)) continue;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t qx = px + dx;
                    if (qx < 0 || qx >= static_cast<int32_t>(a.width)) continue;
                    uint64_t* slot = a.depth + static_cast<uint64_t>(qy) * a.width + qx;
                    if (key < *slot) atomic_min_key(slot, key);
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t colour_of(uint64_t key, uint32_t seed_lo, uint32_t seed_hi) {
    if (key == kEmptyKey) return 0u;
    const uint4 r = philox4x32_10(0u, kTagColour, static_cast<uint32_t>(key), 0u, seed_lo,
                                  seed_hi);
    return r.x | 0xFF000000u;
}

// Two pixels per thread: one 16-byte key load, one 8-byte colour store and
// one 16-byte store of empty keys.
__global__ __launch_bounds__(256) void resolve_kernel(ResolveArgs a) {
    const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
    if (2 * j >= a.npix) return;
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(a.depth);
    const ulonglong2 k = d2[j];
    const uint2 c = make_uint2(colour_of(k.x, a.seed_lo, a.seed_hi),
                               colour_of(k.y, a.seed_lo, a.seed_hi));
    reinterpret_cast<uint2*>(a.colour)[j] = c;
    d2[j] = make_ulonglong2(kEmptyKey, kEmptyKey);
}

__global__ __launch_bounds__(256) void fill_kernel(uint64_t* keys, uint64_t n) {
    const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
    if (j < n) keys[j] = kEmptyKey;
}

template <int DIM, int FOOT, bool WRAP>
const void* pick_phase(Phase phase) {
    switch (phase) {
        case kDisplace: return reinterpret_cast<const void*>(&point_kernel<DIM, 1, WRAP, kDisplace>);
        case kRender: return reinterpret_cast<const void*>(&point_kernel<DIM, FOOT, WRAP, kRender>);
        default: return reinterpret_cast<const void*>(&point_kernel<DIM, FOOT, WRAP, kDisplaceRender>);
    }
}

template <int DIM>
const void* pick(int footprint, bool wrap, Phase phase) {
    if (footprint == 3) {
        return wrap ? pick_phase<DIM, 3, true>(phase) : pick_phase<DIM, 3, false>(phase);
    }
    return wrap ? pick_phase<DIM, 1, true>(phase) : pick_phase<DIM, 1, false>(phase);
}

}  // namespace

Launch point_launch(int dim, int footprint, bool wrap, Phase phase, uint32_t n) {
    Launch l;
    l.func = dim == 2 ? pick<2>(footprint, wrap, phase) : pick<3>(footprint, wrap, phase);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((static_cast<uint64_t>(n) + 255u) / 256u));
    return l;
}

Launch resolve_launch(uint64_t npix) {
    Launch l;
    l.func = reinterpret_cast<const void*>(&resolve_kernel);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((npix / 2 + 255) / 256));
    return l;
}

Launch fill_launch(uint64_t nkeys) {
    Launch l;
    l.func = reinterpret_cast<const void*>(&fill_kernel);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((nkeys + 255) / 256));
    return l;
}

hipError_t launch_point(const PointArgs& a, int dim, int footprint, bool wrap, Phase phase,
                        hipStream_t s) {
    const Launch l = point_launch(dim, footprint, wrap, phase, a.n);
    PointArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(l.func, l.grid, l.block, args, 0, s);
}

hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s) {
    const Launch l = resolve_launch(a.npix);
    ResolveArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(l.func, l.grid, l.block, args, 0, s);
}

hipError_t launch_fill(uint64_t* keys, uint64_t nkeys, hipStream_t s) {
    const Launch l = fill_launch(nkeys);
    void* args[] = {&keys, &nkeys};
    return hipLaunchKernel(l.func, l.grid, l.block, args, 0, s);
}

}  // namespace mm
