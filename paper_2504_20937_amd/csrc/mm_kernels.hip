// Direct-splat kernels of the displace+render frame (gfx950).
//
// point kernel  : one pass over the cloud. Per point: load, Philox draw,
//                 displace (+fold), store, project with the float32 camera,
//                 and a 64-bit atomicMin of (depth_bits << 32 | index) into
//                 every pixel of the marker footprint of a full-screen key
//                 buffer, skipped when a plain load already shows a smaller
//                 key.
// resolve kernel: one pass over the screen. Key -> RGBA8 (colour hash of
//                 the winning index), and the key is reset to empty for the
//                 next frame.
//
// The point kernel with only the displacement phase is also the
// displace-only step of every splat mode.
#include <algorithm>

#include "mm_device.h"

namespace mm {
namespace {

using namespace dev;

template <int DIM, int FOOT, bool WRAP, int PHASE>
__global__ __launch_bounds__(256) void point_kernel(PointArgs a) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i == 0 && a.mark) *a.mark = wall_clock64();
    if (i >= a.c.n) return;
    float x, y, z;
    load_point<DIM>(a.c.pos, i, x, y, z);
    if constexpr ((PHASE & kDisplace) != 0) {
        displace<DIM, WRAP>(a.c, a.c.step, i, x, y, z);
        store_point<DIM>(a.c.pos, i, x, y, z);
    }
    if constexpr ((PHASE & kRender) != 0) {
        int32_t px, py;
        uint32_t bits;
        if (!project<DIM>(a.g, x, y, z, px, py, bits)) return;
        const uint64_t key = (static_cast<uint64_t>(bits) << 32) | i;
        if constexpr (FOOT == 1) {
            uint64_t* slot = a.depth + static_cast<uint64_t>(py) * a.g.width + px;
            if (key < *slot) atomic_min_global(slot, key);
        } else {
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t qy = py + dy;
                if (qy < 0 || qy >= static_cast<int32_t>(a.g.height)) continue;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t qx = px + dx;
                    if (qx < 0 || qx >= static_cast<int32_t>(a.g.width)) continue;
                    uint64_t* slot = a.depth + static_cast<uint64_t>(qy) * a.g.width + qx;
                    if (key < *slot) atomic_min_global(slot, key);
                }
            }
        }
    }
}

// Two pixels per thread: one 16-byte key load, one 8-byte colour store and
// one 16-byte store of empty keys.
__global__ __launch_bounds__(256) void resolve_kernel(ResolveArgs a) {
    const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
    if (2 * j >= a.npix) return;
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(a.depth);
    const ulonglong2 k = d2[j];
    const uint2 c = make_uint2(pixel_colour(k.x, a.seed_lo, a.seed_hi, a.pal),
                               pixel_colour(k.y, a.seed_lo, a.seed_hi, a.pal));
    reinterpret_cast<uint2*>(a.colour)[j] = c;
    d2[j] = make_ulonglong2(kEmptyKey, kEmptyKey);
}

__global__ __launch_bounds__(256) void fill_kernel(uint64_t* keys, uint64_t n, uint64_t value) {
    const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
    if (j < n) keys[j] = value;
}

// Host-staged tables into device memory: 8-byte words read from pinned,
// host-coherent memory with system-scope loads (always the host's latest
// writes, never a stale cached line), plus a tail of single bytes.
__global__ __launch_bounds__(256) void upload_kernel(const uint64_t* src, uint64_t* dst, uint64_t n8,
                                                     const unsigned char* src_tail,
                                                     unsigned char* dst_tail, uint32_t tail) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256u;
    for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x; j < n8; j += stride)
        dst[j] = __hip_atomic_load(src + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (blockIdx.x == 0 && threadIdx.x < tail)
        dst_tail[threadIdx.x] = __hip_atomic_load(src_tail + threadIdx.x, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
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
    l.shared = 0;
    return l;
}

Launch resolve_launch(uint64_t npix) {
    Launch l;
    l.func = reinterpret_cast<const void*>(&resolve_kernel);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((npix / 2 + 255) / 256));
    l.shared = 0;
    return l;
}

hipError_t launch_point(const PointArgs& a, int dim, int footprint, bool wrap, Phase phase,
                        hipStream_t s) {
    const Launch l = point_launch(dim, footprint, wrap, phase, a.c.n);
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

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 7u)
        return hipErrorInvalidValue;
    const uint64_t* src8 = static_cast<const uint64_t*>(src);
    uint64_t* dst8 = static_cast<uint64_t*>(dst);
    uint64_t n8 = bytes / 8;
    const unsigned char* src_tail = static_cast<const unsigned char*>(src) + n8 * 8;
    unsigned char* dst_tail = static_cast<unsigned char*>(dst) + n8 * 8;
    uint32_t tail = static_cast<uint32_t>(bytes % 8);
    const dim3 grid(static_cast<uint32_t>(std::min<uint64_t>((n8 + 255) / 256, 64)) + (n8 == 0 ? 1u : 0u));
    void* args[] = {&src8, &dst8, &n8, &src_tail, &dst_tail, &tail};
    return hipLaunchKernel(reinterpret_cast<const void*>(&upload_kernel), grid, dim3(256), args, 0, s);
}

__global__ __launch_bounds__(64) void mark_kernel(uint64_t* slot) {
    if (threadIdx.x == 0) *slot = wall_clock64();
}

hipError_t launch_mark(uint64_t* slot, hipStream_t s) {
    void* args[] = {&slot};
    return hipLaunchKernel(reinterpret_cast<const void*>(&mark_kernel), dim3(1), dim3(64), args, 0, s);
}

hipError_t launch_fill(uint64_t* keys, uint64_t nkeys, uint64_t value, hipStream_t s) {
    if (nkeys == 0) return hipSuccess;
    const dim3 grid(static_cast<uint32_t>((nkeys + 255) / 256));
    void* args[] = {&keys, &nkeys, &value};
    return hipLaunchKernel(reinterpret_cast<const void*>(&fill_kernel), grid, dim3(256), args, 0,
                           s);
}

}  // namespace mm
