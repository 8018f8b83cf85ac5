// Internal interface between the C ABI runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

constexpr uint64_t kEmptyKey = 0xFFFFFFFFFFFFFFFFull;

// Everything one launch of the point kernel needs, passed by value so the
// whole struct lands in the kernel-argument segment (uniform, SGPRs).
struct PointArgs {
    float* pos;         // AoS float2 / float3
    uint64_t* depth;    // width * height keys
    uint32_t n;         // points
    uint32_t width, height;
    float half_w, half_h;
    float fwidth, fheight;
    uint32_t seed_lo, seed_hi;
    uint32_t step;
    float amp;          // a
    float m[12];        // rows 0, 1 and 3 of the row-major view-projection
};

struct ResolveArgs {
    uint64_t* depth;    // read, then reset to empty
    uint32_t* colour;
    uint64_t npix;      // even
    uint32_t seed_lo, seed_hi;
};

// What the point kernel does in one launch.
enum Phase : int { kDisplace = 1, kRender = 2, kDisplaceRender = 3 };

struct Launch {
    const void* func;   // kernel symbol, usable as a graph kernel node
    dim3 grid, block;
};

// Kernel choice and launch shape for the point kernel.
Launch point_launch(int dim, int footprint, bool wrap, Phase phase, uint32_t n);
Launch resolve_launch(uint64_t npix);
Launch fill_launch(uint64_t nkeys);

hipError_t launch_point(const PointArgs& a, int dim, int footprint, bool wrap, Phase phase,
                        hipStream_t s);
hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s);
hipError_t launch_fill(uint64_t* keys, uint64_t nkeys, hipStream_t s);

}  // namespace mm
