// Internal interface between the C ABI runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mm {

constexpr uint64_t kEmptyKey = 0xFFFFFFFFFFFFFFFFull;

// Everything a point pass needs, passed by value so the whole struct lands
// in the kernel-argument segment (uniform, SGPRs).
struct PointArgs {
    float* pos;         // AoS float2 / float3
    uint64_t* depth;    // direct splat: width * height keys
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

// Binned splat, bin pass.
struct BinArgs {
    PointArgs p;
    uint64_t* seg;       // num_wg * P records, P = 256 * points per thread
    uint16_t* table;     // num_wg rows of ntiles + 1 tile start offsets
    uint32_t* active;    // ntiles: stamp of the last frame the tile received points
    uint32_t* stamp_out; // the frame stamp, for the tile and seam passes
    uint32_t stamp;
    uint32_t tiles_x, ntiles;
    uint32_t shift;      // tile side = 1 << shift
};

// Binned splat, tile and seam passes.
struct TileArgs {
    const uint64_t* seg;
    const uint16_t* table;
    const uint32_t* active;
    const uint32_t* stamp_in;
    uint64_t* part;      // ntiles * splits partial key tiles (apron included)
    uint64_t* border;    // footprint 3: ntiles * 4 * side edge keys
    uint64_t* apron;     // footprint 3: ntiles * (4 * side + 4) apron keys
    uint32_t* colour;
    uint32_t width, height;
    uint32_t tiles_x, tiles_y, ntiles;
    uint32_t num_wg, points_per_wg;
    uint32_t splits;     // tile-pass workgroups per tile
    uint32_t seed_lo, seed_hi;
};

// What a point pass does in one launch.
enum Phase : int { kDisplace = 1, kRender = 2, kDisplaceRender = 3 };

struct Launch {
    const void* func;   // kernel symbol, usable as a graph kernel node
    dim3 grid, block;
    uint32_t shared;    // dynamic LDS bytes
};

// Direct splat.
Launch point_launch(int dim, int footprint, bool wrap, Phase phase, uint32_t n);
Launch resolve_launch(uint64_t npix);
hipError_t launch_point(const PointArgs& a, int dim, int footprint, bool wrap, Phase phase,
                        hipStream_t s);
hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s);
hipError_t launch_fill(uint64_t* keys, uint64_t nkeys, uint64_t value, hipStream_t s);

// Binned splat. Tile side 1 << shift with shift in {4, 5, 6}; points per
// thread in {4, 8, 16}; splits per tile in {1, 2, 4, 8}.
bool binned_shape_ok(int shift, int ppt, uint32_t splits);
size_t bin_lds_bytes(int ppt, uint32_t ntiles);
Launch bin_launch(int dim, bool wrap, Phase phase, int ppt, uint32_t n, uint32_t ntiles);
Launch tile_launch(int footprint, int shift, uint32_t ntiles, uint32_t splits);
Launch merge_launch(int footprint, int shift, uint32_t ntiles);
Launch seam_launch(int shift, uint32_t ntiles);

}  // namespace mm
