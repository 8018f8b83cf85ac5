// Internal interface between the C ABI runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mm {

constexpr uint64_t kEmptyKey = 0xFFFFFFFFFFFFFFFFull;

// One point cloud and its displacement draw.
struct CloudArgs {
    float* pos;         // AoS float2 / float3
    uint32_t n;         // points
    uint32_t seed_lo, seed_hi;
    uint32_t step;
    float amp;          // a
    float fold_lim;     // batched kernels: 1 folds each coordinate into [-1, 1)
                        // after the step, +inf leaves it (plain kernels take the
                        // fold as a template parameter)
};

// The screen mapping of one view.
struct ViewGeom {
    uint32_t width, height;
    float half_w, half_h;
    float fwidth, fheight;
    float m[12];        // rows 0, 1 and 3 of the row-major view-projection
};

// Direct splat: everything a point pass needs, passed by value so the whole
// struct lands in the kernel-argument segment (uniform, SGPRs).
struct PointArgs {
    CloudArgs c;
    ViewGeom g;
    uint64_t* depth;    // width * height keys
    uint64_t* mark;     // frame mark: the device clock when the frame's first
                        // kernel starts (nullptr: none)
};

// Colour source of a view: the per-point hash (table == nullptr), or RGBA8
// table entries, taken through a per-point index buffer of index_size (1, 2
// or 4) byte unsigned integers, or by point index when index == nullptr. An
// index past the table gives colour 0.
struct Palette {
    const uint32_t* table;
    const void* index;
    uint32_t size;
    uint32_t index_size;
};

struct ResolveArgs {
    uint64_t* depth;    // read, then reset to empty
    uint32_t* colour;
    uint64_t npix;      // even
    uint32_t seed_lo, seed_hi;
    Palette pal;
};

// Occlusion cull of a binned view (3D, 1x1 footprint, one tile-pass
// workgroup per tile). Per frame the hint kernel takes the winning point of
// every pixel of the previous frame (the hints), moves it by this frame's
// step and projects it with this frame's camera, and writes one cull record
// per screen tile. A pixel is covered when such a point lands on it; no point
// landing there can then win with a larger depth than that point's. The bin
// kernel drops a record whose pixel is covered and whose depth exceeds the
// bound of its 8x8-pixel block (the largest of the block's covered pixels'
// depths), so the dropped record loses its pixel to a point of this frame:
// the frame is unchanged, only fewer records are written and read.
//
// A cull record of a tile of side S (cull_words(S) u32): the covered bitmap
// (S*S/32 words, bit q of the tile's pixels in row-major order), then the
// bound of each 8x8 block ((S/8)^2 words, depth bits), padded to 16 words.
// The hint kernel merges into the records with atomic OR and MAX, so every
// record is zero before it runs: the one-split 1x1 tile pass zeroes each
// tile's record after the bin pass has read it.
__host__ __device__ constexpr uint32_t cull_bitmap_words(uint32_t side) { return side * side / 32u; }
__host__ __device__ constexpr uint32_t cull_blocks(uint32_t side) { return (side / 8u) * (side / 8u); }
__host__ __device__ constexpr uint32_t cull_words(uint32_t side) {
    return (cull_bitmap_words(side) + cull_blocks(side) + 15u) / 16u * 16u;
}
constexpr uint32_t kNoHint = 0xFFFFFFFFu;

// Binned splat, bin pass side of one view.
struct BinView {
    ViewGeom g;
    uint64_t* seg;       // num_wg * P records, P = 256 * points per thread
    uint16_t* table;     // num_wg rows of ntiles + 1 tile start offsets
    uint32_t* active;    // ntiles: stamp of the last frame the tile received points
    uint32_t tiles_x, ntiles;
    uint32_t* cull;        // occlusion cull: ntiles records (nullptr: no cull)
    const uint32_t* hint;  // occlusion cull: ntiles * S * S point indices, tile-major
                           // (pixel q = y * S + x of tile t at t * S * S + q), kNoHint = none
};

// Binned splat, tile and merge side of one view.
struct TileView {
    const uint64_t* seg;
    const uint16_t* table;
    const uint32_t* active;
    uint64_t* part;      // ntiles * splits partial key tiles (apron included)
    uint64_t* border;    // footprint 3: ntiles * 4 * side edge keys
    uint64_t* apron;     // footprint 3: ntiles * (4 * side + 4) apron keys
    uint32_t* colour;
    uint32_t width, height;
    uint32_t tiles_x, tiles_y, ntiles;
    uint32_t num_wg;     // bin workgroups (chunks of points) of the view's cloud
    uint32_t splits;     // tile-pass workgroups per tile (static splits)
    const uint32_t* piece_first;  // load-balanced: ntiles + 1 first partial block of
                                  // each tile (nullptr: static splits)
    const uint16_t* tcol;         // load-balanced: the table tile-major, row t (of
                                  // ntiles + 1, tcol_stride entries each) holding
                                  // entry t of every table row (nullptr: read the rows)
    uint32_t tcol_stride;
    uint32_t full_clear; // 1: clear every tile not drawn this frame (the frame buffer
                         // holds no earlier frame); 0: only tiles drawn last frame
    uint32_t prev_stamp; // non-zero: the stamp of the frame buffer's previous frame
                         // (a served buffer, drawn by some earlier launch): tiles
                         // drawn then and not now are cleared as well
    uint32_t seed_lo, seed_hi;
    Palette pal;
    uint32_t* hint;      // occlusion cull: the one-split 1x1 pass writes each drawn
                         // tile's winning point indices here (nullptr: none)
    uint32_t* cull;      // occlusion cull: the one-split 1x1 pass zeroes each tile's
                         // cull record (nullptr: none)
};

// Binned splat of one cloud into one view.
struct BinArgs {
    CloudArgs c;
    BinView v;
    uint32_t* stamp_out; // the frame stamp, for the tile, merge and seam passes
    uint32_t stamp;
    uint32_t shift;      // tile side = 1 << shift
    uint64_t* mark;      // frame mark, as PointArgs (stored by the occlusion hint
                         // kernel when it runs first, else by the bin kernel)
};

struct TileArgs {
    TileView v;
    const uint32_t* stamp_in;
    uint32_t points_per_wg;
    // load-balanced tile pass
    uint32_t* col_sum;       // ntiles + 1 column sums of the table (zero between frames)
    uint16_t* tcol;          // written by the transpose pass (the same array as v.tcol)
    uint32_t* piece_first;   // ntiles + 1 (the same array as v.piece_first)
    uint2* items;            // work items: (tile, piece << 16 | pieces of the tile)
    uint32_t* counters;      // [0] next item, [1] items this frame
    uint32_t piece_records;  // records per piece
};

// Tiles the plan kernel handles in LDS (the bin pass allows no more).
constexpr uint32_t kMaxPlanTiles = 4096;

// Batched binned splat: many clouds, each with one or more views, in one
// launch per pass. Work items are listed in device tables; a block takes
// items blockIdx.x, blockIdx.x + gridDim.x, ...
struct BatchBinArgs {
    const CloudArgs* clouds;
    const BinView* views;
    const uint32_t* first_view;  // clouds + 1 entries: the views of cloud c are
                                 // first_view[c] .. first_view[c + 1] - 1
    const uint2* item;           // (cloud, chunk of P points); clouds with views
    uint32_t items;
    const uint2* disp_item;      // (cloud, chunk): clouds without views, displaced only
    uint32_t disp_items;
    uint32_t* stamp_out;
    uint32_t stamp;
    uint32_t shift;
};

// Tile items are (view, tile << 3 | split); merge and seam items (view, tile << 3).
// A view of ~0u is a padding item that does nothing.
struct BatchTileArgs {
    const TileView* views;
    const uint2* item;
    uint32_t items;
    const uint32_t* stamp_in;
    uint32_t points_per_wg;
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
// Stores the device clock (wall_clock64) at *slot when the stream reaches it.
hipError_t launch_mark(uint64_t* slot, hipStream_t s);
// Copies `bytes` from pinned, host-coherent memory (src: its device address,
// 8-byte aligned) to device memory (dst, 8-byte aligned) with a kernel in
// stream order: no switch to a copy engine between the kernels around it.
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

// Bin workgroup shapes that have a culled bin kernel: 1024 threads of 16
// points would need more registers than four waves per SIMD allow.
__host__ __device__ constexpr bool cull_shape_ok(int ppt, uint32_t threads) {
    return !(ppt == 16 && threads == 1024);
}

// Binned splat. Tile side 1 << shift with shift in {4, 5, 6}; bin workgroups
// of `threads` in {256, 512, 1024} threads with points per thread in
// {4, 8, 16} (chunk P = threads * ppt points); splits per tile in
// {1, 2, 4, 8}.
constexpr uint32_t kMaxLdsBytes = 163840;  // per workgroup on gfx950
bool binned_shape_ok(int shift, int ppt, uint32_t threads, uint32_t splits);
size_t bin_lds_bytes(int ppt, uint32_t threads, uint32_t ntiles);
// cull: the kernel reads the view's cull records (3D only).
Launch bin_launch(int dim, bool wrap, Phase phase, int ppt, uint32_t threads, uint32_t n,
                  uint32_t ntiles, bool cull = false);
Launch tile_launch(int footprint, int shift, uint32_t ntiles, uint32_t splits);
Launch merge_launch(int footprint, int shift, uint32_t ntiles);
// 1x1 footprint, one split: the tile pass resolves to RGBA8 itself (no merge).
Launch tile_fused_launch(int shift, uint32_t ntiles);
// Occlusion cull records of a 3D view for this frame (BinArgs of the frame:
// step, camera, stamp); the bin kernel of the frame follows it.
Launch hint_launch(int shift, bool wrap, uint32_t ntiles);
Launch seam_launch(int shift, uint32_t ntiles);
// Load-balanced tile pass: the table made tile-major with the tiles' record
// totals, the plan, then a persistent grid of tile workgroups over the work
// list. The tile-major rows hold tcol_stride(num_wg) entries.
uint32_t tcol_stride(uint32_t num_wg);
Launch transpose_launch(uint32_t ntiles, uint32_t num_wg);
Launch plan_launch();
Launch tile_list_launch(int footprint, int shift, uint32_t grid_blocks);

// Batched binned splat. grid_blocks = 0 launches one block per item;
// otherwise the launch is persistent, each block looping over items.
Launch batch_bin_launch(int dim, Phase phase, int ppt, uint32_t threads, uint32_t items,
                        uint32_t max_tiles, uint32_t grid_blocks);
Launch batch_displace_launch(int dim, int ppt, uint32_t threads, uint32_t items,
                             uint32_t grid_blocks);
Launch batch_tile_launch(int footprint, int shift, uint32_t items, uint32_t grid_blocks);
Launch batch_merge_launch(int footprint, int shift, uint32_t items, uint32_t grid_blocks);
Launch batch_seam_launch(int shift, uint32_t items, uint32_t grid_blocks);

}  // namespace mm
