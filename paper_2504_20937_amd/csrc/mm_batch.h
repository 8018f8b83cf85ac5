// A launch plan of the batched binned splat: a set of clouds and views, the
// scratch of every view, the device work tables and the frame graph. Used
// by batches (fixed clouds and views) and by the server (one plan per
// launch shape).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "mm_host.h"

namespace mmb {

struct Cloud {
    mm::CloudArgs args{};
    uint64_t n = 0;
    bool active = true;  // has bin items (is displaced and drawn) in this plan
};

struct PlanView {
    uint32_t cloud = 0;
    uint32_t width = 0, height = 0;
    float view_proj[16] = {};
    bool full_clear = false;   // frame buffer holds no earlier frame of this view
    uint32_t prev_stamp = 0;   // stamp of the frame buffer's previous frame (0: the previous launch's)
    uint32_t* colour = nullptr;
    bool owns_colour = false;
    // set by shape_views
    uint32_t tiles_x = 0, tiles_y = 0, ntiles = 0, num_wg = 0, splits = 0;
    // scratch (owned by the batch, or lent by the server)
    uint32_t* active = nullptr;  // ntiles tile stamps
    uint64_t* seg = nullptr;
    uint16_t* table = nullptr;
    uint64_t* part = nullptr;
    uint64_t* border = nullptr;
    uint64_t* apron = nullptr;
};

// Host images of one launch's work tables: a static part (TileView per view,
// first_view, bin / tile / merge / displace-only items) and a per-frame part
// (CloudArgs per cloud, BinView per view).
struct TableImage {
    std::vector<unsigned char> stat, frame;
    size_t o_first = 0, o_bin = 0, o_tile = 0, o_merge = 0, o_disp = 0, o_views = 0;
    uint32_t n_bin = 0, n_disp = 0, n_tile = 0, n_merge = 0, max_tiles = 0;

    mm::CloudArgs& cloud(size_t c) { return reinterpret_cast<mm::CloudArgs*>(frame.data())[c]; }
    mm::BinView& view(size_t v) {
        return reinterpret_cast<mm::BinView*>(frame.data() + o_views)[v];
    }
};

struct Node {
    mm::Launch l;
    void* arg;  // argument block (copied into a graph when it is built)
};

// Tiles, bin workgroups and splits of every view (splits 0: by cloud size).
// Tiles, bin workgroups and splits of every view; auto splits (splits == 0)
// never exceed max_splits, which the caller's partial-block buffers hold.
void shape_views(std::vector<PlanView>& views, const std::vector<Cloud>& clouds, uint32_t side,
                 uint32_t P, uint32_t splits, uint32_t max_splits);
// Work tables of a launch; views grouped by cloud, their scratch set. With
// the 1x1 footprint, views of one split get no merge items (the tile pass
// resolves them).
mm_status build_tables(const std::vector<Cloud>& clouds, const std::vector<PlanView>& views,
                       uint32_t P, uint32_t footprint, TableImage& out);
// Argument blocks over device copies of the two images.
void bind_args(const TableImage& img, const unsigned char* dstat, const unsigned char* dframe,
               uint32_t* stamp_slot, uint32_t shift, uint32_t P, mm::BatchBinArgs& b,
               mm::BatchTileArgs& t, mm::BatchTileArgs& m);
// The launch sequence: bin, displace-only (if any), tile, merge, seam (3x3).
std::vector<Node> make_nodes(mm_domain domain, uint32_t footprint, uint32_t shift, uint32_t ppt,
                             uint32_t threads, const TableImage& img, uint32_t grid_blocks,
                             mm::BatchBinArgs* b, mm::BatchTileArgs* t, mm::BatchTileArgs* m);
void xcd_tile_items(const std::vector<PlanView>& views, std::vector<uint2>& out);

struct Plan {
    static constexpr int kRing = 4;

    mm_domain domain = MM_DOMAIN_3D;
    uint32_t footprint = 1;
    std::vector<Cloud> clouds;
    std::vector<PlanView> views;  // grouped by cloud, in cloud order

    mm_batch_tuning tuning{};
    uint32_t shift = 5, ppt = 16, threads = 256, P = 4096, total_tiles = 0;
    uint32_t* active = nullptr;   // tile stamps of all views, then the frame stamp
    uint32_t stamp = 0;
    TableImage img;
    void* dev_static = nullptr;
    void* dev_frame = nullptr;
    void* ring[kRing] = {};       // pinned, host-coherent staging of the per-frame image
    void* ring_dev[kRing] = {};   // the same slots' device addresses
    hipEvent_t ring_ev[kRing] = {};
    int ring_next = 0;
    mm::BatchBinArgs bargs{};
    mm::BatchTileArgs targs{}, margs{};
    std::vector<Node> nodes;      // [0] is the bin pass
    mm::Launch render_bin{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t first = nullptr;
    bool ready = false;

    mm::CloudArgs& cloud_slot(size_t c) { return img.cloud(c); }
    mm::BinView& view_slot(size_t v) { return img.view(v); }

    // Resolves zero (auto) fields of a requested tuning against the views.
    mm_status resolve(const mm_batch_tuning& req, mm_batch_tuning& out) const;
    // Allocates scratch, writes the work tables, fills argument blocks.
    mm_status setup(mm_instance inst, const mm_batch_tuning& t);
    mm_status build_graph();
    void free_scratch();
    mm_status next_stamp(hipStream_t s);
    // Copies the per-frame image (steps, cameras) to the device, in stream
    // order, with a kernel reading the pinned slot.
    mm_status upload_frame(hipStream_t s);
    mm_status launch_graph(hipStream_t s);
    // Render only: the bin pass without displacement, then the tile passes.
    mm_status launch_render(hipStream_t s);
};

}  // namespace mmb
