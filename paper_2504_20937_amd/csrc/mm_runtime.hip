// C ABI runtime: instances, allocations, views and the per-frame graph.
//
// A frame is one hipGraph. Direct splat: [point kernel: displace + project
// + atomicMin] -> [resolve]. Binned splat: [bin kernel: displace + project +
// LDS sort by tile] -> [tile kernel: LDS min + resolve] (-> [seam kernel] for
// 3x3 footprints). The graph is built once per view (and per tuning); per
// frame only the first node's argument block (step, camera, frame stamp) is
// replaced with hipGraphExecKernelNodeSetParams before hipGraphLaunch, so a
// frame costs two host calls and no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "mm_host.h"

namespace {

// Events of a timed frame graph: before the first node, before the point
// pass (after the occlusion hint kernel, if any), after the point pass, and
// after the last node.
constexpr int kFrameEvents = 4;

struct FrameGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t per_frame[2] = {nullptr, nullptr};  // nodes whose arguments change per frame
    hipGraphNode_t ev[kFrameEvents] = {nullptr, nullptr, nullptr, nullptr};
};

// Most frames one graph launch takes (mm_step_render_frames).
constexpr uint32_t kMaxGraphFrames = 64;

// Several frames in one graph: the frame's kernels `frames` times in a chain;
// the first frame carries the timed graph's event nodes, pointed at spare
// events when that frame is not profiled.
struct MultiGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t frames = 0;
    std::vector<hipGraphNode_t> per_frame;  // frame f, per-frame node j: f * frame_nodes + j
    hipGraphNode_t ev[kFrameEvents] = {nullptr, nullptr, nullptr, nullptr};
};

}  // namespace

struct mm_view_s {
    mm_instance inst;
    mm_alloc position;
    // colour source (mm_set_colour): palette table and optional index buffer
    mm_alloc pal_table = nullptr;
    mm_alloc pal_index = nullptr;
    mm::Palette pal{};
    mm_view_desc desc;
    mm_tuning tuning{};
    uint32_t req_splat = MM_SPLAT_AUTO;  // splat of the last tuning request
    uint32_t* colour = nullptr;
    // direct splat
    uint64_t* depth = nullptr;
    // binned splat
    uint64_t* seg = nullptr;
    uint16_t* table = nullptr;
    uint32_t* active = nullptr;  // ntiles stamps + 1 slot for the frame stamp
    uint64_t* part = nullptr;
    uint64_t* border = nullptr;
    uint64_t* apron = nullptr;
    // occlusion cull: per-tile cull records and last frame's winner per pixel
    uint32_t* cull = nullptr;
    uint32_t* hint = nullptr;
    // load-balanced tile pass
    uint32_t* col_sum = nullptr;
    uint16_t* tcol = nullptr;
    uint32_t* piece_first = nullptr;
    uint2* items = nullptr;
    uint32_t* counters = nullptr;
    uint32_t tiles_x = 0, tiles_y = 0, ntiles = 0, num_wg = 0, stamp = 0;
    // kernel arguments
    mm::PointArgs args{};
    mm::ResolveArgs rargs{};
    mm::BinArgs bargs{};
    mm::TileArgs targs{};
    // frame graph kernels in order; the first frame_nodes take the per-frame
    // arguments (the occlusion hint kernel, if any, then the point pass), the
    // rest are the tile passes
    std::vector<mm::Launch> nodes;
    uint32_t frame_nodes = 1;
    FrameGraph plain, timed;
    MultiGraph multi;
    hipEvent_t spare[kFrameEvents] = {nullptr, nullptr, nullptr, nullptr};  // unprofiled multi frames
    std::vector<hipEvent_t> events;  // kFrameEvents per profiled frame
    uint32_t prof_cap = 0, prof_count = 0;
    uint32_t prof_every = 1, prof_skip = 0;  // record 1 frame in prof_every
    bool profiling = false;
    // frame marks: the device clock when each frame's first kernel starts, and
    // one more after the last frame (mark_cap slots)
    uint64_t* mark_ring = nullptr;
    uint32_t mark_cap = 0, mark_count = 0;
    bool marking = false;
    // Frame overlap (binned only): frame f is binned into record set f & 1 on
    // the instance stream while frame f - 1 is drawn from the other set on
    // the render stream. Set 1 mirrors seg / table / active.
    bool overlap = false;
    uint64_t* seg1 = nullptr;
    uint16_t* table1 = nullptr;
    uint32_t* active1 = nullptr;
    mm::BinArgs bargs1{};
    mm::TileArgs targs1{};
    hipStream_t rstream = nullptr;
    hipEvent_t ev_bin[2] = {nullptr, nullptr};     // set binned (instance stream)
    hipEvent_t ev_drawn[2] = {nullptr, nullptr};   // set drawn (render stream)
    int pending = -1;                              // set binned, not yet drawn
    int last_drawn = -1;                           // set whose frame the colour holds
};

namespace {

using namespace mmh;

thread_local std::string g_last_error;

void fill_point_args(mm_view v) {
    const mm_view_desc& d = v->desc;
    mm::PointArgs& a = v->args;
    a.c = cloud_args(v->position->ptr, d.element_count, d.seed, d.amplitude);
    a.g = view_geom(d.width, d.height, d.view_proj);
    a.depth = v->depth;
}

bool binned(mm_view v) { return v->tuning.splat == MM_SPLAT_BINNED; }

// Argument block of frame-graph node k.
void* node_arg(mm_view v, size_t k) {
    if (binned(v)) return k < v->frame_nodes ? static_cast<void*>(&v->bargs) : static_cast<void*>(&v->targs);
    return k == 0 ? static_cast<void*>(&v->args) : static_cast<void*>(&v->rargs);
}

void destroy_graph(FrameGraph& fg) {
    if (fg.exec) (void)hipGraphExecDestroy(fg.exec);
    if (fg.graph) (void)hipGraphDestroy(fg.graph);
    fg = FrameGraph{};
}

void destroy_multi(MultiGraph& mg) {
    if (mg.exec) (void)hipGraphExecDestroy(mg.exec);
    if (mg.graph) (void)hipGraphDestroy(mg.graph);
    mg = MultiGraph{};
}

// The frame graph: the kernels of v->nodes in a chain; with timed set,
// event-record nodes go before the first kernel, before and after the point
// pass, and at the end.
mm_status build_graph(mm_view v, bool timed, FrameGraph& out) {
    FrameGraph fg;
    MM_HIP(hipGraphCreate(&fg.graph, 0));
    hipError_t err = hipSuccess;
    hipGraphNode_t prev = nullptr;
    auto add_event = [&](int j) {
        if (err != hipSuccess) return;
        err = hipGraphAddEventRecordNode(&fg.ev[j], fg.graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                         v->events[j]);
        prev = fg.ev[j];
    };
    const size_t point = v->frame_nodes - 1;  // the point pass
    if (timed) add_event(0);
    for (size_t k = 0; k < v->nodes.size() && err == hipSuccess; ++k) {
        if (timed && k == point) add_event(1);
        void* args[] = {node_arg(v, k)};
        hipKernelNodeParams p = node_params(v->nodes[k], args);
        hipGraphNode_t n = nullptr;
        err = hipGraphAddKernelNode(&n, fg.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (k < v->frame_nodes) fg.per_frame[k] = n;
        prev = n;
        if (timed && k == point) add_event(2);
    }
    if (timed) add_event(3);
    if (err == hipSuccess) err = hipGraphInstantiate(&fg.exec, fg.graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        destroy_graph(fg);
        return fail(MM_ERR_HIP, "building the frame graph failed: %s", hipGetErrorString(err));
    }
    out = fg;
    return MM_OK;
}

// `frames` frames of v->nodes in one chain (MultiGraph).
mm_status build_multi(mm_view v, uint32_t frames, MultiGraph& out) {
    for (hipEvent_t& e : v->spare)
        if (!e) MM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    MultiGraph mg;
    MM_HIP(hipGraphCreate(&mg.graph, 0));
    mg.per_frame.assign(static_cast<size_t>(frames) * v->frame_nodes, nullptr);
    hipError_t err = hipSuccess;
    hipGraphNode_t prev = nullptr;
    auto add_event = [&](int j) {
        if (err != hipSuccess) return;
        err = hipGraphAddEventRecordNode(&mg.ev[j], mg.graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                         v->spare[j]);
        prev = mg.ev[j];
    };
    const size_t point = v->frame_nodes - 1;
    for (uint32_t f = 0; f < frames && err == hipSuccess; ++f) {
        if (f == 0) add_event(0);
        for (size_t k = 0; k < v->nodes.size() && err == hipSuccess; ++k) {
            if (f == 0 && k == point) add_event(1);
            void* args[] = {node_arg(v, k)};
            hipKernelNodeParams p = node_params(v->nodes[k], args);
            hipGraphNode_t n = nullptr;
            err = hipGraphAddKernelNode(&n, mg.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
            if (k < v->frame_nodes) mg.per_frame[static_cast<size_t>(f) * v->frame_nodes + k] = n;
            prev = n;
            if (f == 0 && k == point) add_event(2);
        }
        if (f == 0) add_event(3);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&mg.exec, mg.graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        destroy_multi(mg);
        return fail(MM_ERR_HIP, "building the %u-frame graph failed: %s", frames, hipGetErrorString(err));
    }
    mg.frames = frames;
    out = std::move(mg);
    return MM_OK;
}

void free_splat_buffers(mm_view v) {
    for (void* p : {static_cast<void*>(v->depth), static_cast<void*>(v->seg),
                    static_cast<void*>(v->table), static_cast<void*>(v->active),
                    static_cast<void*>(v->part), static_cast<void*>(v->border),
                    static_cast<void*>(v->apron), static_cast<void*>(v->col_sum),
                    static_cast<void*>(v->tcol),
                    static_cast<void*>(v->piece_first), static_cast<void*>(v->items),
                    static_cast<void*>(v->counters)})
        if (p) (void)hipFree(p);
    for (void* p : {static_cast<void*>(v->seg1), static_cast<void*>(v->table1),
                    static_cast<void*>(v->active1), static_cast<void*>(v->cull),
                    static_cast<void*>(v->hint)})
        if (p) (void)hipFree(p);
    v->cull = nullptr;
    v->hint = nullptr;
    v->seg1 = nullptr;
    v->table1 = nullptr;
    v->active1 = nullptr;
    v->col_sum = nullptr;
    v->tcol = nullptr;
    v->piece_first = nullptr;
    v->items = nullptr;
    v->counters = nullptr;
    v->depth = nullptr;
    v->seg = nullptr;
    v->table = nullptr;
    v->active = nullptr;
    v->part = nullptr;
    v->border = nullptr;
    v->apron = nullptr;
}

// Resolves AUTO and zero fields of a requested tuning for this view.
mm_status resolve_tuning(const mm_view_desc& d, const mm_tuning& req, mm_tuning& out) {
    out = req;
    if (out.splat > MM_SPLAT_BINNED)
        return fail(MM_ERR_INVALID_ARG, "tuning: splat %u unknown", out.splat);
    auto tiles = [&](uint32_t side) {
        return ((d.width + side - 1) / side) * ((d.height + side - 1) / side);
    };
    if (out.splat == MM_SPLAT_AUTO) {
        // Direct atomics for a small cloud on a small screen, where the binned
        // path's fixed per-frame cost dominates (2^16 points at 1080p: 20.8 us
        // against 32.1 us a frame; 2^18: 28.9 against 34.4; 2^20: 62.5 against
        // 38.8); else binned when the screen fits the tile table.
        const uint64_t px = static_cast<uint64_t>(d.width) * d.height;
        if (d.element_count <= (1u << 18) && px <= (1u << 21))
            out.splat = MM_SPLAT_DIRECT;
        else
            out.splat = (tiles(64) <= 4096u) ? MM_SPLAT_BINNED : MM_SPLAT_DIRECT;
    }
    if (out.occlusion_cull > MM_CULL_OFF)
        return fail(MM_ERR_INVALID_ARG, "tuning: occlusion_cull %u unknown", out.occlusion_cull);
    if (out.splat == MM_SPLAT_DIRECT) {
        if (out.occlusion_cull == MM_CULL_ON)
            return fail(MM_ERR_UNSUPPORTED, "tuning: the occlusion cull needs the binned splat");
        out.tile = 0;
        out.points_per_thread = 0;
        out.splits = 0;
        out.bin_threads = 0;
        out.piece_records = 0;
        out.occlusion_cull = MM_CULL_OFF;
        return MM_OK;
    }
    // a view asking for the occlusion cull (3D, 1x1, one static split) by
    // default bins 512 threads of 16 points: the culled bin kernel holds its
    // points longer and keeps two workgroups per CU only in that shape
    const bool cull_default = d.domain == MM_DOMAIN_3D && d.footprint == 1 &&
                              out.occlusion_cull == MM_CULL_ON &&
                              (out.splits == 0 || out.splits == 1) &&
                              (out.piece_records == 0 || out.piece_records == MM_PIECES_STATIC);
    if (out.tile == 0) out.tile = tiles(32) <= 4096u ? 32u : 64u;
    if (out.points_per_thread == 0) out.points_per_thread = cull_default && out.bin_threads != 1024 ? 16 : 8;
    if (out.bin_threads == 0) out.bin_threads = cull_default && out.points_per_thread == 16 ? 512 : 1024;
    // Auto: static splits up to 8191 bin workgroups (2^26 points at the
    // default chunk), where the balanced pass's count and plan kernels cost
    // more than the imbalance they remove; beyond, balanced pieces of about
    // N / 1024 records (2^28 clustered points at 4K: 1.5x the static pass).
    if (out.piece_records == 0) {
        const uint64_t P = static_cast<uint64_t>(out.bin_threads) * out.points_per_thread;
        const uint64_t wgs = (d.element_count + P - 1) / P;
        if (wgs < 8192 || out.splits != 0) {  // explicit splits ask for the static pass
            out.piece_records = MM_PIECES_STATIC;
        } else {
            const uint64_t r = (d.element_count / 1024 + 1023) / 1024 * 1024;
            out.piece_records = static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(r, 4096), 1u << 20));
        }
    }
    if (out.piece_records != MM_PIECES_STATIC) {
        // balanced by load; a tile's piece count must fit 16 bits
        if (out.piece_records < 1024 || out.piece_records > (1u << 20))
            return fail(MM_ERR_INVALID_ARG, "tuning: piece_records %u outside [1024, 2^20]", out.piece_records);
        if (static_cast<uint64_t>(out.piece_records) * 65535u < d.element_count)
            return fail(MM_ERR_INVALID_ARG, "tuning: piece_records %u too small for %llu points",
                        out.piece_records, (unsigned long long)d.element_count);
        out.splits = 0;
    } else if (out.splits == 0) {
        // 1x1 footprint: one 1024-thread workgroup per tile that resolves the
        // tile itself (no partial blocks, no merge pass; 2^24 points at 1080p:
        // 42.6 us for the tile pass against 47.3 us with 2 splits and the
        // merge). 3x3: enough workgroups per tile to spread the densest tiles
        // over the chip once the bin workgroups are many.
        const uint64_t P = static_cast<uint64_t>(out.bin_threads) * out.points_per_thread;
        const uint64_t wgs = (d.element_count + P - 1) / P;
        out.splits = d.footprint == 1 || wgs < 256 ? 1u : 2u;
    }
    if (!mm::binned_shape_ok(static_cast<int>(shift_of(out.tile)), static_cast<int>(out.points_per_thread),
                             out.bin_threads, out.splits == 0 ? 1u : out.splits))
        return fail(MM_ERR_INVALID_ARG,
                    "tuning: tile %u / points_per_thread %u / bin_threads %u / splits %u not in "
                    "{16,32,64} x {4,8,16} x {256,512,1024} x {1,2,4,8}",
                    out.tile, out.points_per_thread, out.bin_threads, out.splits);
    if (tiles(out.tile) > kMaxTiles)
        return fail(MM_ERR_UNSUPPORTED, "tuning: %ux%u screen needs %u tiles of %u px (max %u)",
                    d.width, d.height, tiles(out.tile), out.tile, kMaxTiles);
    // (the cull's window masks and bases: 12 bytes per 64 records)
    const size_t lds = mm::bin_lds_bytes(static_cast<int>(out.points_per_thread), out.bin_threads,
                                         tiles(out.tile)) +
                       12u * out.bin_threads * out.points_per_thread / 64u + 4u;
    if (lds + 1024 > mm::kMaxLdsBytes)
        return fail(MM_ERR_UNSUPPORTED, "tuning: a bin workgroup would need %zu bytes of LDS", lds);
    // the cull takes 3D depths and the one-split 1x1 pass, which resolves
    // each tile whole and writes its winners as the next frame's hints
    const bool cullable = d.domain == MM_DOMAIN_3D && d.footprint == 1 &&
                          out.piece_records == MM_PIECES_STATIC && out.splits == 1 &&
                          mm::cull_shape_ok(static_cast<int>(out.points_per_thread), out.bin_threads);
    if (out.occlusion_cull == MM_CULL_ON && !cullable)
        return fail(MM_ERR_UNSUPPORTED,
                    "tuning: the occlusion cull needs a 3D view, the 1x1 footprint, one static split "
                    "and a bin shape other than 1024 threads x 16 points");
    // auto leaves the cull off: measured on MI355X at 2^24 points, 1080p, the
    // culled bin pass loses more time than the records it saves
    out.occlusion_cull = cullable && out.occlusion_cull == MM_CULL_ON ? MM_CULL_ON : MM_CULL_OFF;
    return MM_OK;
}

// Allocates the splat scratch buffers of v->tuning, fills the kernel
// argument blocks and builds the plain frame graph.
mm_status setup_splat(mm_view v) {
    mm_instance inst = v->inst;
    const mm_view_desc& d = v->desc;
    const uint64_t npix = static_cast<uint64_t>(d.width) * d.height;
    const int dim = static_cast<int>(d.domain), foot = static_cast<int>(d.footprint);
    const bool wrap = d.wrap != 0;
    hipError_t e = hipSuccess;
    v->nodes.clear();
    v->frame_nodes = 1;
    if (!binned(v)) {
        e = alloc_n(&v->depth, npix);
        if (e == hipSuccess) e = mm::launch_fill(v->depth, npix, mm::kEmptyKey, inst->stream);
        if (e != hipSuccess) return hip_fail(e, "direct splat buffers");
        fill_point_args(v);
        v->rargs = mm::ResolveArgs{v->depth, v->colour, npix, v->args.c.seed_lo, v->args.c.seed_hi,
                                   v->pal};
        v->nodes.push_back(mm::point_launch(dim, foot, wrap, mm::kDisplaceRender, v->args.c.n));
        v->nodes.push_back(mm::resolve_launch(npix));
    } else {
        const uint32_t side = v->tuning.tile, shift = shift_of(side);
        const int ppt = static_cast<int>(v->tuning.points_per_thread);
        const uint32_t nthreads = v->tuning.bin_threads;
        const uint64_t P = static_cast<uint64_t>(nthreads) * static_cast<uint64_t>(ppt);
        v->tiles_x = (d.width + side - 1) / side;
        v->tiles_y = (d.height + side - 1) / side;
        v->ntiles = v->tiles_x * v->tiles_y;
        v->num_wg = static_cast<uint32_t>((d.element_count + P - 1) / P);
        e = alloc_n(&v->seg, static_cast<uint64_t>(v->num_wg) * P);
        if (e == hipSuccess) e = alloc_n(&v->table, static_cast<uint64_t>(v->num_wg) * (v->ntiles + 1));
        if (e == hipSuccess) e = alloc_n(&v->active, static_cast<uint64_t>(v->ntiles) + 1);
        if (e == hipSuccess)
            e = hipMemsetAsync(v->active, 0, (static_cast<size_t>(v->ntiles) + 1) * 4, inst->stream);
        const uint64_t side_a = foot == 3 ? side + 2 : side;
        const bool balanced = v->tuning.piece_records != MM_PIECES_STATIC;
        // balanced: every tile holds at most total / R + 1 pieces
        const uint64_t blocks = balanced ? (d.element_count + v->tuning.piece_records - 1) /
                                                   v->tuning.piece_records + v->ntiles
                                         : static_cast<uint64_t>(v->ntiles) * v->tuning.splits;
        if (e == hipSuccess) e = alloc_n(&v->part, blocks * side_a * side_a);
        if (e == hipSuccess && balanced) {
            e = alloc_n(&v->col_sum, static_cast<uint64_t>(v->ntiles) + 1);
            if (e == hipSuccess)
                e = hipMemsetAsync(v->col_sum, 0, sizeof(uint32_t) * (static_cast<size_t>(v->ntiles) + 1),
                                   inst->stream);
            if (e == hipSuccess)
                e = alloc_n(&v->tcol, (static_cast<uint64_t>(v->ntiles) + 1) * mm::tcol_stride(v->num_wg));
            if (e == hipSuccess) e = alloc_n(&v->piece_first, static_cast<uint64_t>(v->ntiles) + 1);
            if (e == hipSuccess) e = alloc_n(&v->items, blocks);
            if (e == hipSuccess) e = alloc_n(&v->counters, 2);
        }
        if (e == hipSuccess && foot == 3) {
            e = alloc_n(&v->border, static_cast<uint64_t>(v->ntiles) * 4 * side);
            if (e == hipSuccess) e = alloc_n(&v->apron, static_cast<uint64_t>(v->ntiles) * (4 * side + 4));
        }
        // not with frame overlap: the draw of frame f - 1, which writes the
        // hints, runs beside the bin pass of frame f
        const bool cull = v->tuning.occlusion_cull == MM_CULL_ON && !v->overlap;
        if (e == hipSuccess && cull) {
            // hints start empty (no bound until a frame is drawn); cull records
            // are written by every frame's hint kernel before they are read
            e = alloc_n(&v->cull, static_cast<uint64_t>(v->ntiles) * mm::cull_words(side));
            if (e == hipSuccess)
                e = hipMemsetAsync(v->cull, 0, static_cast<size_t>(v->ntiles) * mm::cull_words(side) * 4,
                                   inst->stream);
            if (e == hipSuccess) e = alloc_n(&v->hint, static_cast<uint64_t>(v->ntiles) * side * side);
            if (e == hipSuccess)
                e = hipMemsetAsync(v->hint, 0xFF, static_cast<size_t>(v->ntiles) * side * side * 4,
                                   inst->stream);
        }
        if (e != hipSuccess) return hip_fail(e, "binned splat buffers");
        v->stamp = 0;
        fill_point_args(v);
        mm::BinArgs& b = v->bargs;
        b.c = v->args.c;
        b.v.g = v->args.g;
        b.v.seg = v->seg;
        b.v.table = v->table;
        b.v.active = v->active;
        b.v.tiles_x = v->tiles_x;
        b.v.ntiles = v->ntiles;
        b.stamp_out = v->active + v->ntiles;
        b.stamp = 0;
        b.shift = shift;
        b.v.cull = v->cull;
        b.v.hint = v->hint;
        mm::TileArgs& t = v->targs;
        t.v.seg = v->seg;
        t.v.table = v->table;
        t.v.active = v->active;
        t.v.part = v->part;
        t.v.border = v->border;
        t.v.apron = v->apron;
        t.v.colour = v->colour;
        t.v.width = d.width;
        t.v.height = d.height;
        t.v.tiles_x = v->tiles_x;
        t.v.tiles_y = v->tiles_y;
        t.v.ntiles = v->ntiles;
        t.v.num_wg = v->num_wg;
        t.v.splits = v->tuning.splits;
        t.v.piece_first = v->piece_first;
        t.v.tcol = v->tcol;
        t.v.tcol_stride = balanced ? mm::tcol_stride(v->num_wg) : 0u;
        t.v.seed_lo = v->args.c.seed_lo;
        t.v.seed_hi = v->args.c.seed_hi;
        t.v.pal = v->pal;
        t.v.hint = v->hint;
        t.v.cull = v->cull;
        t.stamp_in = v->active + v->ntiles;
        t.points_per_wg = static_cast<uint32_t>(P);
        t.col_sum = v->col_sum;
        t.tcol = v->tcol;
        t.piece_first = v->piece_first;
        t.items = v->items;
        t.counters = v->counters;
        t.piece_records = balanced ? v->tuning.piece_records : 0u;
        if (v->overlap) {
            // second record set; every tile not drawn in a frame is cleared,
            // since the other set's stamps say nothing about this frame buffer
            e = alloc_n(&v->seg1, static_cast<uint64_t>(v->num_wg) * P);
            if (e == hipSuccess) e = alloc_n(&v->table1, static_cast<uint64_t>(v->num_wg) * (v->ntiles + 1));
            if (e == hipSuccess) e = alloc_n(&v->active1, static_cast<uint64_t>(v->ntiles) + 1);
            if (e == hipSuccess)
                e = hipMemsetAsync(v->active1, 0, (static_cast<size_t>(v->ntiles) + 1) * 4, inst->stream);
            if (e != hipSuccess) return hip_fail(e, "overlapped record set");
            t.v.full_clear = 1;
            v->bargs1 = b;
            v->bargs1.v.seg = v->seg1;
            v->bargs1.v.table = v->table1;
            v->bargs1.v.active = v->active1;
            v->bargs1.stamp_out = v->active1 + v->ntiles;
            v->targs1 = t;
            v->targs1.v.seg = v->seg1;
            v->targs1.v.table = v->table1;
            v->targs1.v.active = v->active1;
            v->targs1.stamp_in = v->active1 + v->ntiles;
        }
        v->pending = -1;
        v->last_drawn = -1;
        if (cull) v->nodes.push_back(mm::hint_launch(static_cast<int>(shift), wrap, v->ntiles));
        v->frame_nodes = cull ? 2u : 1u;
        v->nodes.push_back(mm::bin_launch(dim, wrap, mm::kDisplaceRender, ppt, nthreads, v->args.c.n,
                                          v->ntiles, cull));
        if (balanced) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, inst->device) != hipSuccess ||
                cus <= 0)
                cus = 256;
            const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(blocks, 2ull * cus));
            v->nodes.push_back(mm::transpose_launch(v->ntiles, v->num_wg));
            v->nodes.push_back(mm::plan_launch());
            v->nodes.push_back(mm::tile_list_launch(foot, static_cast<int>(shift), grid));
        } else if (foot == 1 && v->tuning.splits == 1) {
            v->nodes.push_back(mm::tile_fused_launch(static_cast<int>(shift), v->ntiles));
        } else {
            v->nodes.push_back(mm::tile_launch(foot, static_cast<int>(shift), v->ntiles, v->tuning.splits));
        }
        if (!(foot == 1 && !balanced && v->tuning.splits == 1))
            v->nodes.push_back(mm::merge_launch(foot, static_cast<int>(shift), v->ntiles));
        if (foot == 3) v->nodes.push_back(mm::seam_launch(static_cast<int>(shift), v->ntiles));
    }
    return build_graph(v, false, v->plain);
}

void destroy_overlap(mm_view v);

void teardown_splat(mm_view v) {
    if (v->rstream) (void)hipStreamSynchronize(v->rstream);
    destroy_graph(v->plain);
    destroy_graph(v->timed);
    destroy_multi(v->multi);
    v->profiling = false;
    free_splat_buffers(v);
}

// The slot of the next frame mark while marks are left (the frame's first
// kernel stores the clock there), else nullptr.
uint64_t* take_mark(mm_view v) {
    if (!v->marking || v->mark_count >= v->mark_cap) return nullptr;
    return v->mark_ring + v->mark_count++;
}

void destroy_view_resources(mm_view v) {
    teardown_splat(v);
    for (hipEvent_t& e : v->spare) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    destroy_overlap(v);
    for (hipEvent_t e : v->events) (void)hipEventDestroy(e);
    v->events.clear();
    if (v->mark_ring) (void)hipFree(v->mark_ring);
    v->mark_ring = nullptr;
    v->marking = false;
    if (v->colour) (void)hipFree(v->colour);
    v->colour = nullptr;
}

mm_status validate_desc(mm_instance inst, const mm_view_desc* d) {
    if (d->domain != MM_DOMAIN_2D && d->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "view: domain %d is not 2D/3D", (int)d->domain);
    const mm_cloud_desc c{d->position, d->element_count, d->format, d->seed, d->amplitude, d->wrap};
    MM_TRY(validate_cloud(inst, c, d->domain, "view"));
    MM_TRY(validate_screen(d->width, d->height, "view"));
    if (d->footprint != 1 && d->footprint != 3)
        return fail(MM_ERR_INVALID_ARG, "view: footprint %u is not 1 or 3", d->footprint);
    if (d->domain == MM_DOMAIN_3D) MM_TRY(validate_camera(d->view_proj, "view"));
    return MM_OK;
}

mm_status flush_frame(mm_view v);

// Next frame stamp of a binned view; on wrap-around the tile stamps restart
// (an overlapped view first draws its pending frame and lets the render
// stream drain, since the stamps of both record sets are reset).
mm_status next_stamp(mm_view v) {
    if (++v->stamp == 0) {
        if (v->overlap) {
            MM_TRY(flush_frame(v));
            MM_HIP(hipStreamSynchronize(v->rstream));
            MM_HIP(hipMemsetAsync(v->active1, 0, (static_cast<size_t>(v->ntiles) + 1) * 4,
                                  v->inst->stream));
        }
        MM_HIP(hipMemsetAsync(v->active, 0, (static_cast<size_t>(v->ntiles) + 1) * 4,
                              v->inst->stream));
        v->stamp = 1;
    }
    v->bargs.stamp = v->stamp;
    v->bargs1.stamp = v->stamp;
    return MM_OK;
}

mm::BinArgs& set_bin(mm_view v, int k) { return k ? v->bargs1 : v->bargs; }
mm::TileArgs& set_tile(mm_view v, int k) { return k ? v->targs1 : v->targs; }

// Draws record set k (binned on the instance stream) on the render stream:
// the tile, merge (and seam) kernels of the frame, then marks the set free.
mm_status draw_set(mm_view v, int k) {
    MM_HIP(hipStreamWaitEvent(v->rstream, v->ev_bin[k], 0));
    void* args[] = {&set_tile(v, k)};
    for (size_t n = v->frame_nodes; n < v->nodes.size(); ++n)
        MM_HIP(hipLaunchKernel(v->nodes[n].func, v->nodes[n].grid, v->nodes[n].block, args,
                               v->nodes[n].shared, v->rstream));
    MM_HIP(hipEventRecord(v->ev_drawn[k], v->rstream));
    v->last_drawn = k;
    return MM_OK;
}

// Draws the pending frame of an overlapped view, and makes the instance
// stream wait for the last draw, so work after it in stream order sees the
// frame buffer of the last frame.
mm_status flush_frame(mm_view v) {
    if (!v->overlap) return MM_OK;
    if (v->pending >= 0) {
        MM_TRY(draw_set(v, v->pending));
        v->pending = -1;
    }
    if (v->last_drawn >= 0) MM_HIP(hipStreamWaitEvent(v->inst->stream, v->ev_drawn[v->last_drawn], 0));
    return MM_OK;
}

// One overlapped frame: bin (with displacement when phase says so) into the
// free record set on the instance stream, and draw the pending set on the
// render stream beside it. With profiling on, events go before and after the
// bin kernel (instance stream) and after the draw (render stream).
mm_status overlap_frame(mm_view v, mm::Phase phase, uint32_t step) {
    MM_TRY(next_stamp(v));
    const int k = static_cast<int>(v->stamp & 1u);
    mm::BinArgs b = set_bin(v, k);
    b.c.step = step;
    b.mark = take_mark(v);
    hipStream_t s = v->inst->stream;
    // the last draw of set k has read its records
    MM_HIP(hipStreamWaitEvent(s, v->ev_drawn[k], 0));
    hipEvent_t* ev = nullptr;
    if (v->profiling && v->prof_count < v->prof_cap && v->prof_skip++ % v->prof_every == 0)
        ev = &v->events[static_cast<size_t>(kFrameEvents) * v->prof_count++];
    if (ev) MM_HIP(hipEventRecord(ev[0], s));
    if (ev) MM_HIP(hipEventRecord(ev[1], s));
    const mm::Launch bl = mm::bin_launch(static_cast<int>(v->desc.domain), v->desc.wrap != 0, phase,
                                         static_cast<int>(v->tuning.points_per_thread),
                                         v->tuning.bin_threads, v->args.c.n, v->ntiles);
    void* args[] = {&b};
    MM_HIP(hipLaunchKernel(bl.func, bl.grid, bl.block, args, bl.shared, s));
    if (ev) MM_HIP(hipEventRecord(ev[2], s));
    MM_HIP(hipEventRecord(v->ev_bin[k], s));
    if (v->pending >= 0) MM_TRY(draw_set(v, v->pending));
    if (ev) MM_HIP(hipEventRecord(ev[3], v->pending >= 0 ? v->rstream : s));
    v->pending = k;
    return MM_OK;
}

void destroy_overlap(mm_view v) {
    for (hipEvent_t* e : {&v->ev_bin[0], &v->ev_bin[1], &v->ev_drawn[0], &v->ev_drawn[1]}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
    if (v->rstream) (void)hipStreamDestroy(v->rstream);
    v->rstream = nullptr;
    v->overlap = false;
}

// The render stream and events of frame overlap; on failure none is kept.
hipError_t open_overlap(mm_view v) {
    hipError_t e = hipStreamCreateWithFlags(&v->rstream, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&v->ev_bin[0], &v->ev_bin[1], &v->ev_drawn[0], &v->ev_drawn[1]})
        // ordering between two streams of one device: a device-scope release
        if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming | hipEventReleaseToDevice);
    if (e != hipSuccess) {
        destroy_overlap(v);
        return e;
    }
    v->overlap = true;
    return hipSuccess;
}

// After a failed change of tuning or mode: the splat of the tuning the view
// had. If even that cannot be set up the view has no splat (its frames then
// fail with MM_ERR_INVALID_ARG) until a later mm_set_tuning succeeds. The
// message of the first failure is kept.
void restore_splat(mm_view v, const mm_tuning& t, uint32_t req_splat) {
    const std::string first = g_last_error;
    teardown_splat(v);
    v->tuning = t;
    v->req_splat = req_splat;
    if (setup_splat(v) != MM_OK) teardown_splat(v);
    g_last_error = first;
}

}  // namespace

namespace {

// Allocations to let through before one fails (mm_debug_fail_allocations);
// negative: none fails.
std::atomic<int64_t> g_fail_after{-1};

bool inject_failure() {
    int64_t n = g_fail_after.load(std::memory_order_relaxed);
    while (n >= 0) {
        if (g_fail_after.compare_exchange_weak(n, n - 1, std::memory_order_relaxed)) return n == 0;
    }
    return false;
}

}  // namespace

namespace mmh {

hipError_t dev_malloc(void** p, size_t bytes) {
    if (inject_failure()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(void** p, size_t bytes) {
    if (inject_failure()) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, hipHostMallocCoherent);
}

mm_status fail(mm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mm_status validate_cloud(mm_instance inst, const mm_cloud_desc& d, mm_domain domain,
                         const char* what) {
    if (!d.position) return fail(MM_ERR_INVALID_ARG, "%s: position alloc is null", what);
    if (inst->allocs.count(d.position) == 0)
        return fail(MM_ERR_INVALID_ARG, "%s: position is not an alloc of this instance", what);
    if (d.format != MM_FLOAT2 && d.format != MM_FLOAT3)
        return fail(MM_ERR_INVALID_ARG, "%s: format %d is not MM_FLOAT2/MM_FLOAT3", what,
                    (int)d.format);
    if ((int)d.format != (int)domain)
        return fail(MM_ERR_UNSUPPORTED, "%s: format float%d with a %dD domain", what,
                    (int)d.format, (int)domain);
    if (d.element_count < 1 || d.element_count > 0xFFFFFFFFull)
        return fail(MM_ERR_INVALID_ARG, "%s: element_count %llu outside [1, 2^32-1]", what,
                    (unsigned long long)d.element_count);
    const uint64_t stride = 4ull * (uint64_t)d.format;
    if (d.element_count > d.position->bytes / stride)
        return fail(MM_ERR_INVALID_ARG, "%s: %llu points of %llu B exceed the %zu-byte alloc",
                    what, (unsigned long long)d.element_count, (unsigned long long)stride,
                    d.position->bytes);
    if (!amplitude_ok(d.amplitude))
        return fail(MM_ERR_INVALID_ARG, "%s: amplitude %g outside {0} U [2^-64, 2^64]", what,
                    (double)d.amplitude);
    if (d.wrap != 0 && d.wrap != 1) return fail(MM_ERR_INVALID_ARG, "%s: wrap must be 0 or 1", what);
    if (d.wrap && d.amplitude > 1.0f)
        return fail(MM_ERR_INVALID_ARG, "%s: wrap needs amplitude <= 1", what);
    return MM_OK;
}

mm_status validate_screen(uint32_t width, uint32_t height, const char* what) {
    if (width < 2 || height < 2 || width > 16384 || height > 16384 || (width & 1u) ||
        (height & 1u))
        return fail(MM_ERR_INVALID_ARG, "%s: screen %ux%u must be even and in [2, 16384]", what,
                    width, height);
    return MM_OK;
}

mm_status validate_camera(const float m[16], const char* what) {
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(m[k]))
            return fail(MM_ERR_INVALID_ARG, "%s: view_proj[%d] is not finite", what, k);
    return MM_OK;
}

}  // namespace mmh

extern "C" {

int32_t mm_version(void) { return 200; }

mm_status mm_debug_fail_allocations(int64_t after) {
    g_fail_after.store(after < 0 ? -1 : after, std::memory_order_relaxed);
    return MM_OK;
}

const char* mm_last_error(void) { return g_last_error.c_str(); }

const char* mm_status_string(mm_status s) {
    switch (s) {
        case MM_OK: return "MM_OK";
        case MM_ERR_INVALID_ARG: return "MM_ERR_INVALID_ARG";
        case MM_ERR_OUT_OF_MEMORY: return "MM_ERR_OUT_OF_MEMORY";
        case MM_ERR_HIP: return "MM_ERR_HIP";
        case MM_ERR_BUDGET: return "MM_ERR_BUDGET";
        case MM_ERR_IN_USE: return "MM_ERR_IN_USE";
        case MM_ERR_UNSUPPORTED: return "MM_ERR_UNSUPPORTED";
        case MM_ERR_NOT_READY: return "MM_ERR_NOT_READY";
        default: return "MM_ERR_UNKNOWN";
    }
}

mm_status mm_create_instance(const mm_instance_desc* desc, mm_instance* out) {
    if (!desc || !out) return fail(MM_ERR_INVALID_ARG, "create_instance: null argument");
    int count = 0;
    MM_HIP(hipGetDeviceCount(&count));
    if (desc->device < 0 || desc->device >= count)
        return fail(MM_ERR_INVALID_ARG, "create_instance: device %d of %d", desc->device, count);
    DeviceGuard guard(desc->device);
    hipStream_t s = static_cast<hipStream_t>(desc->stream);
    bool owns = false;
    if (!s) {
        MM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        owns = true;
    }
    mm_instance inst = new (std::nothrow) mm_instance_s{desc->device, s, owns, {}, {}, {}, {}, {}, {}};
    if (!inst) {
        if (owns) (void)hipStreamDestroy(s);
        return fail(MM_ERR_OUT_OF_MEMORY, "create_instance: host allocation");
    }
    *out = inst;
    return MM_OK;
}

mm_status mm_synchronize(mm_instance inst) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "synchronize: null instance");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    return MM_OK;
}

mm_status mm_destroy_view(mm_view v);

mm_status mm_destroy_instance(mm_instance inst) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "destroy_instance: null instance");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    std::vector<mm_server> servers(inst->servers.begin(), inst->servers.end());
    for (mm_server v : servers) mm_destroy_server(v);
    std::vector<mm_grid> grids(inst->grids.begin(), inst->grids.end());
    for (mm_grid g : grids) mm_destroy_grid(g);
    std::vector<mm_edges> edge_views(inst->edges.begin(), inst->edges.end());
    for (mm_edges g : edge_views) mm_destroy_edges(g);
    std::vector<mm_batch> batches(inst->batches.begin(), inst->batches.end());
    for (mm_batch b : batches) mm_destroy_batch(b);
    std::vector<mm_view> views(inst->views.begin(), inst->views.end());
    for (mm_view v : views) mm_destroy_view(v);
    for (mm_alloc a : inst->allocs) {
        if (a->owned) (void)hipFree(a->ptr);
        delete a;
    }
    for (hipEvent_t e : {inst->prep_ev, inst->upd_ev})
        if (e) (void)hipEventDestroy(e);
    if (inst->owns_stream) (void)hipStreamDestroy(inst->stream);
    delete inst;
    return MM_OK;
}

// Ordering between the instance stream and a simulation's stream on one
// device: a device-scope release is enough.
static mm_status section_event(hipEvent_t& e) {
    if (!e) MM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventReleaseToDevice));
    return MM_OK;
}

mm_status mm_prepare_views(mm_instance inst, void* stream) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "prepare_views: null instance");
    DeviceGuard guard(inst->device);
    MM_TRY(section_event(inst->prep_ev));
    MM_HIP(hipEventRecord(inst->prep_ev, inst->stream));
    MM_HIP(hipStreamWaitEvent(static_cast<hipStream_t>(stream), inst->prep_ev, 0));
    return MM_OK;
}

mm_status mm_update_views(mm_instance inst, void* stream) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "update_views: null instance");
    DeviceGuard guard(inst->device);
    MM_TRY(section_event(inst->upd_ev));
    MM_HIP(hipEventRecord(inst->upd_ev, static_cast<hipStream_t>(stream)));
    MM_HIP(hipStreamWaitEvent(inst->stream, inst->upd_ev, 0));
    return MM_OK;
}

mm_status mm_alloc_linear(mm_instance inst, size_t bytes, void** dev_ptr, mm_alloc* out) {
    if (!inst || !dev_ptr || !out) return fail(MM_ERR_INVALID_ARG, "alloc_linear: null argument");
    if (bytes == 0) return fail(MM_ERR_INVALID_ARG, "alloc_linear: zero bytes");
    DeviceGuard guard(inst->device);
    void* p = nullptr;
    MM_HIP(dev_malloc(&p, bytes));
    mm_alloc a = new (std::nothrow) mm_alloc_s{inst, p, bytes, true, 0};
    if (!a) {
        (void)hipFree(p);
        return fail(MM_ERR_OUT_OF_MEMORY, "alloc_linear: host allocation");
    }
    inst->allocs.insert(a);
    *dev_ptr = p;
    *out = a;
    return MM_OK;
}

mm_status mm_alloc_wrap(mm_instance inst, void* dev_ptr, size_t bytes, mm_alloc* out) {
    if (!inst || !dev_ptr || !out) return fail(MM_ERR_INVALID_ARG, "alloc_wrap: null argument");
    if (bytes == 0) return fail(MM_ERR_INVALID_ARG, "alloc_wrap: zero bytes");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 4 != 0)
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: pointer not 4-byte aligned");
    DeviceGuard guard(inst->device);
    hipPointerAttribute_t attr{};
    const hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != inst->device) {
        (void)hipGetLastError();
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: %p is not device memory of device %d",
                    dev_ptr, inst->device);
    }
    // the whole range must lie inside one device allocation
    hipDeviceptr_t base = nullptr;
    size_t range = 0;
    if (hipMemGetAddressRange(&base, &range, dev_ptr) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: no allocation contains %p", dev_ptr);
    }
    const uintptr_t lo = reinterpret_cast<uintptr_t>(base);
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(dev_ptr);
    if (p0 < lo || bytes > range - (p0 - lo))
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: %zu bytes at %p overrun the %zu-byte allocation",
                    bytes, dev_ptr, range);
    mm_alloc a = new (std::nothrow) mm_alloc_s{inst, dev_ptr, bytes, false, 0};
    if (!a) return fail(MM_ERR_OUT_OF_MEMORY, "alloc_wrap: host allocation");
    inst->allocs.insert(a);
    *out = a;
    return MM_OK;
}

mm_status mm_free(mm_alloc a) {
    if (!a) return fail(MM_ERR_INVALID_ARG, "free: null alloc");
    if (a->users) return fail(MM_ERR_IN_USE, "free: %u view(s) still use this alloc", a->users);
    mm_instance inst = a->inst;
    DeviceGuard guard(inst->device);
    if (a->owned) {
        MM_HIP(hipStreamSynchronize(inst->stream));
        MM_HIP(hipFree(a->ptr));
    }
    inst->allocs.erase(a);
    delete a;
    return MM_OK;
}

mm_status mm_create_view(mm_instance inst, const mm_view_desc* desc, mm_view* out) {
    if (!inst || !desc || !out) return fail(MM_ERR_INVALID_ARG, "create_view: null argument");
    if (!desc->position || inst->allocs.count(desc->position) == 0)
        return fail(MM_ERR_INVALID_ARG, "create_view: position is not an alloc of this instance");
    MM_TRY(validate_desc(inst, desc));
    mm_tuning tuning{};
    MM_TRY(resolve_tuning(*desc, mm_tuning{MM_SPLAT_AUTO, 0, 0, 0, 0, 0, 0}, tuning));
    DeviceGuard guard(inst->device);
    mm_view v = new (std::nothrow) mm_view_s();
    if (!v) return fail(MM_ERR_OUT_OF_MEMORY, "create_view: host allocation");
    v->inst = inst;
    v->position = desc->position;
    v->desc = *desc;
    v->tuning = tuning;
    const uint64_t npix = static_cast<uint64_t>(desc->width) * desc->height;
    hipError_t e = alloc_n(&v->colour, npix);
    if (e == hipSuccess) e = hipMemsetAsync(v->colour, 0, npix * sizeof(uint32_t), inst->stream);
    mm_status st = e == hipSuccess ? setup_splat(v) : hip_fail(e, "create_view: frame buffer");
    if (st != MM_OK) {
        destroy_view_resources(v);
        delete v;
        return st;
    }
    desc->position->users++;
    inst->views.insert(v);
    *out = v;
    return MM_OK;
}

mm_status mm_destroy_view(mm_view v) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "destroy_view: null view");
    mm_instance inst = v->inst;
    if (!inst->views.count(v)) return fail(MM_ERR_INVALID_ARG, "destroy_view: unknown view");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    destroy_view_resources(v);
    v->position->users--;
    if (v->pal_table) v->pal_table->users--;
    if (v->pal_index) v->pal_index->users--;
    inst->views.erase(v);
    delete v;
    return MM_OK;
}

mm_status mm_set_tuning(mm_view v, const mm_tuning* req) {
    if (!v || !req) return fail(MM_ERR_INVALID_ARG, "set_tuning: null argument");
    mm_tuning t{};
    MM_TRY(resolve_tuning(v->desc, *req, t));
    if (v->overlap && t.splat != MM_SPLAT_BINNED)
        return fail(MM_ERR_UNSUPPORTED, "set_tuning: frame overlap needs the binned splat");
    if (v->overlap && req->occlusion_cull == MM_CULL_ON)
        return fail(MM_ERR_UNSUPPORTED, "set_tuning: the occlusion cull is off with frame overlap");
    DeviceGuard guard(v->inst->device);
    MM_TRY(flush_frame(v));
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    const mm_tuning old_tuning = v->tuning;
    const uint32_t old_req = v->req_splat;
    teardown_splat(v);
    v->tuning = t;
    v->req_splat = req->splat;
    const mm_status st = setup_splat(v);
    if (st != MM_OK) restore_splat(v, old_tuning, old_req);
    return st;
}

mm_status mm_autotune(mm_view v, uint32_t frames, mm_tuning* out) {
    if (!v || !out) return fail(MM_ERR_INVALID_ARG, "autotune: null argument");
    if (frames < 1 || frames > 1000) return fail(MM_ERR_INVALID_ARG, "autotune: frames %u outside [1, 1000]", frames);
    mm_instance inst = v->inst;
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    const mm_view_desc& d = v->desc;
    char key[256];
    std::snprintf(key, sizeof key, "view:%s:d%d:n%llu:%ux%u:f%u", device_arch(inst->device).c_str(),
                  (int)d.domain, (unsigned long long)d.element_count, d.width, d.height, d.footprint);
    uint32_t cached[kTuneValues];
    if (tune_cache_lookup(key, cached)) {
        const mm_tuning t{cached[0], cached[1], cached[2], cached[3], cached[4], cached[5], cached[6]};
        if (mm_set_tuning(v, &t) == MM_OK) return mm_get_tuning(v, out);
    }
    const size_t bytes = static_cast<size_t>(d.element_count) * 4u * static_cast<size_t>(d.format);
    void* saved = nullptr;
    MM_HIP(dev_malloc(&saved, bytes));
    hipError_t e = hipMemcpyAsync(saved, v->position->ptr, bytes, hipMemcpyDeviceToDevice, inst->stream);
    std::vector<mm_tuning> cands;
    if (!v->overlap) cands.push_back({MM_SPLAT_DIRECT, 0, 0, 0, 0, 0, 0});
    for (uint32_t tile : {32u, 64u})
        for (uint32_t threads : {256u, 1024u})
            for (uint32_t ppt : {8u, 16u}) {
                for (uint32_t pieces : {0u, 4096u, 16384u})
                    cands.push_back({MM_SPLAT_BINNED, tile, ppt, 0, threads, pieces, 0});
                for (uint32_t splits : {1u, 2u})
                    cands.push_back({MM_SPLAT_BINNED, tile, ppt, splits, threads, MM_PIECES_STATIC, 0});
            }
    mm_tuning best{};
    float best_ms = 0.0f;
    for (const mm_tuning& c : cands) {
        if (e != hipSuccess) break;
        mm_tuning r{};
        if (resolve_tuning(d, c, r) != MM_OK || mm_set_tuning(v, &c) != MM_OK) continue;
        // an overlapped view draws its last frame inside the timed region
        uint32_t calls = 0;
        const float ms = time_frames(inst->stream, frames, [&] {
            mm_status st = mm_step_render(v, 0);
            if (st == MM_OK && ++calls == frames + 1) st = flush_frame(v);
            return st;
        });
        if (ms > 0.0f && (best_ms == 0.0f || ms < best_ms)) {
            best_ms = ms;
            best = r;
        }
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(v->position->ptr, saved, bytes, hipMemcpyDeviceToDevice, inst->stream);
    const hipError_t se = hipStreamSynchronize(inst->stream);
    (void)hipFree(saved);
    if (e != hipSuccess) return hip_fail(e, "autotune: saving or restoring positions");
    if (se != hipSuccess) return hip_fail(se, "autotune: synchronising");
    if (best_ms == 0.0f) return fail(MM_ERR_HIP, "autotune: no candidate ran");
    MM_TRY(mm_set_tuning(v, &best));
    const uint32_t vals[kTuneValues] = {best.splat, best.tile, best.points_per_thread, best.splits,
                                        best.bin_threads, best.piece_records, best.occlusion_cull};
    tune_cache_store(key, vals);
    return mm_get_tuning(v, out);
}

mm_status mm_get_tuning(mm_view v, mm_tuning* out) {
    if (!v || !out) return fail(MM_ERR_INVALID_ARG, "get_tuning: null argument");
    *out = v->tuning;
    if (v->overlap) out->occlusion_cull = MM_CULL_OFF;
    return MM_OK;
}

mm_status mm_set_camera(mm_view v, const float m[16]) {
    if (!v || !m) return fail(MM_ERR_INVALID_ARG, "set_camera: null argument");
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(m[k])) return fail(MM_ERR_INVALID_ARG, "set_camera: m[%d] not finite", k);
    std::memcpy(v->desc.view_proj, m, sizeof(float) * 16);
    set_camera_rows(v->args.g, m);
    set_camera_rows(v->bargs.v.g, m);
    set_camera_rows(v->bargs1.v.g, m);
    return MM_OK;
}

static mm_status require_ready(mm_view v, const char* what) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "%s: null view", what);
    if (!v->plain.exec) return fail(MM_ERR_INVALID_ARG, "%s: view has no usable tuning", what);
    return MM_OK;
}

mm_status mm_step(mm_view v, uint32_t step) {
    MM_TRY(require_ready(v, "step"));
    DeviceGuard guard(v->inst->device);
    mm::PointArgs a = v->args;
    a.c.step = step;
    MM_HIP(mm::launch_point(a, static_cast<int>(v->desc.domain), static_cast<int>(v->desc.footprint),
                            v->desc.wrap != 0, mm::kDisplace, v->inst->stream));
    return MM_OK;
}

mm_status mm_render(mm_view v) {
    MM_TRY(require_ready(v, "render"));
    DeviceGuard guard(v->inst->device);
    hipStream_t s = v->inst->stream;
    const int dim = static_cast<int>(v->desc.domain), foot = static_cast<int>(v->desc.footprint);
    if (!binned(v)) {
        MM_HIP(mm::launch_point(v->args, dim, foot, v->desc.wrap != 0, mm::kRender, s));
        MM_HIP(mm::launch_resolve(v->rargs, s));
        return MM_OK;
    }
    if (v->overlap) {
        MM_TRY(overlap_frame(v, mm::kRender, 0));
        return flush_frame(v);
    }
    MM_TRY(next_stamp(v));
    // no occlusion cull here: its records are built for displaced frames
    const mm::Launch b = mm::bin_launch(dim, v->desc.wrap != 0, mm::kRender,
                                        static_cast<int>(v->tuning.points_per_thread),
                                        v->tuning.bin_threads, v->args.c.n, v->ntiles);
    mm::BinArgs ba = v->bargs;
    ba.v.cull = nullptr;
    ba.mark = nullptr;
    void* bargs[] = {&ba};
    MM_HIP(hipLaunchKernel(b.func, b.grid, b.block, bargs, b.shared, s));
    for (size_t k = v->frame_nodes; k < v->nodes.size(); ++k) {
        void* targs[] = {&v->targs};
        MM_HIP(hipLaunchKernel(v->nodes[k].func, v->nodes[k].grid, v->nodes[k].block, targs,
                               v->nodes[k].shared, s));
    }
    return MM_OK;
}

mm_status mm_step_render(mm_view v, uint32_t step) {
    MM_TRY(require_ready(v, "step_render"));
    DeviceGuard guard(v->inst->device);
    if (v->overlap) return overlap_frame(v, mm::kDisplaceRender, step);
    // per-frame arguments: copies, so that no other launch takes the mark
    mm::BinArgs ba;
    mm::PointArgs pa;
    void* first_arg;
    if (binned(v)) {
        MM_TRY(next_stamp(v));
        ba = v->bargs;
        ba.c.step = step;
        ba.mark = take_mark(v);
        first_arg = &ba;
    } else {
        pa = v->args;
        pa.c.step = step;
        pa.mark = take_mark(v);
        first_arg = &pa;
    }
    void* args[] = {first_arg};
    FrameGraph* fg = &v->plain;
    if (v->profiling && v->prof_count < v->prof_cap && v->prof_skip++ % v->prof_every == 0) {
        const uint32_t k = v->prof_count++;
        for (int j = 0; j < kFrameEvents; ++j)
            MM_HIP(hipGraphExecEventRecordNodeSetEvent(v->timed.exec, v->timed.ev[j],
                                                       v->events[static_cast<size_t>(kFrameEvents) * k + j]));
        fg = &v->timed;
    }
    // the per-frame nodes (hint kernel and point pass) share one argument block
    for (uint32_t j = 0; j < v->frame_nodes; ++j) {
        hipKernelNodeParams pp = node_params(v->nodes[j], args);
        MM_HIP(hipGraphExecKernelNodeSetParams(fg->exec, fg->per_frame[j], &pp));
    }
    MM_HIP(hipGraphLaunch(fg->exec, v->inst->stream));
    return MM_OK;
}

mm_status mm_step_render_frames(mm_view v, uint32_t first_step, uint32_t count, const float* view_proj) {
    MM_TRY(require_ready(v, "step_render_frames"));
    if (count < 1 || count > kMaxGraphFrames)
        return fail(MM_ERR_INVALID_ARG, "step_render_frames: count %u outside [1, %u]", count, kMaxGraphFrames);
    if (view_proj)
        for (uint64_t k = 0; k < 16ull * count; ++k)
            if (!std::isfinite(view_proj[k]))
                return fail(MM_ERR_INVALID_ARG, "step_render_frames: view_proj[%llu] is not finite",
                            (unsigned long long)k);
    DeviceGuard guard(v->inst->device);
    if (v->overlap || count == 1) {  // frame by frame, as the same calls one at a time
        for (uint32_t i = 0; i < count; ++i) {
            if (view_proj) MM_TRY(mm_set_camera(v, view_proj + 16ull * i));
            MM_TRY(mm_step_render(v, first_step + i));
        }
        return MM_OK;
    }
    if (v->multi.frames != count) {
        destroy_multi(v->multi);
        MM_TRY(build_multi(v, count, v->multi));
    }
    // stamps of the whole launch without a wrap in between (a wrap clears
    // the tile flags on the stream, which must come before the launch)
    if (binned(v) && v->stamp > 0xFFFFFFFFu - count) {
        MM_HIP(hipMemsetAsync(v->active, 0, (static_cast<size_t>(v->ntiles) + 1) * 4, v->inst->stream));
        v->stamp = 0;
    }
    MultiGraph& mg = v->multi;
    bool profiled = false;
    for (uint32_t i = 0; i < count; ++i) {
        mm::BinArgs ba;
        mm::PointArgs pa;
        void* first_arg;
        if (binned(v)) {
            MM_TRY(next_stamp(v));
            ba = v->bargs;
            ba.c.step = first_step + i;
            if (view_proj) set_camera_rows(ba.v.g, view_proj + 16ull * i);
            ba.mark = take_mark(v);
            first_arg = &ba;
        } else {
            pa = v->args;
            pa.c.step = first_step + i;
            if (view_proj) set_camera_rows(pa.g, view_proj + 16ull * i);
            pa.mark = take_mark(v);
            first_arg = &pa;
        }
        void* args[] = {first_arg};
        for (uint32_t j = 0; j < v->frame_nodes; ++j) {
            hipKernelNodeParams pp = node_params(v->nodes[j], args);
            MM_HIP(hipGraphExecKernelNodeSetParams(mg.exec, mg.per_frame[static_cast<size_t>(i) * v->frame_nodes + j],
                                                   &pp));
        }
        // the profile samples the first frame of a launch (the one with events)
        if (v->profiling && v->prof_count < v->prof_cap && v->prof_skip++ % v->prof_every == 0 && i == 0) {
            const uint32_t k = v->prof_count++;
            for (int j = 0; j < kFrameEvents; ++j)
                MM_HIP(hipGraphExecEventRecordNodeSetEvent(mg.exec, mg.ev[j],
                                                           v->events[static_cast<size_t>(kFrameEvents) * k + j]));
            profiled = true;
        }
    }
    if (!profiled)
        for (int j = 0; j < kFrameEvents; ++j)
            MM_HIP(hipGraphExecEventRecordNodeSetEvent(mg.exec, mg.ev[j], v->spare[j]));
    MM_HIP(hipGraphLaunch(mg.exec, v->inst->stream));
    if (view_proj) MM_TRY(mm_set_camera(v, view_proj + 16ull * (count - 1)));
    return MM_OK;
}

mm_status mm_set_colour(mm_view v, const mm_colour_desc* d) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "set_colour: null view");
    mm_instance inst = v->inst;
    mm::Palette pal{};
    mm_alloc table = nullptr, index = nullptr;
    if (d && d->palette) {
        table = d->palette;
        if (!inst->allocs.count(table))
            return fail(MM_ERR_INVALID_ARG, "set_colour: palette is not an alloc of this instance");
        if (d->palette_size < 1 || d->palette_size > table->bytes / 4)
            return fail(MM_ERR_INVALID_ARG, "set_colour: %u palette entries do not fit the %zu-byte alloc",
                        d->palette_size, table->bytes);
        const uint64_t n = v->desc.element_count;
        if (d->indices) {
            index = d->indices;
            if (!inst->allocs.count(index))
                return fail(MM_ERR_INVALID_ARG, "set_colour: indices is not an alloc of this instance");
            if (d->index_size != 1 && d->index_size != 2 && d->index_size != 4)
                return fail(MM_ERR_INVALID_ARG, "set_colour: index_size %u is not 1, 2 or 4", d->index_size);
            if (n > index->bytes / d->index_size)
                return fail(MM_ERR_INVALID_ARG, "set_colour: %llu indices of %u B exceed the %zu-byte alloc",
                            (unsigned long long)n, d->index_size, index->bytes);
        } else if (d->palette_size < n) {
            return fail(MM_ERR_INVALID_ARG, "set_colour: per-point palette of %u entries for %llu points",
                        d->palette_size, (unsigned long long)n);
        }
        pal.table = static_cast<const uint32_t*>(table->ptr);
        pal.index = index ? index->ptr : nullptr;
        pal.size = d->palette_size;
        pal.index_size = index ? d->index_size : 0u;
    }
    DeviceGuard guard(inst->device);
    MM_TRY(flush_frame(v));
    MM_HIP(hipStreamSynchronize(inst->stream));
    if (v->pal_table) v->pal_table->users--;
    if (v->pal_index) v->pal_index->users--;
    v->pal_table = table;
    v->pal_index = index;
    if (table) table->users++;
    if (index) index->users++;
    v->pal = pal;
    if (!v->plain.exec) return MM_OK;  // applied by the next successful mm_set_tuning
    teardown_splat(v);
    const mm_status st = setup_splat(v);
    if (st != MM_OK) teardown_splat(v);
    return st;
}

mm_status mm_set_frame_overlap(mm_view v, uint32_t on) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "set_frame_overlap: null view");
    if (on > 1) return fail(MM_ERR_INVALID_ARG, "set_frame_overlap: on must be 0 or 1");
    if ((on != 0) == v->overlap) return MM_OK;
    // a splat left on auto becomes binned, which the overlap needs
    mm_tuning binned_auto{};
    const bool rebin = on && !binned(v) && v->req_splat == MM_SPLAT_AUTO;
    if (rebin) MM_TRY(resolve_tuning(v->desc, mm_tuning{MM_SPLAT_BINNED, 0, 0, 0, 0, 0, 0}, binned_auto));
    if (on && !binned(v) && !rebin)
        return fail(MM_ERR_UNSUPPORTED, "set_frame_overlap: the view's splat was set to direct");
    if (on && !v->plain.exec) return fail(MM_ERR_INVALID_ARG, "set_frame_overlap: view has no usable tuning");
    DeviceGuard guard(v->inst->device);
    MM_TRY(flush_frame(v));
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    const mm_tuning old_tuning = v->tuning;
    const bool was_on = v->overlap;
    teardown_splat(v);
    destroy_overlap(v);
    if (rebin) v->tuning = binned_auto;
    mm_status st = MM_OK;
    if (on) {
        const hipError_t e = open_overlap(v);
        if (e != hipSuccess) st = hip_fail(e, "set_frame_overlap: render stream");
    }
    if (st == MM_OK) st = setup_splat(v);
    if (st != MM_OK) {  // back to the mode and tuning the view had
        teardown_splat(v);
        destroy_overlap(v);
        if (was_on) (void)open_overlap(v);
        restore_splat(v, old_tuning, v->req_splat);
    }
    return st;
}

mm_status mm_flush_frame(mm_view v) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "flush_frame: null view");
    DeviceGuard guard(v->inst->device);
    return flush_frame(v);
}

mm_status mm_frame_device_ptr(mm_view v, const uint32_t** dev_rgba) {
    if (!v || !dev_rgba) return fail(MM_ERR_INVALID_ARG, "frame_device_ptr: null argument");
    *dev_rgba = v->colour;
    return MM_OK;
}

mm_status mm_read_frame(mm_view v, void* host_rgba, size_t bytes) {
    if (!v || !host_rgba) return fail(MM_ERR_INVALID_ARG, "read_frame: null argument");
    const size_t need = static_cast<size_t>(v->desc.width) * v->desc.height * sizeof(uint32_t);
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(v->inst->device);
    if (v->overlap && v->last_drawn >= 0)
        MM_HIP(hipStreamWaitEvent(v->inst->stream, v->ev_drawn[v->last_drawn], 0));
    MM_HIP(hipMemcpyAsync(host_rgba, v->colour, need, hipMemcpyDeviceToHost, v->inst->stream));
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    return MM_OK;
}

mm_status mm_profile_begin(mm_view v, uint32_t capacity) {
    MM_TRY(require_ready(v, "profile_begin"));
    if (capacity == 0 || capacity > (1u << 20))
        return fail(MM_ERR_INVALID_ARG, "profile_begin: capacity outside [1, 2^20]");
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    destroy_graph(v->timed);
    for (hipEvent_t e : v->events) (void)hipEventDestroy(e);
    v->events.assign(static_cast<size_t>(kFrameEvents) * capacity, nullptr);
    // timing only: no system-scope fence (a cache writeback and invalidate
    // per event would slow the frame being measured)
    for (auto& e : v->events) MM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    MM_TRY(build_graph(v, true, v->timed));
    v->prof_cap = capacity;
    v->prof_count = 0;
    v->prof_skip = 0;
    v->profiling = true;
    return MM_OK;
}

mm_status mm_profile_every(mm_view v, uint32_t every) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "profile_every: null view");
    if (every < 1 || every > 1000) return fail(MM_ERR_INVALID_ARG, "profile_every: %u outside [1, 1000]", every);
    v->prof_every = every;
    return MM_OK;
}

mm_status mm_profile_end(mm_view v, float* splat_ms, float* resolve_ms, float* frame_ms,
                         uint32_t* count) {
    if (!v || !count) return fail(MM_ERR_INVALID_ARG, "profile_end: null argument");
    if (!v->profiling) return fail(MM_ERR_INVALID_ARG, "profile_end: no profile_begin");
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    if (v->rstream) MM_HIP(hipStreamSynchronize(v->rstream));
    for (uint32_t k = 0; k < v->prof_count; ++k) {
        float t = 0.0f;
        hipEvent_t* e = &v->events[static_cast<size_t>(kFrameEvents) * k];
        if (splat_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[1], e[2]));
            splat_ms[k] = t;
        }
        if (resolve_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[2], e[3]));
            resolve_ms[k] = t;
        }
        if (frame_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[0], e[3]));
            frame_ms[k] = t;
        }
    }
    *count = v->prof_count;
    v->profiling = false;
    return MM_OK;
}

mm_status mm_mark_begin(mm_view v, uint32_t capacity) {
    MM_TRY(require_ready(v, "mark_begin"));
    if (capacity < 2 || capacity > (1u << 20))
        return fail(MM_ERR_INVALID_ARG, "mark_begin: capacity outside [2, 2^20]");
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    v->marking = false;
    if (v->mark_ring) (void)hipFree(v->mark_ring);
    v->mark_ring = nullptr;
    MM_HIP(dev_malloc(reinterpret_cast<void**>(&v->mark_ring), sizeof(uint64_t) * capacity));
    // a slot no frame wrote reads 0 (refused by mm_mark_read)
    MM_HIP(hipMemsetAsync(v->mark_ring, 0, sizeof(uint64_t) * capacity, v->inst->stream));
    v->mark_cap = capacity;
    v->mark_count = 0;
    v->marking = true;
    return MM_OK;
}

mm_status mm_mark_end(mm_view v) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "mark_end: null view");
    if (!v->marking) return fail(MM_ERR_INVALID_ARG, "mark_end: no mark_begin");
    DeviceGuard guard(v->inst->device);
    if (v->mark_count < v->mark_cap) {  // close the last marked frame
        MM_TRY(flush_frame(v));
        MM_HIP(mm::launch_mark(v->mark_ring + v->mark_count++, v->inst->stream));
    }
    v->marking = false;
    return MM_OK;
}

mm_status mm_mark_read(mm_view v, float* interval_ms, uint32_t* count) {
    if (!v || !count) return fail(MM_ERR_INVALID_ARG, "mark_read: null argument");
    if (v->marking) return fail(MM_ERR_INVALID_ARG, "mark_read: marks not ended (mm_mark_end)");
    const uint32_t marks = v->mark_count;
    if (marks < 2) return fail(MM_ERR_INVALID_ARG, "mark_read: fewer than two marks");
    DeviceGuard guard(v->inst->device);
    int khz = 0;  // the device clock's rate
    MM_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, v->inst->device));
    if (khz <= 0) return fail(MM_ERR_HIP, "mark_read: device clock rate %d kHz", khz);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    std::vector<uint64_t> t(marks);
    MM_HIP(hipMemcpy(t.data(), v->mark_ring, sizeof(uint64_t) * marks, hipMemcpyDeviceToHost));
    for (uint32_t k = 0; k < marks; ++k)
        if (t[k] == 0 || (k > 0 && t[k] < t[k - 1]))
            return fail(MM_ERR_HIP, "mark_read: mark %u was not written in order", k);
    if (interval_ms)
        for (uint32_t k = 0; k + 1 < marks; ++k)
            interval_ms[k] = static_cast<float>(static_cast<double>(t[k + 1] - t[k]) / khz);
    *count = marks - 1;
    return MM_OK;
}

}  // extern "C"
