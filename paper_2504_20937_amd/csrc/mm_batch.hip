// C ABI of batches: many clouds, each drawn into one or more views, with one
// launch per binned-splat pass for the whole batch.
//
// Device tables (written once per shape):
//   TileView per view, first_view per cloud, bin items (cloud, chunk), tile
//   items (view, tile << 3 | split) in an XCD-aware order, merge items
//   (view, tile << 3).
// Per-frame block (uploaded before each frame from a pinned ring):
//   CloudArgs per cloud (step), BinView per view (camera).
// Frame graph: [batch bin] -> [batch tile] -> [batch merge] (-> [batch seam]);
// only the bin node's argument block (the frame stamp) changes per frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cstring>
#include <new>
#include <vector>

#include "mm_batch.h"

using namespace mmh;

namespace mmb {

namespace {

constexpr uint32_t kPad = 0xFFFFFFFFu;

void free_dev(void*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

void Plan::free_scratch() {
    for (PlanView& v : views) {
        free_dev(reinterpret_cast<void*&>(v.seg));
        free_dev(reinterpret_cast<void*&>(v.table));
        free_dev(reinterpret_cast<void*&>(v.part));
        free_dev(reinterpret_cast<void*&>(v.border));
        free_dev(reinterpret_cast<void*&>(v.apron));
    }
    free_dev(reinterpret_cast<void*&>(active));
    free_dev(dev_static);
    free_dev(dev_frame);
    for (int j = 0; j < kRing; ++j) {
        if (ring[j]) (void)hipHostFree(ring[j]);
        ring[j] = nullptr;
        ring_dev[j] = nullptr;
        if (ring_ev[j]) (void)hipEventDestroy(ring_ev[j]);
        ring_ev[j] = nullptr;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    first = nullptr;
    nodes.clear();
    ready = false;
}

mm_status Plan::resolve(const mm_batch_tuning& req, mm_batch_tuning& out) const {
    out = req;
    uint32_t worst32 = 0;
    for (const PlanView& v : views) worst32 = std::max(worst32, tiles_of(v.width, v.height, 32));
    if (out.tile == 0) out.tile = worst32 <= kMaxTiles ? 32u : 64u;
    if (out.points_per_thread == 0) out.points_per_thread = 16;
    if (out.bin_threads == 0) out.bin_threads = 256;
    const uint32_t shift = shift_of(out.tile);
    if (!mm::binned_shape_ok(static_cast<int>(shift), static_cast<int>(out.points_per_thread),
                             out.bin_threads, out.splits == 0 ? 1u : out.splits))
        return fail(MM_ERR_INVALID_ARG,
                    "batch tuning: tile %u / points_per_thread %u / bin_threads %u / splits %u not in "
                    "{16,32,64} x {4,8,16} x {256,512,1024} x {0,1,2,4,8}",
                    out.tile, out.points_per_thread, out.bin_threads, out.splits);
    if (out.grid_blocks != 0 && (out.grid_blocks % 8 != 0 || out.grid_blocks > (1u << 20)))
        return fail(MM_ERR_INVALID_ARG,
                    "batch tuning: grid_blocks %u is not 0 or a multiple of 8 up to 2^20",
                    out.grid_blocks);
    for (const PlanView& v : views) {
        const uint32_t nt = tiles_of(v.width, v.height, out.tile);
        if (nt > kMaxTiles)
            return fail(MM_ERR_UNSUPPORTED, "batch tuning: a %ux%u view needs %u tiles of %u px (max %u)",
                        v.width, v.height, nt, out.tile, kMaxTiles);
        const size_t lds = mm::bin_lds_bytes(static_cast<int>(out.points_per_thread), out.bin_threads, nt);
        if (lds + 1024 > mm::kMaxLdsBytes)
            return fail(MM_ERR_UNSUPPORTED, "batch tuning: a bin workgroup would need %zu bytes of LDS", lds);
    }
    return MM_OK;
}

// Tile items in an XCD-aware order: runs of up to 64 consecutive tiles of one
// (view, split) share table lines, so each run goes to one XCD (item index
// mod 8); the XCD lists are balanced by length and interleaved, short lists
// padded.
void xcd_tile_items(const std::vector<PlanView>& views, std::vector<uint2>& out) {
    std::vector<std::vector<uint2>> xcd(8);
    for (uint32_t vi = 0; vi < views.size(); ++vi) {
        const PlanView& v = views[vi];
        for (uint32_t z = 0; z < v.splits; ++z)
            for (uint32_t t0 = 0; t0 < v.ntiles; t0 += 64) {
                size_t best = 0;
                for (size_t x = 1; x < 8; ++x)
                    if (xcd[x].size() < xcd[best].size()) best = x;
                for (uint32_t t = t0; t < std::min(v.ntiles, t0 + 64); ++t)
                    xcd[best].push_back(make_uint2(vi, (t << 3) | z));
            }
    }
    size_t len = 0;
    for (auto& l : xcd) len = std::max(len, l.size());
    out.assign(len * 8, make_uint2(kPad, 0));
    for (size_t k = 0; k < len; ++k)
        for (size_t x = 0; x < 8; ++x)
            if (k < xcd[x].size()) out[8 * k + x] = xcd[x][k];
}

void shape_views(std::vector<PlanView>& views, const std::vector<Cloud>& clouds, uint32_t side,
                 uint32_t P, uint32_t splits, uint32_t max_splits) {
    for (PlanView& v : views) {
        const Cloud& c = clouds[v.cloud];
        v.tiles_x = (v.width + side - 1) / side;
        v.tiles_y = (v.height + side - 1) / side;
        v.ntiles = v.tiles_x * v.tiles_y;
        v.num_wg = static_cast<uint32_t>((c.n + P - 1) / P);
        // Auto: by the view's points per tile. A tile-pass item takes a
        // share of one tile's records and the densest tile's item bounds the
        // pass; a clustered cloud puts many times the mean on its densest
        // tiles (in the 64-cloud set, 1.1 M records on one 32-pixel tile of a
        // 256-pixel view of 2^22 points: 8 splits make that item 137 K).
        const uint64_t per_tile = c.n / std::max<uint32_t>(1u, v.ntiles);
        uint32_t s = v.num_wg >= 256 || per_tile >= 4096 ? 2u : 1u;
        if (per_tile >= 8192) s = 4;
        if (per_tile >= 16384) s = 8;
        v.splits = splits != 0 ? splits : std::min(s, max_splits);
    }
}

mm_status build_tables(const std::vector<Cloud>& clouds, const std::vector<PlanView>& views,
                       uint32_t P, uint32_t footprint, TableImage& out) {
    for (size_t i = 1; i < views.size(); ++i)
        if (views[i].cloud < views[i - 1].cloud)
            return fail(MM_ERR_INVALID_ARG, "batch: views are not grouped by cloud");
    std::vector<mm::TileView> tv(views.size());
    out.max_tiles = 0;
    for (size_t i = 0; i < views.size(); ++i) {
        const PlanView& v = views[i];
        const Cloud& c = clouds[v.cloud];
        mm::TileView& x = tv[i];
        x.seg = v.seg;
        x.table = v.table;
        x.active = v.active;
        x.part = v.part;
        x.border = v.border;
        x.apron = v.apron;
        x.colour = v.colour;
        x.width = v.width;
        x.height = v.height;
        x.tiles_x = v.tiles_x;
        x.tiles_y = v.tiles_y;
        x.ntiles = v.ntiles;
        x.num_wg = v.num_wg;
        x.splits = v.splits;
        x.full_clear = v.full_clear ? 1u : 0u;
        x.prev_stamp = v.prev_stamp;
        x.seed_lo = c.args.seed_lo;
        x.seed_hi = c.args.seed_hi;
        out.max_tiles = std::max(out.max_tiles, v.ntiles);
    }
    std::vector<uint32_t> first(clouds.size() + 1, 0);
    for (const PlanView& v : views) first[v.cloud + 1]++;
    for (size_t c = 0; c < clouds.size(); ++c) first[c + 1] += first[c];
    // bin items: clouds with more views first (longer items start early)
    std::vector<uint32_t> order(clouds.size());
    for (uint32_t c = 0; c < order.size(); ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return first[a + 1] - first[a] > first[b + 1] - first[b];
    });
    std::vector<uint2> bin_items, disp_items;
    for (uint32_t c : order) {
        if (!clouds[c].active) continue;
        const uint32_t nwg = static_cast<uint32_t>((clouds[c].n + P - 1) / P);
        std::vector<uint2>& dst = first[c + 1] > first[c] ? bin_items : disp_items;
        for (uint32_t k = 0; k < nwg; ++k) dst.push_back(make_uint2(c, k));
    }
    std::vector<uint2> tile_items, merge_items;
    xcd_tile_items(views, tile_items);
    // with the 1x1 footprint a view of one split is resolved by the tile pass
    for (uint32_t vi = 0; vi < views.size(); ++vi)
        if (footprint != 1 || views[vi].splits != 1)
            for (uint32_t tt = 0; tt < views[vi].ntiles; ++tt) merge_items.push_back(make_uint2(vi, tt << 3));
    out.n_bin = static_cast<uint32_t>(bin_items.size());
    out.n_disp = static_cast<uint32_t>(disp_items.size());
    out.n_tile = static_cast<uint32_t>(tile_items.size());
    out.n_merge = static_cast<uint32_t>(merge_items.size());

    out.o_first = align_up(tv.size() * sizeof(mm::TileView), 256);
    out.o_bin = align_up(out.o_first + first.size() * 4, 256);
    out.o_tile = align_up(out.o_bin + bin_items.size() * 8, 256);
    out.o_merge = align_up(out.o_tile + tile_items.size() * 8, 256);
    out.o_disp = align_up(out.o_merge + merge_items.size() * 8, 256);
    out.stat.assign(align_up(out.o_disp + disp_items.size() * 8, 256), 0);
    unsigned char* h = out.stat.data();
    std::memcpy(h, tv.data(), tv.size() * sizeof(mm::TileView));
    std::memcpy(h + out.o_first, first.data(), first.size() * 4);
    std::memcpy(h + out.o_bin, bin_items.data(), bin_items.size() * 8);
    std::memcpy(h + out.o_tile, tile_items.data(), tile_items.size() * 8);
    std::memcpy(h + out.o_merge, merge_items.data(), merge_items.size() * 8);
    std::memcpy(h + out.o_disp, disp_items.data(), disp_items.size() * 8);

    out.o_views = align_up(clouds.size() * sizeof(mm::CloudArgs), 256);
    out.frame.assign(align_up(out.o_views + views.size() * sizeof(mm::BinView), 256), 0);
    for (size_t c = 0; c < clouds.size(); ++c) out.cloud(c) = clouds[c].args;
    for (size_t i = 0; i < views.size(); ++i) {
        const PlanView& v = views[i];
        mm::BinView& b = out.view(i);
        b.g = view_geom(v.width, v.height, v.view_proj);
        b.seg = v.seg;
        b.table = v.table;
        b.active = v.active;
        b.tiles_x = v.tiles_x;
        b.ntiles = v.ntiles;
    }
    return MM_OK;
}

void bind_args(const TableImage& img, const unsigned char* dstat, const unsigned char* dframe,
               uint32_t* stamp_slot, uint32_t shift, uint32_t P, mm::BatchBinArgs& b,
               mm::BatchTileArgs& t, mm::BatchTileArgs& m) {
    b = mm::BatchBinArgs{};
    b.clouds = reinterpret_cast<const mm::CloudArgs*>(dframe);
    b.views = reinterpret_cast<const mm::BinView*>(dframe + img.o_views);
    b.first_view = reinterpret_cast<const uint32_t*>(dstat + img.o_first);
    b.item = reinterpret_cast<const uint2*>(dstat + img.o_bin);
    b.items = img.n_bin;
    b.disp_item = reinterpret_cast<const uint2*>(dstat + img.o_disp);
    b.disp_items = img.n_disp;
    b.stamp_out = stamp_slot;
    b.stamp = 0;
    b.shift = shift;
    t = mm::BatchTileArgs{};
    t.views = reinterpret_cast<const mm::TileView*>(dstat);
    t.item = reinterpret_cast<const uint2*>(dstat + img.o_tile);
    t.items = img.n_tile;
    t.stamp_in = stamp_slot;
    t.points_per_wg = P;
    m = t;
    m.item = reinterpret_cast<const uint2*>(dstat + img.o_merge);
    m.items = img.n_merge;
}

std::vector<Node> make_nodes(mm_domain domain, uint32_t footprint, uint32_t shift, uint32_t ppt,
                             uint32_t threads, const TableImage& img, uint32_t grid_blocks,
                             mm::BatchBinArgs* b, mm::BatchTileArgs* t, mm::BatchTileArgs* m) {
    const int dim = static_cast<int>(domain), foot = static_cast<int>(footprint);
    const int sh = static_cast<int>(shift), ip = static_cast<int>(ppt);
    std::vector<Node> nodes;
    nodes.push_back({mm::batch_bin_launch(dim, mm::kDisplaceRender, ip, threads, img.n_bin,
                                          img.max_tiles, grid_blocks), b});
    if (img.n_disp)
        nodes.push_back({mm::batch_displace_launch(dim, ip, threads, img.n_disp, grid_blocks), b});
    nodes.push_back({mm::batch_tile_launch(foot, sh, img.n_tile, grid_blocks), t});
    nodes.push_back({mm::batch_merge_launch(foot, sh, img.n_merge, grid_blocks), m});
    if (foot == 3) nodes.push_back({mm::batch_seam_launch(sh, img.n_merge, grid_blocks), m});
    return nodes;
}

mm_status Plan::setup(mm_instance inst, const mm_batch_tuning& t) {
    tuning = t;
    shift = shift_of(t.tile);
    ppt = t.points_per_thread;
    threads = t.bin_threads;
    P = threads * ppt;
    hipStream_t s = inst->stream;
    const uint32_t side = t.tile;
    const uint32_t side_a = footprint == 3 ? side + 2 : side;
    hipError_t e = hipSuccess;

    // per-view shape and scratch
    shape_views(views, clouds, side, P, t.splits, 8u);  // partial blocks sized per view below
    total_tiles = 0;
    for (PlanView& v : views) total_tiles += v.ntiles;
    e = alloc_n(&active, static_cast<uint64_t>(total_tiles) + 1);
    if (e == hipSuccess) e = hipMemsetAsync(active, 0, (static_cast<size_t>(total_tiles) + 1) * 4, s);
    uint32_t off = 0;
    for (PlanView& v : views) {
        v.active = active + off;
        off += v.ntiles;
        if (e == hipSuccess) e = alloc_n(&v.seg, static_cast<uint64_t>(v.num_wg) * P);
        if (e == hipSuccess) e = alloc_n(&v.table, static_cast<uint64_t>(v.num_wg) * (v.ntiles + 1));
        if (e == hipSuccess)
            e = alloc_n(&v.part, static_cast<uint64_t>(v.ntiles) * v.splits * side_a * side_a);
        if (e == hipSuccess && footprint == 3) {
            e = alloc_n(&v.border, static_cast<uint64_t>(v.ntiles) * 4 * side);
            if (e == hipSuccess) e = alloc_n(&v.apron, static_cast<uint64_t>(v.ntiles) * (4 * side + 4));
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batch scratch buffers");
    stamp = 0;

    MM_TRY(build_tables(clouds, views, P, footprint, img));
    MM_HIP(dev_malloc(&dev_static, img.stat.size()));
    MM_HIP(hipMemcpyAsync(dev_static, img.stat.data(), img.stat.size(), hipMemcpyHostToDevice, s));
    MM_HIP(hipStreamSynchronize(s));
    MM_HIP(dev_malloc(&dev_frame, img.frame.size()));
    for (int j = 0; j < kRing; ++j) {
        MM_HIP(pinned_malloc(&ring[j], img.frame.size()));
        MM_HIP(hipHostGetDevicePointer(&ring_dev[j], ring[j], 0));
        // marks the upload kernel's reads of slot j done: no cache flush needed
        MM_HIP(hipEventCreateWithFlags(&ring_ev[j], hipEventDisableTiming | hipEventDisableSystemFence));
    }
    ring_next = 0;
    bind_args(img, static_cast<unsigned char*>(dev_static), static_cast<unsigned char*>(dev_frame),
              active + total_tiles, shift, P, bargs, targs, margs);
    nodes = make_nodes(domain, footprint, shift, ppt, threads, img, t.grid_blocks, &bargs, &targs,
                       &margs);
    render_bin = mm::batch_bin_launch(static_cast<int>(domain), mm::kRender, static_cast<int>(ppt), threads,
                                      img.n_bin, img.max_tiles, t.grid_blocks);
    return MM_OK;
}

mm_status Plan::build_graph() {
    MM_HIP(hipGraphCreate(&graph, 0));
    hipGraphNode_t prev = nullptr;
    hipError_t err = hipSuccess;
    for (size_t k = 0; k < nodes.size() && err == hipSuccess; ++k) {
        if (nodes[k].l.grid.x == 0) continue;  // no items
        void* args[] = {nodes[k].arg};
        hipKernelNodeParams p = node_params(nodes[k].l, args);
        hipGraphNode_t n = nullptr;
        err = hipGraphAddKernelNode(&n, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (k == 0) first = n;  // the bin node: its frame stamp changes per frame
        prev = n;
    }
    if (err == hipSuccess && prev == nullptr)
        err = hipGraphAddEmptyNode(&prev, graph, nullptr, 0);
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (err != hipSuccess) return fail(MM_ERR_HIP, "building the batch graph failed: %s",
                                       hipGetErrorString(err));
    ready = true;
    return MM_OK;
}

mm_status Plan::next_stamp(hipStream_t s) {
    if (++stamp == 0) {
        MM_HIP(hipMemsetAsync(active, 0, (static_cast<size_t>(total_tiles) + 1) * 4, s));
        stamp = 1;
    }
    bargs.stamp = stamp;
    return MM_OK;
}

mm_status Plan::upload_frame(hipStream_t s) {
    const int j = ring_next;
    ring_next = (ring_next + 1) % kRing;
    MM_HIP(hipEventSynchronize(ring_ev[j]));  // the upload that last read slot j is done
    std::memcpy(ring[j], img.frame.data(), img.frame.size());
    MM_HIP(mm::launch_upload(dev_frame, ring_dev[j], img.frame.size(), s));
    MM_HIP(hipEventRecord(ring_ev[j], s));
    return MM_OK;
}

mm_status Plan::launch_graph(hipStream_t s) {
    if (first) {
        void* args[] = {&bargs};
        hipKernelNodeParams p = node_params(nodes[0].l, args);
        MM_HIP(hipGraphExecKernelNodeSetParams(exec, first, &p));
    }
    MM_HIP(hipGraphLaunch(exec, s));
    return MM_OK;
}

mm_status Plan::launch_render(hipStream_t s) {
    MM_HIP(launch(render_bin, &bargs, s));
    for (size_t k = 1; k < nodes.size(); ++k)
        if (nodes[k].arg != &bargs) MM_HIP(launch(nodes[k].l, nodes[k].arg, s));
    return MM_OK;
}

}  // namespace mmb

struct mm_batch_s {
    mm_instance inst;
    mmb::Plan plan;
    std::vector<uint32_t> to_internal;  // user view index -> plan view index
    std::vector<mm_alloc> allocs;
    std::vector<hipEvent_t> events;     // 2 per profiled frame
    uint32_t prof_cap = 0, prof_count = 0;
    bool profiling = false;
};

namespace {

void destroy_batch_resources(mm_batch b) {
    b->plan.free_scratch();
    for (mmb::PlanView& v : b->plan.views)
        if (v.colour && v.owns_colour) (void)hipFree(v.colour);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.clear();
}

mm_status batch_ready(mm_batch b, const char* what) {
    if (!b) return fail(MM_ERR_INVALID_ARG, "%s: null batch", what);
    if (!b->plan.ready) return fail(MM_ERR_INVALID_ARG, "%s: batch has no usable tuning", what);
    return MM_OK;
}

mm_status view_index(mm_batch b, uint32_t view, uint32_t& out, const char* what) {
    if (view >= b->to_internal.size())
        return fail(MM_ERR_INVALID_ARG, "%s: view %u of %zu", what, view, b->to_internal.size());
    out = b->to_internal[view];
    return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_create_batch(mm_instance inst, const mm_batch_desc* desc, mm_batch* out) {
    if (!inst || !desc || !out) return fail(MM_ERR_INVALID_ARG, "create_batch: null argument");
    if (desc->domain != MM_DOMAIN_2D && desc->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "create_batch: domain %d is not 2D/3D", (int)desc->domain);
    if (desc->footprint != 1 && desc->footprint != 3)
        return fail(MM_ERR_INVALID_ARG, "create_batch: footprint %u is not 1 or 3", desc->footprint);
    if (desc->n_clouds == 0 || !desc->clouds || desc->n_views == 0 || !desc->views)
        return fail(MM_ERR_INVALID_ARG, "create_batch: no clouds or no views");
    if (desc->n_clouds > (1u << 20) || desc->n_views > (1u << 20))
        return fail(MM_ERR_INVALID_ARG, "create_batch: more than 2^20 clouds or views");
    std::set<mm_alloc> seen;
    for (uint32_t c = 0; c < desc->n_clouds; ++c) {
        MM_TRY(validate_cloud(inst, desc->clouds[c], desc->domain, "create_batch: cloud"));
        if (!seen.insert(desc->clouds[c].position).second)
            return fail(MM_ERR_INVALID_ARG, "create_batch: clouds %u and an earlier one share an alloc", c);
    }
    for (uint32_t i = 0; i < desc->n_views; ++i) {
        const mm_batch_view_desc& v = desc->views[i];
        if (v.cloud >= desc->n_clouds)
            return fail(MM_ERR_INVALID_ARG, "create_batch: view %u names cloud %u of %u", i, v.cloud,
                        desc->n_clouds);
        MM_TRY(validate_screen(v.width, v.height, "create_batch: view"));
        if (tiles_of(v.width, v.height, 64) > kMaxTiles)
            return fail(MM_ERR_UNSUPPORTED, "create_batch: view %u (%ux%u) exceeds %u tiles of 64 px", i,
                        v.width, v.height, kMaxTiles);
        if (desc->domain == MM_DOMAIN_3D) MM_TRY(validate_camera(v.view_proj, "create_batch: view"));
    }
    DeviceGuard guard(inst->device);
    mm_batch b = new (std::nothrow) mm_batch_s();
    if (!b) return fail(MM_ERR_OUT_OF_MEMORY, "create_batch: host allocation");
    b->inst = inst;
    mmb::Plan& p = b->plan;
    p.domain = desc->domain;
    p.footprint = desc->footprint;
    for (uint32_t c = 0; c < desc->n_clouds; ++c) {
        const mm_cloud_desc& d = desc->clouds[c];
        mmb::Cloud cl;
        cl.args = cloud_args(d.position->ptr, d.element_count, d.seed, d.amplitude);
        cl.args.fold_lim = d.wrap ? 1.0f : std::numeric_limits<float>::infinity();
        cl.n = d.element_count;
        p.clouds.push_back(cl);
        b->allocs.push_back(d.position);
    }
    // plan views grouped by cloud (stable, so views of one cloud keep their order)
    std::vector<uint32_t> order(desc->n_views);
    for (uint32_t i = 0; i < desc->n_views; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) {
        return desc->views[a].cloud < desc->views[c].cloud;
    });
    b->to_internal.assign(desc->n_views, 0);
    hipError_t e = hipSuccess;
    for (uint32_t k = 0; k < desc->n_views; ++k) {
        const mm_batch_view_desc& d = desc->views[order[k]];
        mmb::PlanView v;
        v.cloud = d.cloud;
        v.width = d.width;
        v.height = d.height;
        std::memcpy(v.view_proj, d.view_proj, sizeof v.view_proj);
        const uint64_t npix = static_cast<uint64_t>(d.width) * d.height;
        if (e == hipSuccess) e = alloc_n(&v.colour, npix);
        if (e == hipSuccess) e = hipMemsetAsync(v.colour, 0, npix * 4, inst->stream);
        v.owns_colour = true;
        p.views.push_back(v);
        b->to_internal[order[k]] = k;
    }
    mm_status st = e == hipSuccess ? MM_OK : hip_fail(e, "create_batch: frame buffers");
    mm_batch_tuning t{};
    if (st == MM_OK) st = p.resolve(mm_batch_tuning{0, 0, 0, 0, 0}, t);
    if (st == MM_OK) st = p.setup(inst, t);
    if (st == MM_OK) st = p.build_graph();
    if (st != MM_OK) {
        (void)hipStreamSynchronize(inst->stream);
        destroy_batch_resources(b);
        delete b;
        return st;
    }
    for (mm_alloc a : b->allocs) a->users++;
    inst->batches.insert(b);
    *out = b;
    return MM_OK;
}

mm_status mm_destroy_batch(mm_batch b) {
    if (!b) return fail(MM_ERR_INVALID_ARG, "destroy_batch: null batch");
    mm_instance inst = b->inst;
    if (!inst->batches.count(b)) return fail(MM_ERR_INVALID_ARG, "destroy_batch: unknown batch");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    destroy_batch_resources(b);
    for (mm_alloc a : b->allocs) a->users--;
    inst->batches.erase(b);
    delete b;
    return MM_OK;
}

mm_status mm_batch_set_camera(mm_batch b, uint32_t view, const float m[16]) {
    if (!b || !m) return fail(MM_ERR_INVALID_ARG, "batch_set_camera: null argument");
    uint32_t k = 0;
    MM_TRY(view_index(b, view, k, "batch_set_camera"));
    MM_TRY(validate_camera(m, "batch_set_camera"));
    mmb::PlanView& v = b->plan.views[k];
    std::memcpy(v.view_proj, m, sizeof v.view_proj);
    if (b->plan.ready) set_camera_rows(b->plan.view_slot(k).g, m);
    return MM_OK;
}

mm_status mm_batch_set_cameras(mm_batch b, uint32_t first, uint32_t count, const float* m) {
    if (!b || !m) return fail(MM_ERR_INVALID_ARG, "batch_set_cameras: null argument");
    if (first > b->to_internal.size() || count > b->to_internal.size() - first)
        return fail(MM_ERR_INVALID_ARG, "batch_set_cameras: views %u + %u of %zu", first, count,
                    b->to_internal.size());
    for (uint32_t j = 0; j < count; ++j) MM_TRY(validate_camera(m + 16ull * j, "batch_set_cameras"));
    for (uint32_t j = 0; j < count; ++j) {
        const uint32_t k = b->to_internal[first + j];
        mmb::PlanView& v = b->plan.views[k];
        std::memcpy(v.view_proj, m + 16ull * j, sizeof v.view_proj);
        if (b->plan.ready) set_camera_rows(b->plan.view_slot(k).g, v.view_proj);
    }
    return MM_OK;
}

mm_status mm_batch_step_render(mm_batch b, uint32_t step) {
    MM_TRY(batch_ready(b, "batch_step_render"));
    DeviceGuard guard(b->inst->device);
    hipStream_t s = b->inst->stream;
    mmb::Plan& p = b->plan;
    for (size_t c = 0; c < p.clouds.size(); ++c) p.cloud_slot(c).step = step;
    const bool timed = b->profiling && b->prof_count < b->prof_cap;
    const uint32_t k = timed ? b->prof_count++ : 0;
    if (timed) MM_HIP(hipEventRecord(b->events[2ull * k], s));
    MM_TRY(p.next_stamp(s));
    MM_TRY(p.upload_frame(s));
    MM_TRY(p.launch_graph(s));
    if (timed) MM_HIP(hipEventRecord(b->events[2ull * k + 1], s));
    return MM_OK;
}

mm_status mm_batch_render(mm_batch b) {
    MM_TRY(batch_ready(b, "batch_render"));
    DeviceGuard guard(b->inst->device);
    hipStream_t s = b->inst->stream;
    MM_TRY(b->plan.next_stamp(s));
    MM_TRY(b->plan.upload_frame(s));
    MM_TRY(b->plan.launch_render(s));
    return MM_OK;
}

mm_status mm_batch_frame_device_ptr(mm_batch b, uint32_t view, const uint32_t** dev_rgba) {
    if (!b || !dev_rgba) return fail(MM_ERR_INVALID_ARG, "batch_frame_device_ptr: null argument");
    uint32_t k = 0;
    MM_TRY(view_index(b, view, k, "batch_frame_device_ptr"));
    *dev_rgba = b->plan.views[k].colour;
    return MM_OK;
}

mm_status mm_batch_read_frame(mm_batch b, uint32_t view, void* host_rgba, size_t bytes) {
    if (!b || !host_rgba) return fail(MM_ERR_INVALID_ARG, "batch_read_frame: null argument");
    uint32_t k = 0;
    MM_TRY(view_index(b, view, k, "batch_read_frame"));
    const mmb::PlanView& v = b->plan.views[k];
    const size_t need = static_cast<size_t>(v.width) * v.height * 4;
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "batch_read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(b->inst->device);
    MM_HIP(hipMemcpyAsync(host_rgba, v.colour, need, hipMemcpyDeviceToHost, b->inst->stream));
    MM_HIP(hipStreamSynchronize(b->inst->stream));
    return MM_OK;
}

mm_status mm_batch_set_tuning(mm_batch b, const mm_batch_tuning* req) {
    if (!b || !req) return fail(MM_ERR_INVALID_ARG, "batch_set_tuning: null argument");
    mm_batch_tuning t{};
    MM_TRY(b->plan.resolve(*req, t));
    DeviceGuard guard(b->inst->device);
    MM_HIP(hipStreamSynchronize(b->inst->stream));
    const mm_batch_tuning old = b->plan.tuning;
    const bool had = b->plan.exec != nullptr;
    b->plan.free_scratch();
    b->profiling = false;
    mm_status st = b->plan.setup(b->inst, t);
    if (st == MM_OK) st = b->plan.build_graph();
    if (st != MM_OK) {  // back to the tuning the batch had, keeping this message
        const std::string first = mm_last_error();
        (void)hipStreamSynchronize(b->inst->stream);
        b->plan.free_scratch();
        mm_status back = had ? b->plan.setup(b->inst, old) : st;
        if (back == MM_OK) back = b->plan.build_graph();
        if (back != MM_OK) b->plan.free_scratch();  // unusable until a tuning succeeds
        (void)fail(st, "%s", first.c_str());
    }
    return st;
}

mm_status mm_batch_get_tuning(mm_batch b, mm_batch_tuning* out) {
    if (!b || !out) return fail(MM_ERR_INVALID_ARG, "batch_get_tuning: null argument");
    *out = b->plan.tuning;
    return MM_OK;
}

mm_status mm_batch_autotune(mm_batch b, uint32_t frames, mm_batch_tuning* out) {
    if (!b || !out) return fail(MM_ERR_INVALID_ARG, "batch_autotune: null argument");
    if (frames < 1 || frames > 1000)
        return fail(MM_ERR_INVALID_ARG, "batch_autotune: frames %u outside [1, 1000]", frames);
    mm_instance inst = b->inst;
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    mmb::Plan& p = b->plan;
    // FNV-1a over the workload signature
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
        for (int k = 0; k < 8; ++k) {
            h ^= (x >> (8 * k)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    for (const mmb::Cloud& c : p.clouds) mix(c.n);
    for (const mmb::PlanView& v : p.views) mix((uint64_t(v.cloud) << 32) ^ (uint64_t(v.width) << 16) ^ v.height);
    char key[256];
    std::snprintf(key, sizeof key, "batch:%s:d%d:f%u:c%zu:v%zu:%016llx", device_arch(inst->device).c_str(),
                  (int)p.domain, p.footprint, p.clouds.size(), p.views.size(), (unsigned long long)h);
    uint32_t cached[kTuneValues];
    if (tune_cache_lookup(key, cached)) {
        const mm_batch_tuning t{cached[0], cached[1], cached[2], cached[3], cached[4]};
        if (mm_batch_set_tuning(b, &t) == MM_OK) return mm_batch_get_tuning(b, out);
    }
    // save every cloud
    const size_t stride = 4u * static_cast<size_t>(p.domain);
    std::vector<void*> saved(p.clouds.size(), nullptr);
    hipError_t e = hipSuccess;
    for (size_t c = 0; c < p.clouds.size() && e == hipSuccess; ++c) {
        const size_t bytes = p.clouds[c].n * stride;
        e = dev_malloc(&saved[c], bytes);
        if (e == hipSuccess)
            e = hipMemcpyAsync(saved[c], p.clouds[c].args.pos, bytes, hipMemcpyDeviceToDevice, inst->stream);
    }
    mm_batch_tuning best{};
    float best_ms = 0.0f;
    for (uint32_t tile : {32u, 64u})
        for (uint32_t threads : {256u, 512u, 1024u})
            for (uint32_t ppt : {8u, 16u})
                for (uint32_t splits : {0u, 1u})
                    for (uint32_t grid : {0u, 2048u}) {
                        if (e != hipSuccess) break;
                        const mm_batch_tuning c{tile, ppt, splits, grid, threads};
                        mm_batch_tuning r{};
                        if (p.resolve(c, r) != MM_OK || mm_batch_set_tuning(b, &c) != MM_OK) continue;
                        const float ms =
                            time_frames(inst->stream, frames, [&] { return mm_batch_step_render(b, 0); });
                        if (ms > 0.0f && (best_ms == 0.0f || ms < best_ms)) {
                            best_ms = ms;
                            best = r;
                        }
                    }
    for (size_t c = 0; c < p.clouds.size() && e == hipSuccess; ++c)
        e = hipMemcpyAsync(p.clouds[c].args.pos, saved[c], p.clouds[c].n * stride, hipMemcpyDeviceToDevice,
                           inst->stream);
    const hipError_t se = hipStreamSynchronize(inst->stream);
    for (void* q : saved)
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return hip_fail(e, "batch_autotune: saving or restoring positions");
    if (se != hipSuccess) return hip_fail(se, "batch_autotune: synchronising");
    if (best_ms == 0.0f) return fail(MM_ERR_HIP, "batch_autotune: no candidate ran");
    MM_TRY(mm_batch_set_tuning(b, &best));
    const uint32_t vals[kTuneValues] = {best.tile, best.points_per_thread, best.splits,
                                        best.grid_blocks, best.bin_threads, 0u, 0u};
    tune_cache_store(key, vals);
    return mm_batch_get_tuning(b, out);
}

mm_status mm_batch_profile_begin(mm_batch b, uint32_t capacity) {
    MM_TRY(batch_ready(b, "batch_profile_begin"));
    if (capacity == 0 || capacity > (1u << 20))
        return fail(MM_ERR_INVALID_ARG, "batch_profile_begin: capacity outside [1, 2^20]");
    DeviceGuard guard(b->inst->device);
    MM_HIP(hipStreamSynchronize(b->inst->stream));
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.assign(2ull * capacity, nullptr);
    // timing only: no system-scope fence per event
    for (auto& e : b->events) MM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    b->prof_cap = capacity;
    b->prof_count = 0;
    b->profiling = true;
    return MM_OK;
}

mm_status mm_batch_profile_end(mm_batch b, float* frame_ms, uint32_t* count) {
    if (!b || !count) return fail(MM_ERR_INVALID_ARG, "batch_profile_end: null argument");
    if (!b->profiling) return fail(MM_ERR_INVALID_ARG, "batch_profile_end: no profile_begin");
    DeviceGuard guard(b->inst->device);
    MM_HIP(hipStreamSynchronize(b->inst->stream));
    for (uint32_t k = 0; k < b->prof_count; ++k) {
        float t = 0.0f;
        MM_HIP(hipEventElapsedTime(&t, b->events[2ull * k], b->events[2ull * k + 1]));
        if (frame_ms) frame_ms[k] = t;
    }
    *count = b->prof_count;
    b->profiling = false;
    return MM_OK;
}

}  // extern "C"
