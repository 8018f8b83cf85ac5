// Bin pass of the batched binned splat: many clouds, each with one or more
// views, in one launch. Bin items (cloud, chunk) are read from a device
// table; each chunk is displaced once and binned into every view of its
// cloud. See mm_bin_dev.h.
#include <type_traits>

#include "mm_bin_dev.h"

namespace mm {
namespace {

using namespace bin;

// PERSIST: each block loops over items blockIdx.x, blockIdx.x + gridDim.x, ...;
// else one item per block.
template <int DIM, int PHASE, int PPT, uint32_t NT, bool PERSIST>
__global__ __launch_bounds__(NT) void batch_bin_kernel(BatchBinArgs a) {
    constexpr uint32_t P = NT * PPT;
    const BinLds lds = bin_lds<P>();
    __shared__ uint32_t wave_sum[NT / 64];
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) *a.stamp_out = a.stamp;
    auto run_item = [&](uint32_t it) {
        const uint2 item = load_uniform(&a.item[it]);
        const CloudArgs c = load_uniform(&a.clouds[item.x]);
        const uint32_t base = item.y * P;
        const uint32_t v0 = load_uniform(&a.first_view[item.x]);
        const uint32_t v1 = load_uniform(&a.first_view[item.x + 1]);
        for (uint32_t b = tid; b <= load_uniform(&a.views[v0].ntiles); b += NT) lds.hist[b] = 0u;
        float xs[PPT], ys[PPT], zs[PPT];
        load_chunk<DIM, PPT, NT>(c, base, xs, ys, zs);
        __syncthreads();
        // the first view displaces (each cloud has its own step and fold limit)
        bin_view<DIM, PPT, NT>(load_uniform(&a.views[v0]), c.n, item.y, base, a.shift, a.stamp, xs,
                               ys, zs, lds.stage, lds.hist, wave_sum,
                               [&](uint32_t i, float& x, float& y, float& z) {
                                   if constexpr ((PHASE & kDisplace) != 0) displace_cloud<DIM>(c, i, x, y, z);
                               });
        __syncthreads();  // stage and hist free for the next view or item
        // Further views take the displaced chunk from the registers the first
        // view left it in (up to 512 threads: 126 VGPRs, occupancy unchanged;
        // 1.07 against 1.18 ms per batch frame of 64 clouds and 156 views at
        // 256 threads). 1024-thread workgroups have 128 VGPRs a lane and would
        // spill: they read the chunk again, mostly from L2, the empty asm
        // hiding that base2 equals base so the addresses are formed anew.
        uint32_t base2 = base;
        asm volatile("" : "+v"(base2));
        for (uint32_t vi = v0 + 1; vi < v1; ++vi) {
            const BinView v = load_uniform(&a.views[vi]);
            for (uint32_t b = tid; b <= v.ntiles; b += NT) lds.hist[b] = 0u;
            if constexpr (NT > 512) load_chunk<DIM, PPT, NT>(c, base2, xs, ys, zs);
            __syncthreads();
            bin_view<DIM, PPT, NT>(v, c.n, item.y, base2, a.shift, a.stamp, xs, ys, zs, lds.stage,
                                   lds.hist, wave_sum, [](uint32_t, float&, float&, float&) {});
            __syncthreads();
        }
    };
    if constexpr (PERSIST) {
        for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) run_item(it);
    } else {
        if (blockIdx.x < a.items) run_item(blockIdx.x);
    }
}

// Items (cloud, chunk of P points) of clouds without views: displacement only.
template <int DIM, uint32_t P>
__global__ __launch_bounds__(256) void batch_displace_kernel(BatchBinArgs a) {
    for (uint32_t it = blockIdx.x; it < a.disp_items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.disp_item[it]);
        const CloudArgs c = load_uniform(&a.clouds[item.x]);
#pragma unroll 4
        for (uint32_t k = 0; k < P / 256u; ++k) {
            const uint32_t i = item.y * P + k * 256u + threadIdx.x;
            if (i >= c.n) continue;
            float x, y, z;
            load_point<DIM>(c.pos, i, x, y, z);
            displace_cloud<DIM>(c, i, x, y, z);
        }
    }
}

template <int DIM, int PHASE, bool PERSIST>
const void* pick(int ppt, uint32_t nt) {
    return dispatch_bin_shape(ppt, nt, [](auto p, auto t) {
        return reinterpret_cast<const void*>(
            &batch_bin_kernel<DIM, PHASE, decltype(p)::value, decltype(t)::value, PERSIST>);
    });
}

template <int DIM, bool PERSIST>
const void* pick_phase(Phase phase, int ppt, uint32_t nt) {
    return phase == kRender ? pick<DIM, kRender, PERSIST>(ppt, nt)
                            : pick<DIM, kDisplaceRender, PERSIST>(ppt, nt);
}

template <int DIM>
const void* pick_displace(int ppt, uint32_t nt) {
    return dispatch_bin_shape(ppt, nt, [](auto p, auto t) {
        return reinterpret_cast<const void*>(
            &batch_displace_kernel<DIM, decltype(p)::value * decltype(t)::value>);
    });
}

uint32_t batch_grid(uint32_t items, uint32_t grid_blocks) {
    if (grid_blocks == 0 || grid_blocks > items) return items;
    return grid_blocks;
}

}  // namespace

Launch batch_bin_launch(int dim, Phase phase, int ppt, uint32_t threads, uint32_t items,
                        uint32_t max_tiles, uint32_t grid_blocks) {
    Launch l;
    const bool persist = grid_blocks != 0 && grid_blocks < items;
    if (dim == 2)
        l.func = persist ? pick_phase<2, true>(phase, ppt, threads) : pick_phase<2, false>(phase, ppt, threads);
    else
        l.func = persist ? pick_phase<3, true>(phase, ppt, threads) : pick_phase<3, false>(phase, ppt, threads);
    l.block = dim3(threads);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, threads, max_tiles));
    return l;
}

Launch batch_displace_launch(int dim, int ppt, uint32_t threads, uint32_t items,
                             uint32_t grid_blocks) {
    Launch l;
    l.func = dim == 2 ? pick_displace<2>(ppt, threads) : pick_displace<3>(ppt, threads);
    l.block = dim3(256);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = 0;
    return l;
}

}  // namespace mm
