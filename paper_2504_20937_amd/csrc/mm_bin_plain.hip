// Bin pass of the binned splat for one cloud and one view, arguments in the
// kernel-argument segment (uniform, SGPRs). See mm_bin_dev.h.
#include <type_traits>

#include "mm_bin_dev.h"

namespace mm {
namespace {

using namespace bin;

// Two workgroups per CU where the registers allow it: one workgroup's loads
// stream while the other sorts in LDS. With the cull, a thread also holds its
// displaced points until the cull-record loads are out (about 84 registers
// at 8 points per thread), so only 4 points per thread keep 8 waves per SIMD.
template <int PPT, bool CULL>
constexpr int kBinWavesPerEU = PPT <= (CULL ? 4 : 8) ? 8 : 4;

template <int DIM, bool WRAP, int PHASE, int PPT, uint32_t NT, bool CULL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kBinWavesPerEU<PPT, CULL>)))
void bin_kernel(BinArgs a) {
    constexpr uint32_t P = NT * PPT;
    const BinLds lds = bin_lds<P>();
    __shared__ uint32_t wave_sum[NT / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t base = blockIdx.x * P;

    for (uint32_t b = tid; b <= a.v.ntiles; b += NT) lds.hist[b] = 0u;
    if (blockIdx.x == 0 && tid == 0) {
        *a.stamp_out = a.stamp;
        if (a.mark && !CULL) *a.mark = wall_clock64();  // with the cull the hint kernel ran first
    }
    float xs[PPT], ys[PPT], zs[PPT];
    load_chunk<DIM, PPT, NT>(a.c, base, xs, ys, zs);
    __syncthreads();
    const CloudArgs c = a.c;  // by value: the key schedule is then shared by all points
    // With the cull, the positions are stored once the cull-record loads are
    // issued: the vector memory counter covers loads and stores in issue
    // order, so a wait for those loads does not then wait for these stores.
    auto pre = [c](uint32_t i, float& x, float& y, float& z) {
        if constexpr ((PHASE & kDisplace) != 0) {
            displace<DIM, WRAP>(c, c.step, i, x, y, z);
            if constexpr (!CULL) store_point<DIM>(c.pos, i, x, y, z);
        }
    };
    auto store_all = [&]() {
        if constexpr (CULL && (PHASE & kDisplace) != 0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const uint32_t i = base + k * NT + tid;
                if (i < c.n) store_point<DIM>(c.pos, i, xs[k], ys[k], zs[k]);
            }
        }
    };
    bin_view<DIM, PPT, NT, decltype(pre), CULL>(a.v, c.n, blockIdx.x, base, a.shift, a.stamp, xs,
                                                ys, zs, lds.stage, lds.hist, wave_sum, pre, store_all);
}

template <int DIM, bool WRAP, int PHASE, bool CULL>
const void* pick(int ppt, uint32_t nt) {
    return dispatch_bin_shape(ppt, nt, [](auto p, auto t) {
        constexpr int PPT = decltype(p)::value;
        constexpr uint32_t NT = decltype(t)::value;
        // no culled kernel where its registers would spill (cull_shape_ok)
        constexpr bool C = CULL && cull_shape_ok(PPT, NT);
        return reinterpret_cast<const void*>(&bin_kernel<DIM, WRAP, PHASE, PPT, NT, C>);
    });
}

// The occlusion cull reads 3D depths: 2D views (depth 0) never use it.
template <int DIM, bool WRAP>
const void* pick_phase(Phase phase, int ppt, uint32_t nt, bool cull) {
    if constexpr (DIM == 3) {
        if (cull)
            return phase == kRender ? pick<DIM, WRAP, kRender, true>(ppt, nt)
                                    : pick<DIM, WRAP, kDisplaceRender, true>(ppt, nt);
    }
    return phase == kRender ? pick<DIM, WRAP, kRender, false>(ppt, nt)
                            : pick<DIM, WRAP, kDisplaceRender, false>(ppt, nt);
}

}  // namespace

bool binned_shape_ok(int shift, int ppt, uint32_t threads, uint32_t splits) {
    return (shift == 4 || shift == 5 || shift == 6) && (ppt == 4 || ppt == 8 || ppt == 16) &&
           (threads == 256 || threads == 512 || threads == 1024) &&
           (splits == 1 || splits == 2 || splits == 4 || splits == 8);
}

size_t bin_lds_bytes(int ppt, uint32_t threads, uint32_t ntiles) {
    return sizeof(uint64_t) * threads * static_cast<uint32_t>(ppt) + sizeof(uint32_t) * (ntiles + 1u);
}

Launch bin_launch(int dim, bool wrap, Phase phase, int ppt, uint32_t threads, uint32_t n,
                  uint32_t ntiles, bool cull) {
    Launch l;
    if (dim == 2)
        l.func = wrap ? pick_phase<2, true>(phase, ppt, threads, false)
                      : pick_phase<2, false>(phase, ppt, threads, false);
    else
        l.func = wrap ? pick_phase<3, true>(phase, ppt, threads, cull)
                      : pick_phase<3, false>(phase, ppt, threads, cull);
    const uint64_t P = static_cast<uint64_t>(threads) * static_cast<uint64_t>(ppt);
    l.block = dim3(threads);
    l.grid = dim3(static_cast<uint32_t>((static_cast<uint64_t>(n) + P - 1) / P));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, threads, ntiles));
    return l;
}

}  // namespace mm
