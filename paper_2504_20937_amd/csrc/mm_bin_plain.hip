// Bin pass of the binned splat for one cloud and one view, arguments in the
// kernel-argument segment (uniform, SGPRs). See mm_bin_dev.h.
#include <type_traits>

#include "mm_bin_dev.h"

namespace mm {
namespace {

using namespace bin;

template <int DIM, bool WRAP, int PHASE, int PPT, uint32_t NT>
__global__ __launch_bounds__(NT) void bin_kernel(BinArgs a) {
    constexpr uint32_t P = NT * PPT;
    const BinLds lds = bin_lds<P>();
    __shared__ uint32_t wave_sum[NT / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t base = blockIdx.x * P;

    for (uint32_t b = tid; b <= a.v.ntiles; b += NT) lds.hist[b] = 0u;
    if (blockIdx.x == 0 && tid == 0) *a.stamp_out = a.stamp;
    float xs[PPT], ys[PPT], zs[PPT];
    load_chunk<DIM, PPT, NT>(a.c, base, xs, ys, zs);
    __syncthreads();
    const CloudArgs c = a.c;  // by value: the key schedule is then shared by all points
    bin_view<DIM, PPT, NT>(a.v, c.n, blockIdx.x, base, a.shift, a.stamp, xs, ys, zs, lds.stage,
                           lds.hist, wave_sum, [c](uint32_t i, float& x, float& y, float& z) {
                               if constexpr ((PHASE & kDisplace) != 0) {
                                   displace<DIM, WRAP>(c, c.step, i, x, y, z);
                                   store_point<DIM>(c.pos, i, x, y, z);
                               }
                           });
}

template <int DIM, bool WRAP, int PHASE>
const void* pick(int ppt, uint32_t nt) {
    return dispatch_bin_shape(ppt, nt, [](auto p, auto t) {
        return reinterpret_cast<const void*>(&bin_kernel<DIM, WRAP, PHASE, decltype(p)::value, decltype(t)::value>);
    });
}

template <int DIM, bool WRAP>
const void* pick_phase(Phase phase, int ppt, uint32_t nt) {
    return phase == kRender ? pick<DIM, WRAP, kRender>(ppt, nt)
                            : pick<DIM, WRAP, kDisplaceRender>(ppt, nt);
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
                  uint32_t ntiles) {
    Launch l;
    if (dim == 2)
        l.func = wrap ? pick_phase<2, true>(phase, ppt, threads) : pick_phase<2, false>(phase, ppt, threads);
    else
        l.func = wrap ? pick_phase<3, true>(phase, ppt, threads) : pick_phase<3, false>(phase, ppt, threads);
    const uint64_t P = static_cast<uint64_t>(threads) * static_cast<uint64_t>(ppt);
    l.block = dim3(threads);
    l.grid = dim3(static_cast<uint32_t>((static_cast<uint64_t>(n) + P - 1) / P));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, threads, ntiles));
    return l;
}

}  // namespace mm
