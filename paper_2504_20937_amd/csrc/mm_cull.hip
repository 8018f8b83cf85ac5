// Hint kernel of the occlusion cull (the cull records are described beside
// BinView in mm_internal.h): this frame's cull records, from the points that
// won the pixels of the previous frame.
//
// One workgroup per screen tile drawn in the previous frame (the source
// tile). Each of its pixels' winners (the hints) is moved by this frame's
// step and projected with this frame's camera, exactly as the bin kernel that
// follows will do, and lowers the depth bound of the pixel it now lands on:
// an LDS minimum per pixel over a window of the tile and kHintMargin pixels
// around it (a hint landing further away is not used). The workgroup then
// merges its bounds into the records of the (up to nine) tiles the window
// overlaps: atomic OR of the covered bitmap words, atomic MAX of each 8x8
// block's largest covered bound. The bound of a block is thus the largest,
// over workgroups, of the largest per-pixel minimum of one workgroup's
// hints; for every covered pixel of the block it is at least the depth of a
// point of this frame drawn there. A block bound of 0 never covers: covered
// depths exceed the near plane's 0.1, so their bits are never 0.
//
// A hint is any point index: whichever point it names, that point is drawn
// in this frame at the pixel it lands on, so the bounds hold for any hint
// set; hints only decide how many records the cull can drop.
#include "mm_device.h"

namespace mm {
namespace {

using namespace dev;

constexpr uint32_t kHintThreads = 256;
constexpr uint32_t kNoBound = 0xFFFFFFFFu;

// One point's position, read with an ordinary (cached) load.
__device__ __forceinline__ void load_point3(const float* pos, uint32_t i, float& x, float& y,
                                            float& z) {
    const float* p = pos + 3ull * i;
    x = p[0];
    y = p[1];
    z = p[2];
}

// Pixels around the source tile where its hints may land and still be used
// (at the orbit camera's 1 degree per frame, winners move a few pixels).
constexpr uint32_t kHintMargin = 8;

template <int SHIFT, bool WRAP>
__global__ __launch_bounds__(kHintThreads) void hint_kernel(BinArgs a) {
    constexpr uint32_t S = 1u << SHIFT, NPIX = S * S;
    constexpr uint32_t H = NPIX / kHintThreads;  // hints per thread: 1, 4 or 16
    constexpr uint32_t HB = H < 8 ? H : 8;      // loaded together
    constexpr uint32_t BMW = cull_bitmap_words(S), NBLK = cull_blocks(S), WORDS = cull_words(S);
    constexpr uint32_t BPR = S / 8;                        // blocks per tile row
    constexpr uint32_t W = S + 2 * kHintMargin, WPIX = W * W;  // the window around the tile
    static_assert(NPIX % kHintThreads == 0, "whole hints per thread");
    static_assert(kHintMargin <= S, "the window lies within the tile's eight neighbours");
    __shared__ uint32_t ub[WPIX];               // per window pixel: the least hint depth
    __shared__ uint32_t bm[9][BMW];             // per destination tile d = (dy + 1) * 3 + dx + 1
    __shared__ uint32_t bmax[9][NBLK];
    const uint32_t t = blockIdx.x;
    if (t == 0 && threadIdx.x == 0 && a.mark) *a.mark = wall_clock64();  // the frame's first kernel
    if (t >= a.v.ntiles) return;
    if (load_flag(&a.v.active[t]) != a.stamp - 1u) return;  // not drawn in the previous frame
    const uint32_t tid = threadIdx.x;
    for (uint32_t q = tid; q < WPIX; q += kHintThreads) ub[q] = kNoBound;
    for (uint32_t q = tid; q < 9 * BMW; q += kHintThreads) (&bm[0][0])[q] = 0u;
    for (uint32_t q = tid; q < 9 * NBLK; q += kHintThreads) (&bmax[0][0])[q] = 0u;
    __syncthreads();

    const uint32_t tiles_x = a.v.tiles_x, tiles_y = a.v.ntiles / tiles_x;
    const int32_t tx = static_cast<int32_t>(t % tiles_x), ty = static_cast<int32_t>(t / tiles_x);
    const int32_t xw = (tx << SHIFT) - static_cast<int32_t>(kHintMargin);
    const int32_t yw = (ty << SHIFT) - static_cast<int32_t>(kHintMargin);
    const CloudArgs c = a.c;
    const uint32_t* h = a.v.hint + static_cast<uint64_t>(t) * NPIX;
#pragma unroll
    for (uint32_t k0 = 0; k0 < H; k0 += HB) {
        uint32_t idx[HB];
#pragma unroll
        for (uint32_t u = 0; u < HB; ++u) idx[u] = h[(k0 + u) * kHintThreads + tid];
        float px[HB], py[HB], pz[HB];
#pragma unroll
        for (uint32_t u = 0; u < HB; ++u) {
            px[u] = py[u] = pz[u] = 0.0f;
            if (idx[u] < c.n) load_point3(c.pos, idx[u], px[u], py[u], pz[u]);
        }
#pragma unroll
        for (uint32_t u = 0; u < HB; ++u) {
            if (idx[u] >= c.n) continue;  // kNoHint
            float x = px[u], y = py[u], z = pz[u];
            displace<3, WRAP>(c, c.step, idx[u], x, y, z);
            int32_t sx, sy;
            uint32_t bits;
            if (!project<3>(a.v.g, x, y, z, sx, sy, bits)) continue;
            const uint32_t wx = static_cast<uint32_t>(sx - xw), wy = static_cast<uint32_t>(sy - yw);
            if (wx >= W || wy >= W) continue;  // beyond the window (also negative)
            atomicMin(&ub[wy * W + wx], bits);
        }
    }
    __syncthreads();

    // window pixel -> destination tile, pixel and block; consecutive lanes
    // take consecutive window pixels (conflict-free reads of ub)
    for (uint32_t p = tid; p < WPIX; p += kHintThreads) {
        const uint32_t u = ub[p];
        if (u == kNoBound) continue;
        const int32_t gx = xw + static_cast<int32_t>(p % W), gy = yw + static_cast<int32_t>(p / W);
        const int32_t dx = (gx >> SHIFT) - tx, dy = (gy >> SHIFT) - ty;  // in -1 .. 1
        const uint32_t d = static_cast<uint32_t>((dy + 1) * 3 + dx + 1);
        const uint32_t lx = static_cast<uint32_t>(gx) & (S - 1u), ly = static_cast<uint32_t>(gy) & (S - 1u);
        const uint32_t q = (ly << SHIFT) | lx;
        atomicOr(&bm[d][q >> 5], 1u << (q & 31u));
        atomicMax(&bmax[d][(ly >> 3) * BPR + (lx >> 3)], u);
    }
    __syncthreads();

    // merge into the destination records (on screen): bitmap words by atomic
    // OR, block bounds by atomic MAX, only where something was covered
    for (uint32_t it = tid; it < 9 * (BMW + NBLK); it += kHintThreads) {
        const uint32_t d = it / (BMW + NBLK), k = it % (BMW + NBLK);
        const uint32_t val = k < BMW ? bm[d][k] : bmax[d][k - BMW];
        if (val == 0u) continue;
        const int32_t nx = tx + static_cast<int32_t>(d % 3) - 1, ny = ty + static_cast<int32_t>(d / 3) - 1;
        if (nx < 0 || ny < 0 || nx >= static_cast<int32_t>(tiles_x) || ny >= static_cast<int32_t>(tiles_y))
            continue;
        uint32_t* rec = a.v.cull + static_cast<uint64_t>(static_cast<uint32_t>(ny) * tiles_x + static_cast<uint32_t>(nx)) * WORDS;
        if (k < BMW) atomicOr(&rec[k], val);
        else atomicMax(&rec[k], val);
    }
}

template <bool WRAP>
const void* pick_hint(int shift) {
    switch (shift) {
        case 4: return reinterpret_cast<const void*>(&hint_kernel<4, WRAP>);
        case 5: return reinterpret_cast<const void*>(&hint_kernel<5, WRAP>);
        default: return reinterpret_cast<const void*>(&hint_kernel<6, WRAP>);
    }
}

}  // namespace

Launch hint_launch(int shift, bool wrap, uint32_t ntiles) {
    Launch l;
    l.func = wrap ? pick_hint<true>(shift) : pick_hint<false>(shift);
    l.block = dim3(kHintThreads);
    l.grid = dim3(ntiles);
    l.shared = 0;
    return l;
}

}  // namespace mm
