// Bin pass of the binned splat: per workgroup of NT threads, a chunk of
// P = NT * PPT consecutive points is loaded (and displaced), projected,
// counted per screen tile in LDS, scanned, placed in LDS sorted by tile, and
// written out as the chunk's segment of 8-byte records plus one table row of
// u16 tile start offsets.
//
//   record = depth_bits << 32 | local_index << 16 | 8 (y_in_tile * side + x_in_tile)
//
// (the low half-word is the byte offset of the pixel's key in the tile pass's
// LDS key block, below 2^15 for tiles up to 64 pixels, so the depth test
// finds its address with one AND)
//
// Larger chunks give the tile pass longer runs per (chunk, tile) and a
// smaller table, at the cost of LDS per workgroup (8 P + 4 (tiles + 1) bytes).
#pragma once

#include <type_traits>

#include "mm_device.h"

namespace mm {
namespace bin {

using namespace dev;

constexpr uint32_t kNoPixel = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of h[0..count) in place by the NW waves of the block;
// h[count] = total. Each wave owns a contiguous run of 64-bin blocks and
// reads every block with consecutive lanes on consecutive words, so LDS
// accesses never conflict.
template <uint32_t NW>
__device__ __forceinline__ void block_exclusive_scan(uint32_t* h, uint32_t count,
                                                     uint32_t* wave_sum) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nblk = (count + 63u) / 64u;
    const uint32_t per = (nblk + NW - 1) / NW;
    const uint32_t b0 = min(nblk, wave * per), b1 = min(nblk, b0 + per);
    uint32_t lsum = 0;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t i = b * 64u + lane;
        lsum += i < count ? h[i] : 0u;
    }
    const uint32_t wtot = __shfl(wave_inclusive_scan(lsum, lane), 63, 64);
    if (lane == 0) wave_sum[wave] = wtot;
    __syncthreads();
    uint32_t carry = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < NW; ++w) {
        carry += w < wave ? wave_sum[w] : 0u;
        total += wave_sum[w];
    }
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t i = b * 64u + lane;
        const uint32_t v = i < count ? h[i] : 0u;
        const uint32_t inc = wave_inclusive_scan(v, lane);
        if (i < count) h[i] = carry + inc - v;
        carry += __shfl(inc, 63, 64);
    }
    if (tid == 0) h[count] = total;
}

// The PPT points per thread of chunk [base, base + P). Lanes past the end of
// the cloud load its last point instead (their values are never used): no
// branch around the loads, so all PPT loads are in flight together.
template <int DIM, int PPT, uint32_t NT>
__device__ __forceinline__ void load_chunk(const CloudArgs& c, uint32_t base, float (&xs)[PPT],
                                           float (&ys)[PPT], float (&zs)[PPT]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = min(base + k * NT + tid, c.n - 1u);
        load_point<DIM>(c.pos, i, xs[k], ys[k], zs[k]);
    }
}

// One step of point i of cloud c with the cloud's own fold limit, stored back.
template <int DIM>
__device__ __forceinline__ void displace_cloud(const CloudArgs& c, uint32_t i, float& x, float& y,
                                               float& z) {
    displace<DIM, false>(c, c.step, i, x, y, z);
    x = fold_to(x, c.fold_lim);
    y = fold_to(y, c.fold_lim);
    if constexpr (DIM == 3) z = fold_to(z, c.fold_lim);
    store_point<DIM>(c.pos, i, x, y, z);
}

// The tile holding stage record j: the number of tiles whose run ends at or
// before j (hist[b] = end of tile b's run, non-decreasing), found with a
// fixed 12-step branch-free search, so a thread's searches for its PPT
// records interleave.
__device__ __forceinline__ uint32_t tile_of_record(const uint32_t* hist, uint32_t nt, uint32_t j) {
    static_assert(kMaxPlanTiles == 4096, "12 steps cover 4096 tiles");
    uint32_t b = 0;
#pragma unroll
    for (uint32_t step = 2048; step != 0; step >>= 1) {
        const uint32_t c = b + step;
        if (c <= nt && hist[c - 1] <= j) b = c;
    }
    return b;
}

// Survivors before stage position j, from the windows' keep masks and
// exclusive bases (window w = records 64 w .. 64 w + 63).
__device__ __forceinline__ uint32_t kept_before(const uint64_t* mask, const uint32_t* base,
                                                uint32_t j) {
    const uint32_t w = j >> 6, bit = j & 63u;
    const uint64_t below = bit ? (mask[w] & (~0ull >> (64u - bit))) : 0ull;
    return base[w] + static_cast<uint32_t>(__popcll(below));
}

// The culled write of a chunk sorted by tile in the stage (hist[b] = end of
// tile b's run, hist[nt] = total): every thread takes its records j = tid,
// tid + NT, ... (consecutive lanes, consecutive records), finds each one's
// tile, reads the tile's cull record (bitmap word of the pixel and bound of
// its 8x8 block, all loads in flight together; neighbouring lanes mostly
// share a tile, so a wave touches few cache lines), and keeps the record
// unless its pixel is covered and its depth exceeds the bound. Survivors keep
// their stage order: a record's output position is the number of survivors
// before it (per-window ballots and a scan of the window counts), so each
// tile's survivors form one run and the table row holds the surviving starts.
// Tiles are stamped from the counts before the cull: a tile's winner is never
// ruled out, so a tile with points keeps a survivor in some chunk.
// post() runs once the cull-record loads are issued (the kernel's deferred
// position stores).
// LDS beside the stage and histogram: mask (P / 64 u64) and base (P / 64 + 1 u32).
template <int PPT, uint32_t NT, typename Post>
__device__ __forceinline__ void cull_write(const BinView& v, uint32_t chunk, uint32_t shift,
                                           uint32_t stamp, const uint64_t* stage,
                                           const uint32_t* hist, uint64_t* mask, uint32_t* base,
                                           Post post) {
    constexpr uint32_t P = NT * PPT, NW = NT / 64, NWIN = P / 64;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nt = v.ntiles, total = hist[nt];
    const uint32_t side = 1u << shift, words = cull_words(side), bmw = cull_bitmap_words(side);
    const uint32_t blk_shift = shift - 3u;
    // every record's two cull-record words are loaded first (all in flight
    // together; a record is read again from LDS where it is needed, so only
    // the loaded words stay in registers), then post() issues the deferred
    // stores, then the words are used
    uint32_t word[PPT], bound[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t j = static_cast<uint32_t>(k) * NT + tid;
        const uint64_t r = j < total ? stage[j] : 0ull;
        // past the chunk's records: any tile (the record is not kept)
        const uint32_t tb = min(tile_of_record(hist, nt, j), nt - 1u);
        const uint32_t q = (static_cast<uint32_t>(r) & 0xFFFFu) >> 3;
        const uint32_t blk = (((q >> shift) >> 3) << blk_shift) | ((q & (side - 1u)) >> 3);
        const uint32_t* rec = v.cull + static_cast<uint64_t>(tb) * words;
        word[k] = rec[q >> 5];
        bound[k] = rec[bmw + blk];
    }
    post();
    uint32_t keep = 0;  // bit k: record k of this thread survives
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t j = static_cast<uint32_t>(k) * NT + tid;
        const uint64_t r = j < total ? stage[j] : 0ull;
        const uint32_t q = (static_cast<uint32_t>(r) & 0xFFFFu) >> 3;
        const bool covered = ((word[k] >> (q & 31u)) & 1u) != 0u;
        const bool kp = j < total && !(covered && static_cast<uint32_t>(r >> 32) > bound[k]);
        keep |= (kp ? 1u : 0u) << k;
        const uint64_t m = __ballot(kp);
        if (lane == 0) mask[static_cast<uint32_t>(k) * NW + wave] = m;
    }
    __syncthreads();
    if (wave == 0) {  // exclusive scan of the windows' counts
        uint32_t carry = 0;
        for (uint32_t w0 = 0; w0 < NWIN; w0 += 64u) {
            const uint32_t w = w0 + lane;
            const uint32_t c = w < NWIN ? static_cast<uint32_t>(__popcll(mask[w])) : 0u;
            const uint32_t inc = wave_inclusive_scan(c, lane);
            if (w < NWIN) base[w] = carry + inc - c;
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) base[NWIN] = carry;
    }
    __syncthreads();
    uint64_t* seg = v.seg + static_cast<uint64_t>(chunk) * P;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t j = static_cast<uint32_t>(k) * NT + tid;
        if ((keep >> k) & 1u) seg[kept_before(mask, base, j)] = stage[j];
    }
    uint16_t* row = v.table + static_cast<uint64_t>(chunk) * (nt + 1u);
    for (uint32_t b = tid; b <= nt; b += NT) {
        const uint32_t s = b == 0 ? 0u : hist[b - 1];
        row[b] = static_cast<uint16_t>(s >= P ? base[NWIN] : kept_before(mask, base, s));
    }
    for (uint32_t b = tid; b < nt; b += NT) {
        const uint32_t s = b == 0 ? 0u : hist[b - 1];
        if (hist[b] > s) store_flag(&v.active[b], stamp);
    }
}

// Bin one chunk of points into the tiles of one view: segment `chunk` of
// v.seg, row `chunk` of v.table, and the stamps of the tiles that received
// points. pre(i, x, y, z) runs on each point before its projection, in the
// same loop (the displacement: its stores then drain under the projection
// and histogram work). On entry hist[0..ntiles] is zero and visible to the
// whole block. With CULL the records the view's cull records rule out are
// not written (see cull_write); the table then holds the surviving runs.
struct NoOp {
    __device__ void operator()() const {}
};

template <int DIM, int PPT, uint32_t NT, typename Pre, bool CULL = false, typename Post = NoOp>
__device__ __forceinline__ void bin_view(const BinView& v, uint32_t n, uint32_t chunk,
                                         uint32_t base, uint32_t shift, uint32_t stamp,
                                         float (&xs)[PPT], float (&ys)[PPT], float (&zs)[PPT],
                                         uint64_t* stage, uint32_t* hist, uint32_t* wave_sum,
                                         Pre pre, Post post = Post{}) {
    constexpr uint32_t P = NT * PPT;
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = v.ntiles;
    const uint32_t mask = (1u << shift) - 1u;

    uint32_t pix[PPT], dep[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = base + k * NT + tid;
        pix[k] = kNoPixel;
        dep[k] = 0u;
        if (i < n) {
            pre(i, xs[k], ys[k], zs[k]);
            int32_t px, py;
            uint32_t bits;
            if (project<DIM>(v.g, xs[k], ys[k], zs[k], px, py, bits)) {
                const uint32_t ux = static_cast<uint32_t>(px), uy = static_cast<uint32_t>(py);
                pix[k] = (uy << 16) | ux;
                dep[k] = bits;
                atomicAdd(&hist[(uy >> shift) * v.tiles_x + (ux >> shift)], 1u);
            }
        }
    }
    __syncthreads();
    block_exclusive_scan<NT / 64>(hist, nt, wave_sum);
    __syncthreads();

#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (pix[k] == kNoPixel) continue;
        const uint32_t ux = pix[k] & 0xFFFFu, uy = pix[k] >> 16;
        const uint32_t slot = atomicAdd(&hist[(uy >> shift) * v.tiles_x + (ux >> shift)], 1u);
        const uint32_t local = static_cast<uint32_t>(k) * NT + tid;
        stage[slot] = (static_cast<uint64_t>(dep[k]) << 32) |
                      static_cast<uint64_t>((local << 16) | ((((uy & mask) << shift) | (ux & mask)) << 3));
    }
    __syncthreads();

    if constexpr (CULL) {
        if (v.cull) {
            __shared__ uint64_t cull_mask[P / 64];
            __shared__ uint32_t cull_base[P / 64 + 1];
            cull_write<PPT, NT>(v, chunk, shift, stamp, stage, hist, cull_mask, cull_base, post);
            return;
        }
        post();
    }
    // hist[b] is now the end of bin b (= start of bin b + 1); hist[nt] the total
    const uint32_t total = hist[nt];
    uint64_t* seg = v.seg + static_cast<uint64_t>(chunk) * P;
    for (uint32_t j = tid; j < total; j += NT) seg[j] = stage[j];
    uint16_t* row = v.table + static_cast<uint64_t>(chunk) * (nt + 1u);
    for (uint32_t b = tid; b <= nt; b += NT)
        row[b] = static_cast<uint16_t>(b == 0 ? 0u : hist[b - 1]);
    // Stamp the tiles that received points. All workgroups write the same
    // value, so the stores are plain cached ones (relaxed atomics at
    // wavefront scope carry no cache-bypass bits); the kernel boundary makes
    // them visible to the tile pass.
    for (uint32_t b = tid; b < nt; b += NT) {
        const uint32_t s = b == 0 ? 0u : hist[b - 1];
        if (hist[b] > s) store_flag(&v.active[b], stamp);
    }
}

// LDS of a bin workgroup: the stage first, then the histogram.
struct BinLds {
    uint64_t* stage;
    uint32_t* hist;
};

template <uint32_t P>
__device__ __forceinline__ BinLds bin_lds() {
    extern __shared__ __align__(16) unsigned char smem[];
    return BinLds{reinterpret_cast<uint64_t*>(smem),
                  reinterpret_cast<uint32_t*>(smem + sizeof(uint64_t) * P)};
}

// Calls fn(integral_constant<int, PPT>, integral_constant<uint32_t, NT>) for
// the bin shape (ppt, nt): PPT in {4, 8, 16}, NT in {256, 512, 1024}.
template <uint32_t NT, typename Fn>
const void* dispatch_bin_ppt(int ppt, Fn fn) {
    switch (ppt) {
        case 4: return fn(std::integral_constant<int, 4>{}, std::integral_constant<uint32_t, NT>{});
        case 8: return fn(std::integral_constant<int, 8>{}, std::integral_constant<uint32_t, NT>{});
        default: return fn(std::integral_constant<int, 16>{}, std::integral_constant<uint32_t, NT>{});
    }
}

template <typename Fn>
const void* dispatch_bin_shape(int ppt, uint32_t nt, Fn fn) {
    switch (nt) {
        case 256: return dispatch_bin_ppt<256>(ppt, fn);
        case 512: return dispatch_bin_ppt<512>(ppt, fn);
        default: return dispatch_bin_ppt<1024>(ppt, fn);
    }
}

}  // namespace bin
}  // namespace mm
