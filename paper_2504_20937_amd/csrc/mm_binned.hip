// Binned splat (gfx950): the depth test runs in LDS, with no global atomics.
//
// Global 64-bit atomics execute outside the XCD's L2 on this part and top
// out near 27 G/s whatever the address pattern, so the splat is split:
//
// bin kernel  (one workgroup per P = 256 * PPT consecutive points):
//   load -> displace (+store) -> project; count points per screen tile in
//   LDS; exclusive scan; place each point's 8-byte record in LDS sorted by
//   tile; write the records (coalesced) as the workgroup's segment and the
//   tile start offsets as one table row (u16). Tiles that received points
//   are stamped active for the frame.
//   record = depth_bits << 32 | local_index << 16 | y_in_tile << 8 | x_in_tile
//
// tile kernel (one workgroup per screen tile):
//   (split into `splits` workgroups per tile, each over a share of the bin
//   workgroups) pull the tile's column of the table into LDS, read the
//   chunks coalesced (a group of lanes per chunk, many chunks in flight),
//   take the min (depth_bits << 32 | index) per pixel with LDS atomics, and
//   write the partial keys of the tile.
// merge kernel (one workgroup per tile): min over the splits, resolve to
//   RGBA8 directly: no full-screen key buffer, no clear pass. With the 3x3
//   footprint the tile carries a one-pixel apron; edge pixels and the apron
//   go to small global arrays, and the seam kernel merges edges across tile
//   borders.
//
// The per-chunk, per-tile and per-merge work are device functions. The plain
// kernels take one cloud and one view from their kernel arguments; the
// batched kernels run many clouds and views in one launch per pass, each
// block walking a list of work items held in device memory: a bin item
// displaces its chunk once and then bins it into every view of its cloud.
#include "mm_device.h"

namespace mm {
namespace {

using namespace dev;

constexpr uint32_t kNoPixel = 0xFFFFFFFFu;
constexpr uint32_t kPadItem = 0xFFFFFFFFu;

// Work tables do not change during a launch: reading them through the
// constant address space lets the compiler use scalar loads even after the
// kernel's own global stores, so item, cloud and view fields stay uniform
// (SGPRs) instead of being treated as per-lane values.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized fields");
    using CWord = const __attribute__((address_space(4))) uint32_t;
    CWord* q = (CWord*)(p);
    T out;
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (size_t k = 0; k < sizeof(T) / 4; ++k) o[k] = q[k];
    return out;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Per-tile frame stamps: relaxed atomics at wavefront scope, which compile to
// plain cached loads and stores.
__device__ __forceinline__ void store_flag(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint32_t load_flag(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Exclusive scan of h[0..count) in place by 256 threads; h[count] = total.
// Each wave owns a contiguous run of 64-bin blocks and reads every block with
// consecutive lanes on consecutive words, so LDS accesses never conflict.
__device__ void block_exclusive_scan(uint32_t* h, uint32_t count, uint32_t* wave_sum) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nblk = (count + 63u) / 64u;
    const uint32_t per = (nblk + 3u) / 4u;
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
    for (uint32_t w = 0; w < 4; ++w) {
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
template <int DIM, int PPT>
__device__ __forceinline__ void load_chunk(const CloudArgs& c, uint32_t base, float (&xs)[PPT],
                                           float (&ys)[PPT], float (&zs)[PPT]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = min(base + k * 256u + tid, c.n - 1u);
        load_point<DIM>(c.pos, i, xs[k], ys[k], zs[k]);
    }
}

// Displace the chunk's points and store them back. Kept after the block's
// first barrier: a barrier waits for the block's outstanding stores, and the
// stores then drain while the projection runs.
template <int DIM, bool WRAP, int PPT>
__device__ __forceinline__ void displace_chunk(const CloudArgs& c, uint32_t step, uint32_t base,
                                               float (&xs)[PPT], float (&ys)[PPT],
                                               float (&zs)[PPT]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = base + k * 256u + tid;
        if (i < c.n) {
            displace<DIM, WRAP>(c, step, i, xs[k], ys[k], zs[k]);
            store_point<DIM>(c.pos, i, xs[k], ys[k], zs[k]);
        }
    }
}

// Bin one chunk of points into the tiles of one view: segment `chunk` of
// v.seg, row `chunk` of v.table, and the stamps of the tiles that received
// points. pre(i, x, y, z) runs on each point before its projection, in the
// same loop (the displacement: its stores then drain under the projection
// and histogram work). On entry hist[0..ntiles] is zero and visible to the
// whole block.
template <int DIM, int PPT, typename Pre>
__device__ __forceinline__ void bin_view(const BinView& v, uint32_t n, uint32_t chunk,
                                         uint32_t base, uint32_t shift, uint32_t stamp,
                                         float (&xs)[PPT], float (&ys)[PPT], float (&zs)[PPT],
                                         uint64_t* stage, uint32_t* hist, uint32_t* wave_sum,
                                         Pre pre) {
    constexpr uint32_t P = 256u * PPT;
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = v.ntiles;
    const uint32_t mask = (1u << shift) - 1u;

    uint32_t pix[PPT], dep[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = base + k * 256u + tid;
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
    block_exclusive_scan(hist, nt, wave_sum);
    __syncthreads();

#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (pix[k] == kNoPixel) continue;
        const uint32_t ux = pix[k] & 0xFFFFu, uy = pix[k] >> 16;
        const uint32_t slot = atomicAdd(&hist[(uy >> shift) * v.tiles_x + (ux >> shift)], 1u);
        const uint32_t local = static_cast<uint32_t>(k) * 256u + tid;
        stage[slot] = (static_cast<uint64_t>(dep[k]) << 32) |
                      static_cast<uint64_t>((local << 16) | ((uy & mask) << 8) | (ux & mask));
    }
    __syncthreads();

    // hist[b] is now the end of bin b (= start of bin b + 1); hist[nt] the total
    const uint32_t total = hist[nt];
    uint64_t* seg = v.seg + static_cast<uint64_t>(chunk) * P;
    for (uint32_t j = tid; j < total; j += 256u) seg[j] = stage[j];
    uint16_t* row = v.table + static_cast<uint64_t>(chunk) * (nt + 1u);
    for (uint32_t b = tid; b <= nt; b += 256u)
        row[b] = static_cast<uint16_t>(b == 0 ? 0u : hist[b - 1]);
    // Stamp the tiles that received points. All workgroups write the same
    // value, so the stores are plain cached ones (relaxed atomics at
    // wavefront scope carry no cache-bypass bits); the kernel boundary makes
    // them visible to the tile pass.
    for (uint32_t b = tid; b < nt; b += 256u) {
        const uint32_t s = b == 0 ? 0u : hist[b - 1];
        if (hist[b] > s) store_flag(&v.active[b], stamp);
    }
}

template <int DIM, bool WRAP, int PHASE, int PPT>
__global__ __launch_bounds__(256) void bin_kernel(BinArgs a) {
    constexpr uint32_t P = 256u * PPT;
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + sizeof(uint64_t) * P);
    __shared__ uint32_t wave_sum[4];
    const uint32_t tid = threadIdx.x;
    const uint32_t base = blockIdx.x * P;

    for (uint32_t b = tid; b <= a.v.ntiles; b += 256u) hist[b] = 0u;
    if (blockIdx.x == 0 && tid == 0) *a.stamp_out = a.stamp;
    float xs[PPT], ys[PPT], zs[PPT];
    load_chunk<DIM, PPT>(a.c, base, xs, ys, zs);
    __syncthreads();
    const CloudArgs c = a.c;  // by value: the key schedule is then shared by all points
    bin_view<DIM, PPT>(a.v, c.n, blockIdx.x, base, a.shift, a.stamp, xs, ys, zs, stage, hist,
                       wave_sum, [c](uint32_t i, float& x, float& y, float& z) {
                           if constexpr ((PHASE & kDisplace) != 0) {
                               displace<DIM, WRAP>(c, c.step, i, x, y, z);
                               store_point<DIM>(c.pos, i, x, y, z);
                           }
                       });
}

// One step of point i of cloud c with the cloud's own fold limit.
template <int DIM>
__device__ __forceinline__ void displace_cloud(const CloudArgs& c, uint32_t i, float& x, float& y,
                                               float& z) {
    displace<DIM, false>(c, c.step, i, x, y, z);
    x = fold_to(x, c.fold_lim);
    y = fold_to(y, c.fold_lim);
    if constexpr (DIM == 3) z = fold_to(z, c.fold_lim);
    store_point<DIM>(c.pos, i, x, y, z);
}

// Items (cloud, chunk): displace the chunk once, then bin it into each of the
// cloud's views in turn, reusing the LDS stage and histogram. Each cloud
// carries its own step and fold limit. PERSIST: each block loops over items
// blockIdx.x, blockIdx.x + gridDim.x, ...; else one item per block.
template <int DIM, int PHASE, int PPT, bool PERSIST>
__global__ __launch_bounds__(256) void batch_bin_kernel(BatchBinArgs a) {
    constexpr uint32_t P = 256u * PPT;
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + sizeof(uint64_t) * P);
    __shared__ uint32_t wave_sum[4];
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) *a.stamp_out = a.stamp;
    auto run_item = [&](uint32_t it) {
        const uint2 item = load_uniform(&a.item[it]);
        const CloudArgs c = load_uniform(&a.clouds[item.x]);
        const uint32_t base = item.y * P;
        const uint32_t v0 = load_uniform(&a.first_view[item.x]);
        const uint32_t v1 = load_uniform(&a.first_view[item.x + 1]);
        for (uint32_t b = tid; b <= load_uniform(&a.views[v0].ntiles); b += 256u) hist[b] = 0u;
        float xs[PPT], ys[PPT], zs[PPT];
        load_chunk<DIM, PPT>(c, base, xs, ys, zs);
        __syncthreads();
        // the first view displaces
        bin_view<DIM, PPT>(load_uniform(&a.views[v0]), c.n, item.y, base, a.shift, a.stamp, xs, ys,
                           zs, stage, hist, wave_sum, [&](uint32_t i, float& x, float& y, float& z) {
                               if constexpr ((PHASE & kDisplace) != 0) displace_cloud<DIM>(c, i, x, y, z);
                           });
        __syncthreads();  // stage and hist free for the next view or item
        // Further views read the (displaced) chunk again, mostly from L2:
        // keeping it, or its addresses, in registers across the first view
        // costs more in occupancy than the reload. The empty asm hides that
        // base2 equals base, so the addresses are formed anew.
        uint32_t base2 = base;
        asm volatile("" : "+v"(base2));
        for (uint32_t vi = v0 + 1; vi < v1; ++vi) {
            const BinView v = load_uniform(&a.views[vi]);
            for (uint32_t b = tid; b <= v.ntiles; b += 256u) hist[b] = 0u;
            load_chunk<DIM, PPT>(c, base2, xs, ys, zs);
            __syncthreads();
            bin_view<DIM, PPT>(v, c.n, item.y, base2, a.shift, a.stamp, xs, ys, zs, stage, hist,
                               wave_sum, [](uint32_t, float&, float&, float&) {});
            __syncthreads();
        }
    };
    if constexpr (PERSIST) {
        for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) run_item(it);
    } else {
        if (blockIdx.x < a.items) run_item(blockIdx.x);
    }
}

// Items (cloud, chunk) of clouds without views: displacement only.
template <int DIM, int PPT>
__global__ __launch_bounds__(256) void batch_displace_kernel(BatchBinArgs a) {
    constexpr uint32_t P = 256u * PPT;
    for (uint32_t it = blockIdx.x; it < a.disp_items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.disp_item[it]);
        const CloudArgs c = load_uniform(&a.clouds[item.x]);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint32_t i = item.y * P + k * 256u + threadIdx.x;
            if (i >= c.n) continue;
            float x, y, z;
            load_point<DIM>(c.pos, i, x, y, z);
            displace_cloud<DIM>(c, i, x, y, z);
        }
    }
}

// 64 consecutive tiles share one 128-byte line of every table row; blocks go
// round-robin over the 8 XCDs, so each run of 64 tiles (for one split of the
// column) is mapped onto one XCD, to read every table line into one L2 once.
// Block b -> (tile, split); the grid is ceil(ntiles / 512) * 512 * splits.
__device__ __forceinline__ void tile_of_block(uint32_t b, uint32_t splits, uint32_t& t,
                                              uint32_t& z) {
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t q = k >> 6;
    t = ((q / splits) * 8u + x) * 64u + (k & 63u);
    z = q % splits;
}

// Position q on the ring of an (S+2)^2 apron tile <-> LDS coordinates.
template <uint32_t S>
__device__ __forceinline__ void ring_coord(uint32_t q, uint32_t& ax, uint32_t& ay) {
    if (q < S + 2) {
        ax = q;
        ay = 0;
    } else if (q < 2 * S + 4) {
        ax = q - (S + 2);
        ay = S + 1;
    } else if (q < 3 * S + 4) {
        ax = 0;
        ay = q - (2 * S + 4) + 1;
    } else {
        ax = S + 1;
        ay = q - (3 * S + 4) + 1;
    }
}

template <uint32_t S>
__device__ __forceinline__ uint32_t ring_index(uint32_t ax, uint32_t ay) {
    if (ay == 0) return ax;
    if (ay == S + 1) return S + 2 + ax;
    if (ax == 0) return 2 * S + 4 + ay - 1;
    return 3 * S + 4 + ay - 1;
}

// The frame stamp is never 0 and rises by one per render; a tile's flag
// equal to stamp - 1 means the tile was drawn in the previous frame.
__device__ __forceinline__ uint32_t tile_flag(const TileView& v, uint32_t t) {
    return load_flag(&v.active[t]);
}

template <int FOOT, uint32_t S, uint32_t A>
__device__ __forceinline__ void splat_record(uint64_t* keys, uint64_t r, uint32_t gbase) {
    const uint32_t lo = static_cast<uint32_t>(r);
    const uint32_t cx = lo & 0xFFu, cy = (lo >> 8) & 0xFFu;
    const uint64_t key = (r & 0xFFFFFFFF00000000ull) | static_cast<uint64_t>(gbase + (lo >> 16));
    if constexpr (FOOT == 1) {
        atomic_min_lds(&keys[cy * S + cx], key);
    } else {
#pragma unroll
        for (uint32_t dy = 0; dy < 3; ++dy)
#pragma unroll
            for (uint32_t dx = 0; dx < 3; ++dx) atomic_min_lds(&keys[(cy + dy) * A + cx + dx], key);
    }
}

template <int FOOT, int SHIFT>
struct TileShape {
    static constexpr uint32_t S = 1u << SHIFT;
    static constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    static constexpr uint32_t kCol = 4096;  // bin workgroups per pass over the column
};

// Split z of tile t: the per-pixel minimum over the records of bin workgroups
// [num_wg * z / splits, num_wg * (z + 1) / splits), written as partial keys.
// 1024 threads; keys (A * A) and col (kCol) are LDS. Ends with the block
// synchronised.
template <int FOOT, int SHIFT>
__device__ __forceinline__ void tile_split(const TileView& v, uint32_t t, uint32_t z, uint32_t P,
                                           uint64_t* keys, uint32_t* col) {
    using Sh = TileShape<FOOT, SHIFT>;
    constexpr uint32_t S = Sh::S, A = Sh::A, kCol = Sh::kCol;
    constexpr uint32_t kGroup = S;     // lanes reading one chunk
    constexpr uint32_t kGroups = 1024u / kGroup;
    constexpr uint32_t kInFlight = 16; // chunks per lane group per round
    constexpr uint32_t kPieces = 2;    // records per lane per chunk per round
    const uint32_t tid = threadIdx.x;
    const uint32_t w_lo = static_cast<uint32_t>(static_cast<uint64_t>(v.num_wg) * z / v.splits);
    const uint32_t w_hi = static_cast<uint32_t>(static_cast<uint64_t>(v.num_wg) * (z + 1) / v.splits);
    for (uint32_t q = tid; q < A * A; q += 1024u) keys[q] = kEmptyKey;
    const uint32_t group = tid / kGroup, sub = tid % kGroup;
    const uint32_t stride = v.ntiles + 1u;

    for (uint32_t base = w_lo; base < w_hi; base += kCol) {
        const uint32_t nb = min(kCol, w_hi - base);
        __syncthreads();  // keys initialised / previous pass done with col
        uint32_t cs[kCol / 1024], ce[kCol / 1024];
#pragma unroll
        for (uint32_t k = 0; k < kCol / 1024; ++k) {
            const uint32_t c = tid + k * 1024u;
            cs[k] = 0;
            ce[k] = 0;
            if (c < nb) {
                const uint16_t* row = v.table + static_cast<uint64_t>(base + c) * stride;
                cs[k] = row[t];
                ce[k] = row[t + 1];
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < kCol / 1024; ++k) {
            const uint32_t c = tid + k * 1024u;
            if (c < nb) col[c] = (cs[k] << 16) | (ce[k] - cs[k]);
        }
        __syncthreads();
        for (uint32_t c0 = group; c0 < nb; c0 += kGroups * kInFlight) {
            uint64_t r[kInFlight][kPieces];
            uint32_t cv[kInFlight];  // start << 16 | count of chunk c0 + u * kGroups
#pragma unroll
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t c = c0 + u * kGroups;
                cv[u] = c < nb ? col[c] : 0u;
                const uint64_t* src = v.seg + static_cast<uint64_t>(base + c) * P + (cv[u] >> 16);
#pragma unroll
                for (uint32_t p = 0; p < kPieces; ++p) {
                    const uint32_t j = sub + p * kGroup;
                    r[u][p] = j < (cv[u] & 0xFFFFu) ? src[j] : 0ull;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t gbase = (base + c0 + u * kGroups) * P;
#pragma unroll
                for (uint32_t p = 0; p < kPieces; ++p)
                    if (sub + p * kGroup < (cv[u] & 0xFFFFu))
                        splat_record<FOOT, S, A>(keys, r[u][p], gbase);
            }
            // the rest of chunks longer than kPieces * kGroup records
#pragma unroll 1
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t cnt = cv[u] & 0xFFFFu;
                if (cnt <= kPieces * kGroup) continue;
                const uint32_t gbase = (base + c0 + u * kGroups) * P;
                const uint64_t* src = v.seg + static_cast<uint64_t>(gbase) + (cv[u] >> 16);
                for (uint32_t j = kPieces * kGroup + sub; j < cnt; j += 4 * kGroup) {
                    uint64_t rr[4];
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) rr[q] = j + q * kGroup < cnt ? src[j + q * kGroup] : 0ull;
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q)
                        if (j + q * kGroup < cnt) splat_record<FOOT, S, A>(keys, rr[q], gbase);
                }
            }
        }
    }
    __syncthreads();
    uint64_t* part = v.part + (static_cast<uint64_t>(t) * v.splits + z) * (A * A);
    for (uint32_t q = tid; q < A * A; q += 1024u) part[q] = keys[q];
    __syncthreads();
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(1024) void tile_kernel(TileArgs a) {
    using Sh = TileShape<FOOT, SHIFT>;
    __shared__ uint64_t keys[Sh::A * Sh::A];
    __shared__ uint32_t col[Sh::kCol];  // start << 16 | count, per bin workgroup
    uint32_t t, z;
    tile_of_block(blockIdx.x, a.v.splits, t, z);
    if (t >= a.v.ntiles) return;
    if (tile_flag(a.v, t) != *a.stamp_in) return;  // nothing to draw
    tile_split<FOOT, SHIFT>(a.v, t, z, a.points_per_wg, keys, col);
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(1024) void batch_tile_kernel(BatchTileArgs a) {
    using Sh = TileShape<FOOT, SHIFT>;
    __shared__ uint64_t keys[Sh::A * Sh::A];
    __shared__ uint32_t col[Sh::kCol];
    const uint32_t stamp = *a.stamp_in;
    for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.item[it]);
        if (item.x == kPadItem) continue;
        const TileView v = load_uniform(&a.views[item.x]);
        const uint32_t t = item.y >> 3, z = item.y & 7u;
        if (tile_flag(v, t) != stamp) continue;
        tile_split<FOOT, SHIFT>(v, t, z, a.points_per_wg, keys, col);
    }
}

// Tile t: the minimum of the splits' partial keys, then RGBA8 (edge keys and
// the apron of 3x3 footprints go to the seam pass). A tile with nothing to
// draw is cleared if the previous frame drew it; otherwise its pixels are
// already 0. 256 threads.
template <int FOOT, int SHIFT>
__device__ __forceinline__ void merge_tile(const TileView& v, uint32_t t, uint32_t stamp) {
    constexpr uint32_t S = 1u << SHIFT;
    constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    const uint32_t tid = threadIdx.x;
    const uint32_t tx = t % v.tiles_x, ty = t / v.tiles_x;
    const uint32_t x0 = tx << SHIFT, y0 = ty << SHIFT;
    const uint32_t wt = min(S, v.width - x0), ht = min(S, v.height - y0);
    uint32_t* out = v.colour + static_cast<uint64_t>(y0) * v.width + x0;
    const uint32_t flag = tile_flag(v, t);
    if (flag != stamp) {
        if (flag == stamp - 1u || v.full_clear) {
            for (uint32_t q = tid; q < S * S; q += 256u) {
                const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
                if (lx < wt && ly < ht) out[static_cast<uint64_t>(ly) * v.width + lx] = 0u;
            }
        }
        return;
    }
    const uint64_t* part = v.part + static_cast<uint64_t>(t) * v.splits * (A * A);
    auto key_at = [&](uint32_t q) {
        uint64_t k = part[q];
        for (uint32_t z = 1; z < v.splits; ++z) {
            const uint64_t p = part[static_cast<uint64_t>(z) * (A * A) + q];
            k = p < k ? p : k;
        }
        return k;
    };
    for (uint32_t q = tid; q < S * S; q += 256u) {
        const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
        if (lx >= wt || ly >= ht) continue;
        if constexpr (FOOT == 1) {
            out[static_cast<uint64_t>(ly) * v.width + lx] = colour_of(key_at(q), v.seed_lo, v.seed_hi);
        } else {
            const uint64_t k = key_at((ly + 1) * A + lx + 1);
            if (lx == 0 || ly == 0 || lx == S - 1 || ly == S - 1) {
                uint64_t* bd = v.border + static_cast<uint64_t>(t) * (4 * S);
                if (ly == 0) bd[lx] = k;
                if (ly == S - 1) bd[S + lx] = k;
                if (lx == 0) bd[2 * S + ly] = k;
                if (lx == S - 1) bd[3 * S + ly] = k;
            } else {
                out[static_cast<uint64_t>(ly) * v.width + lx] = colour_of(k, v.seed_lo, v.seed_hi);
            }
        }
    }
    if constexpr (FOOT == 3) {
        uint64_t* ap = v.apron + static_cast<uint64_t>(t) * (4 * S + 4);
        for (uint32_t q = tid; q < 4 * S + 4; q += 256u) {
            uint32_t ax, ay;
            ring_coord<S>(q, ax, ay);
            ap[q] = key_at(ay * A + ax);
        }
    }
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(256) void merge_kernel(TileArgs a) {
    const uint32_t t = blockIdx.x;
    if (t >= a.v.ntiles) return;
    merge_tile<FOOT, SHIFT>(a.v, t, *a.stamp_in);
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(256) void batch_merge_kernel(BatchTileArgs a) {
    const uint32_t stamp = *a.stamp_in;
    for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.item[it]);
        if (item.x == kPadItem) continue;
        const TileView v = load_uniform(&a.views[item.x]);
        merge_tile<FOOT, SHIFT>(v, item.y >> 3, stamp);
    }
}

// Edge pixels of tile t with the 3x3 footprint: min of the tile's own edge
// keys and the aprons of the (active) neighbours that cover them, then
// resolve. 256 threads.
template <int SHIFT>
__device__ __forceinline__ void seam_tile(const TileView& v, uint32_t t, uint32_t stamp) {
    constexpr uint32_t S = 1u << SHIFT;
    const int32_t tx = static_cast<int32_t>(t % v.tiles_x), ty = static_cast<int32_t>(t / v.tiles_x);
    const uint32_t x0 = static_cast<uint32_t>(tx) << SHIFT, y0 = static_cast<uint32_t>(ty) << SHIFT;
    const uint32_t wt = min(S, v.width - x0), ht = min(S, v.height - y0);
    const uint32_t own_flag = tile_flag(v, t);
    const bool own = own_flag == stamp;
    // edges need work if this tile or a neighbour is drawn now, or was drawn
    // in the previous frame (its edge pixels may hold last frame's colours)
    bool nb_active[9];
    bool any = own || own_flag == stamp - 1u;
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
            const int nx = tx + ox, ny = ty + oy;
            bool act = false;
            if ((ox != 0 || oy != 0) && nx >= 0 && ny >= 0 && nx < static_cast<int32_t>(v.tiles_x) &&
                ny < static_cast<int32_t>(v.tiles_y)) {
                const uint32_t f = tile_flag(v, static_cast<uint32_t>(ny) * v.tiles_x + nx);
                act = f == stamp;
                any = any || act || f == stamp - 1u;
            }
            nb_active[(oy + 1) * 3 + ox + 1] = act;
        }
    if (!any) return;
    uint32_t* out = v.colour + static_cast<uint64_t>(y0) * v.width + x0;
    const uint64_t* bd = v.border + static_cast<uint64_t>(t) * (4 * S);
    for (uint32_t q = threadIdx.x; q < 4 * S; q += 256u) {
        const uint32_t side = q >> SHIFT, pos = q & (S - 1u);
        if (side >= 2 && (pos == 0 || pos == S - 1)) continue;  // corners: done by rows
        const uint32_t lx = side == 0 || side == 1 ? pos : (side == 2 ? 0u : S - 1u);
        const uint32_t ly = side == 2 || side == 3 ? pos : (side == 0 ? 0u : S - 1u);
        if (lx >= wt || ly >= ht) continue;
        uint64_t k = own ? bd[q] : kEmptyKey;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                if (!nb_active[(oy + 1) * 3 + ox + 1]) continue;
                const int32_t ax = static_cast<int32_t>(lx) - ox * static_cast<int32_t>(S) + 1;
                const int32_t ay = static_cast<int32_t>(ly) - oy * static_cast<int32_t>(S) + 1;
                if (ax < 0 || ay < 0 || ax > static_cast<int32_t>(S) + 1 || ay > static_cast<int32_t>(S) + 1)
                    continue;
                const uint32_t n = static_cast<uint32_t>(ty + oy) * v.tiles_x + static_cast<uint32_t>(tx + ox);
                const uint64_t p = v.apron[static_cast<uint64_t>(n) * (4 * S + 4) +
                                           ring_index<S>(static_cast<uint32_t>(ax), static_cast<uint32_t>(ay))];
                k = p < k ? p : k;
            }
        out[static_cast<uint64_t>(ly) * v.width + lx] = colour_of(k, v.seed_lo, v.seed_hi);
    }
}

template <int SHIFT>
__global__ __launch_bounds__(256) void seam_kernel(TileArgs a) {
    const uint32_t t = blockIdx.x;
    if (t >= a.v.ntiles) return;
    seam_tile<SHIFT>(a.v, t, *a.stamp_in);
}

template <int SHIFT>
__global__ __launch_bounds__(256) void batch_seam_kernel(BatchTileArgs a) {
    const uint32_t stamp = *a.stamp_in;
    for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.item[it]);
        if (item.x == kPadItem) continue;
        const TileView v = load_uniform(&a.views[item.x]);
        seam_tile<SHIFT>(v, item.y >> 3, stamp);
    }
}

template <int DIM, bool WRAP, int PPT>
const void* pick_bin_phase(Phase phase) {
    if (phase == kRender) return reinterpret_cast<const void*>(&bin_kernel<DIM, WRAP, kRender, PPT>);
    return reinterpret_cast<const void*>(&bin_kernel<DIM, WRAP, kDisplaceRender, PPT>);
}

template <int DIM, bool WRAP>
const void* pick_bin_ppt(int ppt, Phase phase) {
    switch (ppt) {
        case 4: return pick_bin_phase<DIM, WRAP, 4>(phase);
        case 8: return pick_bin_phase<DIM, WRAP, 8>(phase);
        default: return pick_bin_phase<DIM, WRAP, 16>(phase);
    }
}

const void* pick_bin(int dim, bool wrap, int ppt, Phase phase) {
    if (dim == 2) return wrap ? pick_bin_ppt<2, true>(ppt, phase) : pick_bin_ppt<2, false>(ppt, phase);
    return wrap ? pick_bin_ppt<3, true>(ppt, phase) : pick_bin_ppt<3, false>(ppt, phase);
}

template <int DIM, int PPT, bool PERSIST>
const void* pick_batch_bin_phase(Phase phase) {
    if (phase == kRender)
        return reinterpret_cast<const void*>(&batch_bin_kernel<DIM, kRender, PPT, PERSIST>);
    return reinterpret_cast<const void*>(&batch_bin_kernel<DIM, kDisplaceRender, PPT, PERSIST>);
}

template <int DIM, bool PERSIST>
const void* pick_batch_bin_ppt(int ppt, Phase phase) {
    switch (ppt) {
        case 4: return pick_batch_bin_phase<DIM, 4, PERSIST>(phase);
        case 8: return pick_batch_bin_phase<DIM, 8, PERSIST>(phase);
        default: return pick_batch_bin_phase<DIM, 16, PERSIST>(phase);
    }
}

template <int DIM>
const void* pick_batch_displace(int ppt) {
    switch (ppt) {
        case 4: return reinterpret_cast<const void*>(&batch_displace_kernel<DIM, 4>);
        case 8: return reinterpret_cast<const void*>(&batch_displace_kernel<DIM, 8>);
        default: return reinterpret_cast<const void*>(&batch_displace_kernel<DIM, 16>);
    }
}

template <int FOOT, int SHIFT>
const void* tile_func(bool batched) {
    return batched ? reinterpret_cast<const void*>(&batch_tile_kernel<FOOT, SHIFT>)
                   : reinterpret_cast<const void*>(&tile_kernel<FOOT, SHIFT>);
}

template <int FOOT, int SHIFT>
const void* merge_func(bool batched) {
    return batched ? reinterpret_cast<const void*>(&batch_merge_kernel<FOOT, SHIFT>)
                   : reinterpret_cast<const void*>(&merge_kernel<FOOT, SHIFT>);
}

template <int SHIFT>
const void* seam_func(bool batched) {
    return batched ? reinterpret_cast<const void*>(&batch_seam_kernel<SHIFT>)
                   : reinterpret_cast<const void*>(&seam_kernel<SHIFT>);
}

template <int FOOT>
const void* pick_tile(int shift, bool batched) {
    switch (shift) {
        case 4: return tile_func<FOOT, 4>(batched);
        case 5: return tile_func<FOOT, 5>(batched);
        default: return tile_func<FOOT, 6>(batched);
    }
}

template <int FOOT>
const void* pick_merge(int shift, bool batched) {
    switch (shift) {
        case 4: return merge_func<FOOT, 4>(batched);
        case 5: return merge_func<FOOT, 5>(batched);
        default: return merge_func<FOOT, 6>(batched);
    }
}

const void* pick_seam(int shift, bool batched) {
    switch (shift) {
        case 4: return seam_func<4>(batched);
        case 5: return seam_func<5>(batched);
        default: return seam_func<6>(batched);
    }
}

uint32_t batch_grid(uint32_t items, uint32_t grid_blocks) {
    if (grid_blocks == 0 || grid_blocks > items) return items;
    return grid_blocks;
}

}  // namespace

bool binned_shape_ok(int shift, int ppt, uint32_t splits) {
    return (shift == 4 || shift == 5 || shift == 6) && (ppt == 4 || ppt == 8 || ppt == 16) &&
           (splits == 1 || splits == 2 || splits == 4 || splits == 8);
}

size_t bin_lds_bytes(int ppt, uint32_t ntiles) {
    return sizeof(uint64_t) * 256u * static_cast<uint32_t>(ppt) + sizeof(uint32_t) * (ntiles + 1u);
}

Launch bin_launch(int dim, bool wrap, Phase phase, int ppt, uint32_t n, uint32_t ntiles) {
    Launch l;
    l.func = pick_bin(dim, wrap, ppt, phase);
    const uint64_t P = 256ull * static_cast<uint64_t>(ppt);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((static_cast<uint64_t>(n) + P - 1) / P));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, ntiles));
    return l;
}

Launch tile_launch(int footprint, int shift, uint32_t ntiles, uint32_t splits) {
    Launch l;
    l.func = footprint == 3 ? pick_tile<3>(shift, false) : pick_tile<1>(shift, false);
    l.block = dim3(1024);
    l.grid = dim3((ntiles + 511u) / 512u * 512u * splits);  // whole runs of 8 XCDs x 64 tiles
    l.shared = 0;
    return l;
}

Launch merge_launch(int footprint, int shift, uint32_t ntiles) {
    Launch l;
    l.func = footprint == 3 ? pick_merge<3>(shift, false) : pick_merge<1>(shift, false);
    l.block = dim3(256);
    l.grid = dim3(ntiles);
    l.shared = 0;
    return l;
}

Launch seam_launch(int shift, uint32_t ntiles) {
    Launch l;
    l.func = pick_seam(shift, false);
    l.block = dim3(256);
    l.grid = dim3(ntiles);
    l.shared = 0;
    return l;
}

Launch batch_bin_launch(int dim, Phase phase, int ppt, uint32_t items, uint32_t max_tiles,
                        uint32_t grid_blocks) {
    Launch l;
    const bool persist = grid_blocks != 0 && grid_blocks < items;
    if (dim == 2)
        l.func = persist ? pick_batch_bin_ppt<2, true>(ppt, phase) : pick_batch_bin_ppt<2, false>(ppt, phase);
    else
        l.func = persist ? pick_batch_bin_ppt<3, true>(ppt, phase) : pick_batch_bin_ppt<3, false>(ppt, phase);
    l.block = dim3(256);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, max_tiles));
    return l;
}

Launch batch_displace_launch(int dim, int ppt, uint32_t items, uint32_t grid_blocks) {
    Launch l;
    l.func = dim == 2 ? pick_batch_displace<2>(ppt) : pick_batch_displace<3>(ppt);
    l.block = dim3(256);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = 0;
    return l;
}

Launch batch_tile_launch(int footprint, int shift, uint32_t items, uint32_t grid_blocks) {
    Launch l;
    l.func = footprint == 3 ? pick_tile<3>(shift, true) : pick_tile<1>(shift, true);
    l.block = dim3(1024);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = 0;
    return l;
}

Launch batch_merge_launch(int footprint, int shift, uint32_t items, uint32_t grid_blocks) {
    Launch l;
    l.func = footprint == 3 ? pick_merge<3>(shift, true) : pick_merge<1>(shift, true);
    l.block = dim3(256);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = 0;
    return l;
}

Launch batch_seam_launch(int shift, uint32_t items, uint32_t grid_blocks) {
    Launch l;
    l.func = pick_seam(shift, true);
    l.block = dim3(256);
    l.grid = dim3(batch_grid(items, grid_blocks));
    l.shared = 0;
    return l;
}

}  // namespace mm
