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
#include "mm_device.h"

namespace mm {
namespace {

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

template <int DIM, bool WRAP, int PHASE, int PPT>
__global__ __launch_bounds__(256) void bin_kernel(BinArgs a) {
    constexpr uint32_t P = 256u * PPT;
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + sizeof(uint64_t) * P);
    __shared__ uint32_t wave_sum[4];
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = a.ntiles;
    const uint32_t shift = a.shift;
    const uint32_t mask = (1u << shift) - 1u;
    const uint32_t base = blockIdx.x * P;
    const PointArgs& p = a.p;

    for (uint32_t b = tid; b <= nt; b += 256u) hist[b] = 0u;
    if (blockIdx.x == 0 && tid == 0) *a.stamp_out = a.stamp;

    float xs[PPT], ys[PPT], zs[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = base + k * 256u + tid;
        if (i < p.n) {
            load_point<DIM>(p.pos, i, xs[k], ys[k], zs[k]);
        } else {
            xs[k] = 0.0f;
            ys[k] = 0.0f;
            zs[k] = 0.0f;
        }
    }
    __syncthreads();

    uint32_t pix[PPT], dep[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t i = base + k * 256u + tid;
        pix[k] = kNoPixel;
        dep[k] = 0u;
        if (i < p.n) {
            float x = xs[k], y = ys[k], z = zs[k];
            if constexpr ((PHASE & kDisplace) != 0) {
                displace<DIM, WRAP>(p, i, x, y, z);
                store_point<DIM>(p.pos, i, x, y, z);
            }
            int32_t px, py;
            uint32_t bits;
            if (project<DIM>(p, x, y, z, px, py, bits)) {
                const uint32_t ux = static_cast<uint32_t>(px), uy = static_cast<uint32_t>(py);
                pix[k] = (uy << 16) | ux;
                dep[k] = bits;
                atomicAdd(&hist[(uy >> shift) * a.tiles_x + (ux >> shift)], 1u);
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
        const uint32_t slot = atomicAdd(&hist[(uy >> shift) * a.tiles_x + (ux >> shift)], 1u);
        const uint32_t local = static_cast<uint32_t>(k) * 256u + tid;
        stage[slot] = (static_cast<uint64_t>(dep[k]) << 32) |
                      static_cast<uint64_t>((local << 16) | ((uy & mask) << 8) | (ux & mask));
    }
    __syncthreads();

    // hist[b] is now the end of bin b (= start of bin b + 1); hist[nt] the total
    const uint32_t total = hist[nt];
    uint64_t* seg = a.seg + static_cast<uint64_t>(blockIdx.x) * P;
    for (uint32_t j = tid; j < total; j += 256u) seg[j] = stage[j];
    uint16_t* row = a.table + static_cast<uint64_t>(blockIdx.x) * (nt + 1u);
    for (uint32_t b = tid; b <= nt; b += 256u)
        row[b] = static_cast<uint16_t>(b == 0 ? 0u : hist[b - 1]);
    // Stamp the tiles that received points. All workgroups write the same
    // value, so the stores are plain cached ones (relaxed atomics at
    // wavefront scope carry no cache-bypass bits); the kernel boundary makes
    // them visible to the tile pass.
    for (uint32_t b = tid; b < nt; b += 256u) {
        const uint32_t s = b == 0 ? 0u : hist[b - 1];
        if (hist[b] > s) store_flag(&a.active[b], a.stamp);
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
__device__ __forceinline__ uint32_t tile_flag(const TileArgs& a, uint32_t t) {
    return load_flag(&a.active[t]);
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
__global__ __launch_bounds__(1024) void tile_kernel(TileArgs a) {
    constexpr uint32_t S = 1u << SHIFT;
    constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    constexpr uint32_t kCol = 4096;    // bin workgroups per pass over the column
    constexpr uint32_t kGroup = S;     // lanes reading one chunk
    constexpr uint32_t kGroups = 1024u / kGroup;
    constexpr uint32_t kInFlight = 16; // chunks per lane group per round
    constexpr uint32_t kPieces = 2;    // records per lane per chunk per round
    __shared__ uint64_t keys[A * A];
    __shared__ uint32_t col[kCol];     // start << 16 | count, per bin workgroup
    uint32_t t, z;
    tile_of_block(blockIdx.x, a.splits, t, z);
    if (t >= a.ntiles) return;
    if (tile_flag(a, t) != *a.stamp_in) return;  // nothing to draw
    const uint32_t tid = threadIdx.x;
    // this split takes bin workgroups [w_lo, w_hi)
    const uint32_t w_lo = static_cast<uint32_t>(static_cast<uint64_t>(a.num_wg) * z / a.splits);
    const uint32_t w_hi = static_cast<uint32_t>(static_cast<uint64_t>(a.num_wg) * (z + 1) / a.splits);
    for (uint32_t q = tid; q < A * A; q += 1024u) keys[q] = kEmptyKey;
    const uint32_t group = tid / kGroup, sub = tid % kGroup;
    const uint32_t stride = a.ntiles + 1u;
    const uint32_t P = a.points_per_wg;

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
                const uint16_t* row = a.table + static_cast<uint64_t>(base + c) * stride;
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
            uint32_t v[kInFlight];  // start << 16 | count of chunk c0 + u * kGroups
#pragma unroll
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t c = c0 + u * kGroups;
                v[u] = c < nb ? col[c] : 0u;
                const uint64_t* src = a.seg + static_cast<uint64_t>(base + c) * P + (v[u] >> 16);
#pragma unroll
                for (uint32_t p = 0; p < kPieces; ++p) {
                    const uint32_t j = sub + p * kGroup;
                    r[u][p] = j < (v[u] & 0xFFFFu) ? src[j] : 0ull;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t gbase = (base + c0 + u * kGroups) * P;
#pragma unroll
                for (uint32_t p = 0; p < kPieces; ++p)
                    if (sub + p * kGroup < (v[u] & 0xFFFFu))
                        splat_record<FOOT, S, A>(keys, r[u][p], gbase);
            }
            // the rest of chunks longer than kPieces * kGroup records
#pragma unroll 1
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint32_t cnt = v[u] & 0xFFFFu;
                if (cnt <= kPieces * kGroup) continue;
                const uint32_t gbase = (base + c0 + u * kGroups) * P;
                const uint64_t* src = a.seg + static_cast<uint64_t>(gbase) + (v[u] >> 16);
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
    uint64_t* part = a.part + (static_cast<uint64_t>(t) * a.splits + z) * (A * A);
    for (uint32_t q = tid; q < A * A; q += 1024u) part[q] = keys[q];
}

// Per tile: the minimum of the splits' partial keys, then RGBA8 (edge keys and
// the apron of 3x3 footprints go to the seam pass). A tile with nothing to
// draw is cleared if the previous frame drew it; otherwise its pixels are
// already 0.
template <int FOOT, int SHIFT>
__global__ __launch_bounds__(256) void merge_kernel(TileArgs a) {
    constexpr uint32_t S = 1u << SHIFT;
    constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    const uint32_t t = blockIdx.x;
    if (t >= a.ntiles) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t tx = t % a.tiles_x, ty = t / a.tiles_x;
    const uint32_t x0 = tx << SHIFT, y0 = ty << SHIFT;
    const uint32_t wt = min(S, a.width - x0), ht = min(S, a.height - y0);
    uint32_t* out = a.colour + static_cast<uint64_t>(y0) * a.width + x0;
    const uint32_t stamp = *a.stamp_in, flag = tile_flag(a, t);
    if (flag != stamp) {
        if (flag == stamp - 1u) {
            for (uint32_t q = tid; q < S * S; q += 256u) {
                const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
                if (lx < wt && ly < ht) out[static_cast<uint64_t>(ly) * a.width + lx] = 0u;
            }
        }
        return;
    }
    const uint64_t* part = a.part + static_cast<uint64_t>(t) * a.splits * (A * A);
    auto key_at = [&](uint32_t q) {
        uint64_t k = part[q];
        for (uint32_t z = 1; z < a.splits; ++z) {
            const uint64_t v = part[static_cast<uint64_t>(z) * (A * A) + q];
            k = v < k ? v : k;
        }
        return k;
    };
    for (uint32_t q = tid; q < S * S; q += 256u) {
        const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
        if (lx >= wt || ly >= ht) continue;
        if constexpr (FOOT == 1) {
            out[static_cast<uint64_t>(ly) * a.width + lx] = colour_of(key_at(q), a.seed_lo, a.seed_hi);
        } else {
            const uint64_t k = key_at((ly + 1) * A + lx + 1);
            if (lx == 0 || ly == 0 || lx == S - 1 || ly == S - 1) {
                uint64_t* bd = a.border + static_cast<uint64_t>(t) * (4 * S);
                if (ly == 0) bd[lx] = k;
                if (ly == S - 1) bd[S + lx] = k;
                if (lx == 0) bd[2 * S + ly] = k;
                if (lx == S - 1) bd[3 * S + ly] = k;
            } else {
                out[static_cast<uint64_t>(ly) * a.width + lx] = colour_of(k, a.seed_lo, a.seed_hi);
            }
        }
    }
    if constexpr (FOOT == 3) {
        uint64_t* ap = a.apron + static_cast<uint64_t>(t) * (4 * S + 4);
        for (uint32_t q = tid; q < 4 * S + 4; q += 256u) {
            uint32_t ax, ay;
            ring_coord<S>(q, ax, ay);
            ap[q] = key_at(ay * A + ax);
        }
    }
}

// Edge pixels of the 3x3 footprint: min of the tile's own edge keys and the
// aprons of the (active) neighbours that cover them, then resolve.
template <int SHIFT>
__global__ __launch_bounds__(256) void seam_kernel(TileArgs a) {
    constexpr uint32_t S = 1u << SHIFT;
    const uint32_t t = blockIdx.x;
    if (t >= a.ntiles) return;
    const uint32_t stamp = *a.stamp_in;
    const int32_t tx = static_cast<int32_t>(t % a.tiles_x), ty = static_cast<int32_t>(t / a.tiles_x);
    const uint32_t x0 = static_cast<uint32_t>(tx) << SHIFT, y0 = static_cast<uint32_t>(ty) << SHIFT;
    const uint32_t wt = min(S, a.width - x0), ht = min(S, a.height - y0);
    const uint32_t own_flag = tile_flag(a, t);
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
            if ((ox != 0 || oy != 0) && nx >= 0 && ny >= 0 && nx < static_cast<int32_t>(a.tiles_x) &&
                ny < static_cast<int32_t>(a.tiles_y)) {
                const uint32_t f = tile_flag(a, static_cast<uint32_t>(ny) * a.tiles_x + nx);
                act = f == stamp;
                any = any || act || f == stamp - 1u;
            }
            nb_active[(oy + 1) * 3 + ox + 1] = act;
        }
    if (!any) return;
    uint32_t* out = a.colour + static_cast<uint64_t>(y0) * a.width + x0;
    const uint64_t* bd = a.border + static_cast<uint64_t>(t) * (4 * S);
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
                const uint32_t n = static_cast<uint32_t>(ty + oy) * a.tiles_x + static_cast<uint32_t>(tx + ox);
                const uint64_t v = a.apron[static_cast<uint64_t>(n) * (4 * S + 4) +
                                           ring_index<S>(static_cast<uint32_t>(ax), static_cast<uint32_t>(ay))];
                k = v < k ? v : k;
            }
        out[static_cast<uint64_t>(ly) * a.width + lx] = colour_of(k, a.seed_lo, a.seed_hi);
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

template <int FOOT>
const void* pick_tile(int shift) {
    switch (shift) {
        case 4: return reinterpret_cast<const void*>(&tile_kernel<FOOT, 4>);
        case 5: return reinterpret_cast<const void*>(&tile_kernel<FOOT, 5>);
        default: return reinterpret_cast<const void*>(&tile_kernel<FOOT, 6>);
    }
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
    if (dim == 2)
        l.func = wrap ? pick_bin_ppt<2, true>(ppt, phase) : pick_bin_ppt<2, false>(ppt, phase);
    else
        l.func = wrap ? pick_bin_ppt<3, true>(ppt, phase) : pick_bin_ppt<3, false>(ppt, phase);
    const uint64_t P = 256ull * static_cast<uint64_t>(ppt);
    l.block = dim3(256);
    l.grid = dim3(static_cast<uint32_t>((static_cast<uint64_t>(n) + P - 1) / P));
    l.shared = static_cast<uint32_t>(bin_lds_bytes(ppt, ntiles));
    return l;
}

Launch tile_launch(int footprint, int shift, uint32_t ntiles, uint32_t splits) {
    Launch l;
    l.func = footprint == 3 ? pick_tile<3>(shift) : pick_tile<1>(shift);
    l.block = dim3(1024);
    l.grid = dim3((ntiles + 511u) / 512u * 512u * splits);  // whole runs of 8 XCDs x 64 tiles
    l.shared = 0;
    return l;
}

Launch merge_launch(int footprint, int shift, uint32_t ntiles) {
    Launch l;
    if (footprint == 3)
        l.func = shift == 4 ? reinterpret_cast<const void*>(&merge_kernel<3, 4>)
               : shift == 5 ? reinterpret_cast<const void*>(&merge_kernel<3, 5>)
                            : reinterpret_cast<const void*>(&merge_kernel<3, 6>);
    else
        l.func = shift == 4 ? reinterpret_cast<const void*>(&merge_kernel<1, 4>)
               : shift == 5 ? reinterpret_cast<const void*>(&merge_kernel<1, 5>)
                            : reinterpret_cast<const void*>(&merge_kernel<1, 6>);
    l.block = dim3(256);
    l.grid = dim3(ntiles);
    l.shared = 0;
    return l;
}

Launch seam_launch(int shift, uint32_t ntiles) {
    Launch l;
    switch (shift) {
        case 4: l.func = reinterpret_cast<const void*>(&seam_kernel<4>); break;
        case 5: l.func = reinterpret_cast<const void*>(&seam_kernel<5>); break;
        default: l.func = reinterpret_cast<const void*>(&seam_kernel<6>); break;
    }
    l.block = dim3(256);
    l.grid = dim3(ntiles);
    l.shared = 0;
    return l;
}

}  // namespace mm
