// Tile side of the binned splat (gfx950): the per-tile depth test in LDS,
// the merge of the splits with the RGBA8 resolve, and the seam pass of 3x3
// footprints, each as a plain kernel (one view, kernel arguments) and a
// batched kernel (items (view, tile) from a device table).
//
// tile kernel (one workgroup per screen tile and split, or per piece of a
//   tile with the load-balanced pass): gather the tile's (start, end) pairs
//   from the table (or its tile-major copy, which the load-balanced pass
//   makes first), compact the non-empty runs with a block scan, walk the
//   tile's records as one flat list (64 consecutive records per wave step,
//   runs found through an LDS bitmap of run starts), take the min
//   (depth_bits << 32 | index) per centre pixel with LDS atomics, and write
//   the tile's partial keys (a 3x3 footprint as a 3x3 minimum over them).
// merge kernel (one workgroup per tile, four for 64-pixel tiles): min over
//   the splits or pieces, resolve to RGBA8 directly: no full-screen key
//   buffer, no clear pass. With the 3x3 footprint the tile carries a
//   one-pixel apron; edge pixels and the apron go to small global arrays,
//   and the seam kernel merges edges across tile borders.
#include "mm_device.h"

namespace mm {
namespace {

using namespace dev;

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

// Threads of a tile workgroup (the depth test of one tile or one piece of
// it). 512 keeps two workgroups resident per CU, so one workgroup's table
// reads and scans overlap another's record stream.
constexpr uint32_t kTileThreads = 512;

// The record's key into its centre pixel of the tile (S x S keys in LDS; the
// record's low half-word is the byte offset of the pixel's key). A 3x3
// footprint is applied afterwards, by a 3x3 minimum over the centre minima
// (exact: a pixel's key is the minimum over the records centred in its
// neighbourhood, in any grouping), so every record costs one LDS atomic
// whatever the footprint.
template <uint32_t S>
__device__ __forceinline__ void splat_record(uint64_t* keys, uint64_t r, uint32_t gbase) {
    const uint32_t lo = static_cast<uint32_t>(r);
    uint64_t* key_at = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(keys) + (lo & 0xFFFFu));
    const uint64_t key = (r & 0xFFFFFFFF00000000ull) | static_cast<uint64_t>(gbase + (lo >> 16));
    atomic_min_lds(key_at, key);
}

// Partial key block (A x A) of the tile from its centre minima: with the 3x3
// footprint, block entry (i, j) is pixel (j - 1, i - 1) of the tile and takes
// the minimum over centres (cx, cy) in [j - 2, j] x [i - 2, i] inside the tile.
template <int FOOT, uint32_t S, uint32_t A, uint32_t NT>
__device__ __forceinline__ void write_part(const uint64_t* keys, uint64_t* part) {
    const uint32_t tid = threadIdx.x;
    if constexpr (FOOT == 1) {
        for (uint32_t q = tid; q < S * S; q += NT) part[q] = keys[q];
    } else {
        for (uint32_t q = tid; q < A * A; q += NT) {
            const uint32_t i = q / A, j = q % A;
            uint64_t m = kEmptyKey;
#pragma unroll
            for (uint32_t dy = 0; dy < 3; ++dy) {
                const uint32_t cy = i - dy;  // wraps past 0: rejected below
                if (cy >= S) continue;
#pragma unroll
                for (uint32_t dx = 0; dx < 3; ++dx) {
                    const uint32_t cx = j - dx;
                    if (cx < S) m = min(m, keys[cy * S + cx]);
                }
            }
            part[q] = m;
        }
    }
}

// Sets tile t's pixels to 0 (nothing drawn): pixels q = first, first + step, ...
template <int SHIFT>
__device__ __forceinline__ void clear_tile(const TileView& v, uint32_t t, uint32_t first,
                                           uint32_t step) {
    constexpr uint32_t S = 1u << SHIFT;
    const uint32_t x0 = (t % v.tiles_x) << SHIFT, y0 = (t / v.tiles_x) << SHIFT;
    const uint32_t wt = min(S, v.width - x0), ht = min(S, v.height - y0);
    uint32_t* out = v.colour + static_cast<uint64_t>(y0) * v.width + x0;
    for (uint32_t q = first; q < S * S; q += step) {
        const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
        if (lx < wt && ly < ht) out[static_cast<uint64_t>(ly) * v.width + lx] = 0u;
    }
}

template <int FOOT, int SHIFT, uint32_t NT = kTileThreads>
struct TileShape {
    static constexpr uint32_t S = 1u << SHIFT;
    static constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    // Batched tile workgroups (256 threads) take many small tiles: a shorter
    // pass and segment leave 25 KB of LDS a workgroup instead of 49 KB, so
    // five workgroups share a CU instead of three (the 64-cloud batch frame:
    // 0.96 against 1.03 ms). Clouds of more bin workgroups take more passes.
    static constexpr uint32_t kCol = NT == 256 ? 1024 : 2048;  // bin workgroups per pass over the column
    static constexpr uint32_t kSeg = NT == 256 ? 1u << 15 : 1u << 17;  // records per segment of a pass
    static constexpr uint32_t kWindows = NT == 256 ? 6 : 12;  // 64-record windows in flight per lane
    // LDS words beside the keys: run offsets (kCol + 1, padded to even), run
    // address bias and index base (2 kCol), the segment's run-start bitmap
    // (kSeg / 32) and the scan's wave sums (2 per wave)
    static constexpr uint32_t kColLds = (kCol + 2) + 2 * kCol + kSeg / 32 + 2 * (NT / 64);
};

// Inclusive scan of two values over the 64 lanes of a wave.
__device__ __forceinline__ void wave_scan2(uint32_t& a, uint32_t& b, uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t ua = __shfl_up(a, d, 64), ub = __shfl_up(b, d, 64);
        if (lane >= d) {
            a += ua;
            b += ub;
        }
    }
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x, uint32_t lane_id) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(x), lane_id);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(x >> 32), lane_id);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Records [r0, r1) of a segment starting at record s0 of the pass's flat
// record list (the tile's non-empty runs end to end; run k holds records
// [roff[k], roff[k + 1])), splatted by one wave; r0 - s0 is a multiple of 64.
// The wave takes 64 consecutive records per window, one per lane. Bit p of
// window word i of `starts` is set when a run starts at record s0 + 64 i + p,
// so a lane's run is the window's first run plus the starts at or before it
// (mbcnt), and the next window's first run follows by a popcount: the U
// windows of a batch need no LDS round trip after their start words, which
// one read brings in. runs[k] = (address bias, index base): record f of run
// k is seg[bias + f] with point index base + local.
template <uint32_t S, uint32_t U>
__device__ __forceinline__ void splat_segment(const uint64_t* seg, uint64_t* keys,
                                              const uint32_t* roff, const uint2* runs,
                                              const uint64_t* starts, uint32_t nruns,
                                              uint32_t s0, uint32_t r0, uint32_t r1) {
    const uint32_t lane = threadIdx.x & 63u;
    // run holding record r0: roff[k] <= r0 < roff[k + 1] (roff[nruns] > r0)
    uint32_t lo = 0, hi = nruns;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (roff[mid] <= r0) lo = mid;
        else hi = mid;
    }
    uint32_t k = lo;
    const uint32_t wend = (r1 - s0 + 63u) >> 6;  // window words of the segment in use
    for (uint32_t w0 = r0; w0 < r1; w0 += 64u * U) {
        const uint32_t i0 = (w0 - s0) >> 6;
        // lane u holds the start word of window i0 + u (words past the range are 0)
        const uint64_t mine = i0 + lane < wend && lane <= U ? starts[i0 + lane] : 0ull;
        uint64_t r[U];
        uint32_t gb[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint64_t m = uniform_u64(mine, u);
            // runs started after the window's first record, up to this lane's
            const uint64_t after = m >> 1;
            const uint32_t upto = __builtin_amdgcn_mbcnt_hi(
                static_cast<uint32_t>(after >> 32),
                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(after), 0u));
            const uint32_t f = w0 + 64u * u + lane;
            const uint2 run = runs[min(k + upto, nruns - 1u)];
            const uint32_t off = f < r1 ? run.x + f : 0u;
            r[u] = *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(seg) +
                                                      (static_cast<uint64_t>(off) << 3));
            gb[u] = run.y;
            const uint64_t next = uniform_u64(mine, u + 1u);
            k += static_cast<uint32_t>(__popcll(after)) + static_cast<uint32_t>(next & 1ull);
        }
        if (w0 + 64u * U <= r1) {
            // whole windows (all but a range's last batch): no lane is past
            // the range, so no branch keeps a load from issuing with the others
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) splat_record<S>(keys, r[u], gb[u]);
        } else {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (w0 + 64u * u + lane < r1) splat_record<S>(keys, r[u], gb[u]);
        }
    }
}

// Tile t over bin workgroups [w_lo, w_hi): the per-pixel minimum of their
// records, written as partial key block `piece` of v.part, or with RESOLVE
// (1x1 footprint, the tile's whole column) resolved to RGBA8 in the frame.
// NT threads; keys (S * S centre minima) and lds (kColLds words) are LDS.
// Ends with the block synchronised.
//
// Per pass over up to kCol bin workgroups: each thread reads the (start,
// end) pairs of 4 consecutive workgroups from the table, and a block scan
// over the non-empty runs gives their flat offsets (roff) and locations. The
// flat record list is then taken in segments of up to kSeg records: the run
// starts of a segment are marked in an LDS bitmap, and its 64-record windows
// are cut into equal ranges, one per wave. A wave's work thus depends on
// the records, not on how they fall into runs.
template <int FOOT, int SHIFT, uint32_t NT = kTileThreads, bool RESOLVE = false>
__device__ __forceinline__ void tile_range(const TileView& v, uint32_t t, uint32_t w_lo,
                                           uint32_t w_hi, uint32_t piece, uint32_t P,
                                           uint64_t* keys, uint32_t* lds) {
    static_assert(!RESOLVE || FOOT == 1, "a 3x3 footprint needs the seam pass");
    using Sh = TileShape<FOOT, SHIFT, NT>;
    constexpr uint32_t S = Sh::S, A = Sh::A, kCol = Sh::kCol, kSeg = Sh::kSeg;
    constexpr uint32_t kWaves = NT / 64;
    constexpr uint32_t kPer = kCol / NT;  // bin workgroups per thread and pass
    uint32_t* roff = lds;
    uint2* runs = reinterpret_cast<uint2*>(lds + kCol + 2);
    uint32_t* bits = lds + kCol + 2 + 2 * kCol;
    uint32_t* wsum = bits + kSeg / 32;  // [0, waves): records, [waves, 2 waves): runs
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    for (uint32_t q = tid; q < S * S; q += NT) keys[q] = kEmptyKey;
    const uint32_t stride = v.ntiles + 1u;

    for (uint32_t base = w_lo; base < w_hi; base += kCol) {
        const uint32_t nb = min(kCol, w_hi - base);
        __syncthreads();  // keys initialised / previous pass done with the LDS
        // Branch-free within a lane: lanes past the column's end read its last
        // entry (count forced to 0), so all of a lane's table loads are in
        // flight together. Entries k >= per, which no lane holds for a column
        // this short (a small cloud), are neither loaded nor counted.
        const uint32_t per = (nb + NT - 1u) / NT;  // in 1 .. kPer, the same for the block
        uint32_t cs[kPer], cn[kPer];
        if (v.tcol) {  // tile-major copy: entries t and t + 1 of each row, contiguous
            const uint16_t* e0 = v.tcol + static_cast<uint64_t>(t) * v.tcol_stride + base;
            const uint16_t* e1 = e0 + v.tcol_stride;
#pragma unroll
            for (uint32_t k = 0; k < kPer; ++k) {
                const uint32_t c = min(tid * per + k, nb - 1u);
                cs[k] = k < per ? e0[c] : 0u;
                cn[k] = k < per ? e1[c] : 0u;
            }
        } else {
#pragma unroll
            for (uint32_t k = 0; k < kPer; ++k) {
                const uint32_t c = tid * per + k;
                const uint16_t* row = v.table + static_cast<uint64_t>(base + min(c, nb - 1u)) * stride;
                cs[k] = k < per ? row[t] : 0u;
                cn[k] = k < per ? row[t + 1] : 0u;
            }
        }
        uint32_t tc = 0, tr = 0;  // this thread's records and non-empty runs
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            cn[k] = k < per && tid * per + k < nb ? cn[k] - cs[k] : 0u;
            tc += cn[k];
            tr += cn[k] != 0u;
        }
        uint32_t ic = tc, ir = tr;
        wave_scan2(ic, ir, lane);
        if (lane == 63u) {
            wsum[wave] = ic;
            wsum[kWaves + wave] = ir;
        }
        __syncthreads();
        uint32_t total = 0, nruns = 0, oc = ic - tc, orr = ir - tr;
#pragma unroll
        for (uint32_t w = 0; w < kWaves; ++w) {
            const uint32_t c = wsum[w], r = wsum[kWaves + w];
            total += c;
            nruns += r;
            oc += w < wave ? c : 0u;
            orr += w < wave ? r : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            if (cn[k] != 0u) {
                const uint32_t c = tid * per + k;
                roff[orr] = oc;
                // record f of this run is seg[base P + c P + start + f - oc]
                runs[orr] = make_uint2(c * P + cs[k] - oc, (base + c) * P);
                oc += cn[k];
                ++orr;
            }
        }
        if (tid == 0) roff[nruns] = total;
        const uint64_t* seg = v.seg + static_cast<uint64_t>(base) * P;
        for (uint32_t s0 = 0; s0 < total; s0 += kSeg) {
            const uint32_t len = min(kSeg, total - s0);
            const uint32_t words = ((len + 63u) >> 6) * 2u;
            __syncthreads();  // runs written / previous segment done with the bitmap
            for (uint32_t q = tid; q < words; q += NT) bits[q] = 0u;
            __syncthreads();
            for (uint32_t k = tid; k < nruns; k += NT) {
                const uint32_t pos = roff[k] - s0;
                if (pos < len) atomicOr(&bits[pos >> 5], 1u << (pos & 31u));
            }
            __syncthreads();
            const uint32_t nwin = (len + 63u) >> 6;
            const uint32_t r0 = s0 + (nwin * wave / kWaves) * 64u;
            const uint32_t r1 = s0 + min(len, (nwin * (wave + 1u) / kWaves) * 64u);
            // windows in flight per lane: 12 for the few dense tiles of one view;
            // 6 for the many small batched tiles, whose workgroups gain more from
            // sharing a CU (72 VGPRs, six a CU: 0.92 against 0.96 ms per batch frame)
            if (r0 < r1)
                splat_segment<S, Sh::kWindows>(seg, keys, roff, runs,
                                               reinterpret_cast<const uint64_t*>(bits), nruns, s0, r0, r1);
        }
    }
    __syncthreads();
    if constexpr (RESOLVE) {
        const uint32_t x0 = (t % v.tiles_x) << SHIFT, y0 = (t / v.tiles_x) << SHIFT;
        const uint32_t wt = min(S, v.width - x0), ht = min(S, v.height - y0);
        uint32_t* out = v.colour + static_cast<uint64_t>(y0) * v.width + x0;
        for (uint32_t q = tid; q < S * S; q += NT) {
            const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
            if (lx < wt && ly < ht)
                out[static_cast<uint64_t>(ly) * v.width + lx] =
                    pixel_colour(keys[q], v.seed_lo, v.seed_hi, v.pal);
        }
        if (v.hint) {  // the tile's winners, the next frame's occlusion hints
            uint32_t* h = v.hint + static_cast<uint64_t>(t) * (S * S);
            for (uint32_t q = tid; q < S * S; q += NT)
                h[q] = keys[q] == kEmptyKey ? kNoHint : static_cast<uint32_t>(keys[q]);
        }
    } else {
        write_part<FOOT, S, A, NT>(keys, v.part + static_cast<uint64_t>(piece) * (A * A));
    }
    __syncthreads();
}

// Split z of tile t: bin workgroups [num_wg * z / splits, num_wg * (z + 1) /
// splits), partial block t * splits + z.
template <int FOOT, int SHIFT, uint32_t NT = kTileThreads>
__device__ __forceinline__ void tile_split(const TileView& v, uint32_t t, uint32_t z, uint32_t P,
                                           uint64_t* keys, uint32_t* col) {
    const uint32_t w_lo = static_cast<uint32_t>(static_cast<uint64_t>(v.num_wg) * z / v.splits);
    const uint32_t w_hi = static_cast<uint32_t>(static_cast<uint64_t>(v.num_wg) * (z + 1) / v.splits);
    tile_range<FOOT, SHIFT, NT>(v, t, w_lo, w_hi, t * v.splits + z, P, keys, col);
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(kTileThreads) void tile_kernel(TileArgs a) {
    using Sh = TileShape<FOOT, SHIFT>;
    __shared__ uint64_t keys[Sh::S * Sh::S];
    __shared__ uint32_t col[Sh::kColLds];
    uint32_t t, z;
    tile_of_block(blockIdx.x, a.v.splits, t, z);
    if (t >= a.v.ntiles) return;
    if (tile_flag(a.v, t) != *a.stamp_in) return;  // nothing to draw
    tile_split<FOOT, SHIFT>(a.v, t, z, a.points_per_wg, keys, col);
}

// One workgroup per tile for the 1x1 footprint: the tile's whole column,
// resolved to RGBA8 in place (no partial blocks, no merge pass). 1024 threads
// give a dense tile the issue rate that two workgroups of a split would. A
// tile with nothing to draw is cleared if the previous frame drew it (or
// every frame, with full_clear), as the merge pass does.
constexpr uint32_t kFusedThreads = 1024;

template <int SHIFT>
__global__ __launch_bounds__(kFusedThreads) void tile_fused_kernel(TileArgs a) {
    using Sh = TileShape<1, SHIFT, kFusedThreads>;
    constexpr uint32_t S = Sh::S;
    __shared__ uint64_t keys[S * S];
    __shared__ uint32_t col[Sh::kColLds];
    uint32_t t, z;
    tile_of_block(blockIdx.x, 1u, t, z);
    if (t >= a.v.ntiles) return;
    if (a.v.cull) {  // read by this frame's bin pass; the next frame's hint kernel adds to it
        uint32_t* rec = a.v.cull + static_cast<uint64_t>(t) * cull_words(S);
        for (uint32_t w = threadIdx.x; w < cull_words(S); w += kFusedThreads) rec[w] = 0u;
    }
    const uint32_t stamp = *a.stamp_in, flag = tile_flag(a.v, t);
    if (flag != stamp) {
        if (flag == stamp - 1u || (a.v.prev_stamp != 0u && flag == a.v.prev_stamp) || a.v.full_clear) {
            clear_tile<SHIFT>(a.v, t, threadIdx.x, kFusedThreads);
            if (a.v.hint)  // no winners now: no hints for the next frame
                for (uint32_t q = threadIdx.x; q < S * S; q += kFusedThreads)
                    a.v.hint[static_cast<uint64_t>(t) * (S * S) + q] = kNoHint;
        }
        return;
    }
    tile_range<1, SHIFT, kFusedThreads, true>(a.v, t, 0u, a.v.num_wg, t, a.points_per_wg, keys, col);
}

// Load-balanced tile pass. The transpose kernel copies the table tile-major
// and sums every tile's records over all bin workgroups; the plan kernel cuts
// every tile into pieces of about piece_records records (ranges of bin
// workgroups of equal length), lays the pieces out tile by tile (piece_first)
// and lists them as work items; a persistent grid of tile workgroups takes
// items from a counter, so dense tiles spread over many CUs and no workgroup
// is launched for an empty tile. With the tile-major copy a piece reads its
// tile's entries as two contiguous runs instead of one 128-byte line per bin
// workgroup: the column gather of a row-major table fetches lines that the
// 64 tiles sharing them read at different times, long after L2 has let them go.

// Tile-major rows are whole 128-byte lines apart.
constexpr uint32_t kTcolAlign = 64;
// Table rows (bin workgroups) per transpose workgroup, and rows of loads each
// wave keeps in flight.
constexpr uint32_t kTransRows = 256;
constexpr uint32_t kTransBatch = 32;

// One workgroup per (column group, row group), 256 threads. A table row is
// ntiles + 1 entries long, so a 64-column span mostly straddles two lines
// that the neighbouring column groups share: block b runs on XCD b mod 8, and
// blocks b, b + 8, b + 16, ... take column groups 0, 1, 2, ... of one row
// group, reading the shared lines into one L2 at about the same time. The
// workgroup stages table columns [t0, t0 + 64) of rows [c0, c0 + kTransRows)
// in LDS (each row read as one 128-byte span), writes tile-major rows t0 ..
// t0 + 63 of those entries (a thread 4 consecutive entries), and adds each
// column's sum over its rows to col_sum. Tile t's records over all bin
// workgroups are col_sum[t + 1] - col_sum[t] (the table rows are exclusive
// scans), exact in 32-bit wrap-around arithmetic.
__global__ __launch_bounds__(256) void transpose_kernel(TileArgs a) {
    __shared__ uint16_t s[kTransRows][65];
    __shared__ uint32_t part[4][64];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t cols_total = a.v.ntiles + 1u;
    const uint32_t groups = (cols_total + 63u) / 64u;
    const uint32_t k = blockIdx.x >> 3;
    const uint32_t rg = (k / groups) * 8u + (blockIdx.x & 7u);
    if (rg * kTransRows >= a.v.num_wg) return;
    const uint32_t t0 = (k % groups) * 64u, c0 = rg * kTransRows;
    const uint32_t rows = min(kTransRows, a.v.num_wg - c0);
    const uint32_t cols = min(64u, cols_total - t0);  // columns staged: t0 .. t0 + cols - 1
    const uint32_t col = min(lane, cols - 1u);
    // wave w stages rows [32 w, 32 w + 32), [32 w + 128, ...); rows past the
    // end repeat the last one and count nothing
    uint32_t acc = 0;
    for (uint32_t r0 = wave * kTransBatch; r0 < rows; r0 += 4u * kTransBatch) {
        uint32_t x[kTransBatch];
#pragma unroll
        for (uint32_t u = 0; u < kTransBatch; ++u)
            x[u] = a.v.table[static_cast<uint64_t>(c0 + min(r0 + u, rows - 1u)) * cols_total + t0 + col];
#pragma unroll
        for (uint32_t u = 0; u < kTransBatch; ++u) {
            if (r0 + u < rows) {
                s[r0 + u][lane] = static_cast<uint16_t>(x[u]);
                acc += x[u];
            }
        }
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0u && lane < cols)
        atomicAdd(&a.col_sum[t0 + lane], part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
    // tile-major rows t0 + j: thread (j mod 4 = wave, lane) writes entries
    // 4 lane .. 4 lane + 3 of the workgroup's rows
    const uint32_t stride = a.v.tcol_stride;
    const uint32_t r = 4u * lane;
    for (uint32_t j = wave; j < cols; j += 4u) {
        uint16_t* dst = a.tcol + static_cast<uint64_t>(t0 + j) * stride + c0 + r;
        if (r + 3u < rows) {
            const uint64_t w4 = static_cast<uint64_t>(s[r][j]) |
                                (static_cast<uint64_t>(s[r + 1u][j]) << 16) |
                                (static_cast<uint64_t>(s[r + 2u][j]) << 32) |
                                (static_cast<uint64_t>(s[r + 3u][j]) << 48);
            *reinterpret_cast<uint64_t*>(dst) = w4;
        } else {
            for (uint32_t q = 0; r + q < rows; ++q) dst[q] = s[r + q][j];
        }
    }
}

// One workgroup of 1024 threads: pieces per tile, their exclusive scan
// (piece_first), the work items, the item count; resets the work counter and
// the column sums for the next frame.
__global__ __launch_bounds__(1024) void plan_kernel(TileArgs a) {
    __shared__ uint32_t pieces[kMaxPlanTiles + 1];
    __shared__ uint32_t wave_sum[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nt = a.v.ntiles;
    for (uint32_t t = tid; t < nt; t += 1024u) {
        const uint32_t total = a.col_sum[t + 1u] - a.col_sum[t];
        pieces[t] = (total + a.piece_records - 1) / a.piece_records;
    }
    __syncthreads();  // every sum read before any is reset
    for (uint32_t t = tid; t <= nt; t += 1024u) a.col_sum[t] = 0u;
    // exclusive scan of pieces[0..nt): each wave a contiguous run of 64-blocks
    const uint32_t nblk = (nt + 63u) / 64u, per = (nblk + 15u) / 16u;
    const uint32_t b0 = min(nblk, wave * per), b1 = min(nblk, b0 + per);
    uint32_t lsum = 0;
    for (uint32_t b = b0; b < b1; ++b) lsum += b * 64u + lane < nt ? pieces[b * 64u + lane] : 0u;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(lsum, d, 64);
        if (lane >= d) lsum += u;
    }
    if (lane == 63) wave_sum[wave] = lsum;
    __syncthreads();
    uint32_t carry = 0, total = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        carry += w < wave ? wave_sum[w] : 0u;
        total += wave_sum[w];
    }
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t i = b * 64u + lane;
        const uint32_t v = i < nt ? pieces[i] : 0u;
        uint32_t inc = v;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        if (i < nt) {
            const uint32_t first = carry + inc - v;
            a.piece_first[i] = first;
            for (uint32_t j = 0; j < v; ++j) a.items[first + j] = make_uint2(i, (j << 16) | v);
        }
        carry += __shfl(inc, 63, 64);
    }
    if (tid == 0) {
        a.piece_first[nt] = total;
        a.counters[0] = 0u;      // next item to take
        a.counters[1] = total;   // items this frame
    }
}

// Persistent grid: each workgroup takes items (tile, piece j of k) until the
// list is done; piece j covers bin workgroups [num_wg * j / k, num_wg * (j + 1) / k).
template <int FOOT, int SHIFT>
__global__ __launch_bounds__(kTileThreads) void tile_list_kernel(TileArgs a) {
    using Sh = TileShape<FOOT, SHIFT>;
    __shared__ uint64_t keys[Sh::S * Sh::S];
    __shared__ uint32_t col[Sh::kColLds];
    __shared__ uint32_t next;
    const uint32_t n_items = __hip_atomic_load(&a.counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&a.counters[0], 1u);
        __syncthreads();
        const uint32_t it = next;
        __syncthreads();  // every thread has read `next` before it is written again
        if (it >= n_items) break;
        const uint2 item = a.items[it];
        const uint32_t t = item.x, j = item.y >> 16, k = item.y & 0xFFFFu;
        const uint32_t w_lo = static_cast<uint32_t>(static_cast<uint64_t>(a.v.num_wg) * j / k);
        const uint32_t w_hi = static_cast<uint32_t>(static_cast<uint64_t>(a.v.num_wg) * (j + 1) / k);
        tile_range<FOOT, SHIFT>(a.v, t, w_lo, w_hi, a.v.piece_first[t] + j, a.points_per_wg, keys, col);
    }
}

// Threads of a batched tile workgroup: the batch's tiles are many and small
// (about 1,700 records each for 64 clouds and 156 views), so smaller
// workgroups, more of them per CU, spend less on barriers and overlap more of
// each other's table reads (1.229 ms per batch frame against 1.244 ms with
// 512 threads).
constexpr uint32_t kBatchThreads = 256;

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(kBatchThreads) void batch_tile_kernel(BatchTileArgs a) {
    using Sh = TileShape<FOOT, SHIFT, kBatchThreads>;
    __shared__ uint64_t keys[Sh::S * Sh::S];
    __shared__ uint32_t col[Sh::kColLds];
    const uint32_t stamp = *a.stamp_in;
    for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.item[it]);
        if (item.x == kPadItem) continue;
        const TileView v = load_uniform(&a.views[item.x]);
        const uint32_t t = item.y >> 3, z = item.y & 7u;
        // 1x1 footprint with one split: the tile is resolved here (its view
        // has no merge items), so a tile not drawn is cleared here too
        const bool resolve = FOOT == 1 && v.splits == 1u;
        const uint32_t flag = tile_flag(v, t);
        if (flag != stamp) {
            if (resolve && (flag == stamp - 1u || (v.prev_stamp != 0u && flag == v.prev_stamp) ||
                            v.full_clear))
                clear_tile<SHIFT>(v, t, threadIdx.x, kBatchThreads);
            continue;
        }
        if constexpr (FOOT == 1) {
            if (resolve) {
                tile_range<1, SHIFT, kBatchThreads, true>(v, t, 0u, v.num_wg, t, a.points_per_wg, keys,
                                                          col);
                continue;
            }
        }
        tile_split<FOOT, SHIFT, kBatchThreads>(v, t, z, a.points_per_wg, keys, col);
    }
}

// Tile t: the minimum of the splits' partial keys, then RGBA8 (edge keys and
// the apron of 3x3 footprints go to the seam pass). A tile with nothing to
// draw is cleared if the previous frame drew it; otherwise its pixels are
// already 0. 256 threads; workgroup g of G takes pixels (and apron keys) q
// with q / 256 = g mod G, so a tile of many pieces is merged by several CUs.
template <int FOOT, int SHIFT>
__device__ __forceinline__ void merge_tile(const TileView& v, uint32_t t, uint32_t stamp,
                                           uint32_t g, uint32_t G) {
    constexpr uint32_t S = 1u << SHIFT;
    constexpr uint32_t A = FOOT == 3 ? S + 2 : S;
    const uint32_t tid = threadIdx.x + 256u * g, step = 256u * G;
    const uint32_t tx = t % v.tiles_x, ty = t / v.tiles_x;
    const uint32_t x0 = tx << SHIFT, y0 = ty << SHIFT;
    const uint32_t wt = min(S, v.width - x0), ht = min(S, v.height - y0);
    uint32_t* out = v.colour + static_cast<uint64_t>(y0) * v.width + x0;
    const uint32_t flag = tile_flag(v, t);
    if (flag != stamp) {
        if (flag == stamp - 1u || (v.prev_stamp != 0u && flag == v.prev_stamp) || v.full_clear)
            clear_tile<SHIFT>(v, t, tid, step);
        return;
    }
    // the tile's partial blocks: its pieces, or its `splits` static splits
    const uint32_t first = v.piece_first ? v.piece_first[t] : t * v.splits;
    const uint32_t count = v.piece_first ? v.piece_first[t + 1] - first : v.splits;
    const uint64_t* part = v.part + static_cast<uint64_t>(first) * (A * A);
    // eight partial blocks per round in flight: a tile balanced by load can
    // have tens of pieces
    auto key_at = [&](uint32_t q) {
        uint64_t k = kEmptyKey;
        uint32_t z = 0;
        for (; z + 8 <= count; z += 8) {
            uint64_t p[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) p[u] = part[static_cast<uint64_t>(z + u) * (A * A) + q];
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) k = p[u] < k ? p[u] : k;
        }
        for (; z < count; ++z) {
            const uint64_t p = part[static_cast<uint64_t>(z) * (A * A) + q];
            k = p < k ? p : k;
        }
        return k;
    };
    for (uint32_t q = tid; q < S * S; q += step) {
        const uint32_t lx = q & (S - 1u), ly = q >> SHIFT;
        if (lx >= wt || ly >= ht) continue;
        if constexpr (FOOT == 1) {
            out[static_cast<uint64_t>(ly) * v.width + lx] = pixel_colour(key_at(q), v.seed_lo, v.seed_hi, v.pal);
        } else {
            const uint64_t k = key_at((ly + 1) * A + lx + 1);
            if (lx == 0 || ly == 0 || lx == S - 1 || ly == S - 1) {
                uint64_t* bd = v.border + static_cast<uint64_t>(t) * (4 * S);
                if (ly == 0) bd[lx] = k;
                if (ly == S - 1) bd[S + lx] = k;
                if (lx == 0) bd[2 * S + ly] = k;
                if (lx == S - 1) bd[3 * S + ly] = k;
            } else {
                out[static_cast<uint64_t>(ly) * v.width + lx] = pixel_colour(k, v.seed_lo, v.seed_hi, v.pal);
            }
        }
    }
    if constexpr (FOOT == 3) {
        uint64_t* ap = v.apron + static_cast<uint64_t>(t) * (4 * S + 4);
        for (uint32_t q = tid; q < 4 * S + 4; q += step) {
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
    merge_tile<FOOT, SHIFT>(a.v, t, *a.stamp_in, blockIdx.y, gridDim.y);
}

template <int FOOT, int SHIFT>
__global__ __launch_bounds__(256) void batch_merge_kernel(BatchTileArgs a) {
    const uint32_t stamp = *a.stamp_in;
    for (uint32_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const uint2 item = load_uniform(&a.item[it]);
        if (item.x == kPadItem) continue;
        const TileView v = load_uniform(&a.views[item.x]);
        merge_tile<FOOT, SHIFT>(v, item.y >> 3, stamp, 0u, 1u);
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
        out[static_cast<uint64_t>(ly) * v.width + lx] = pixel_colour(k, v.seed_lo, v.seed_hi, v.pal);
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

Launch tile_launch(int footprint, int shift, uint32_t ntiles, uint32_t splits) {
    Launch l;
    l.func = footprint == 3 ? pick_tile<3>(shift, false) : pick_tile<1>(shift, false);
    l.block = dim3(kTileThreads);
    l.grid = dim3((ntiles + 511u) / 512u * 512u * splits);  // whole runs of 8 XCDs x 64 tiles
    l.shared = 0;
    return l;
}

Launch tile_fused_launch(int shift, uint32_t ntiles) {
    Launch l;
    switch (shift) {
        case 4: l.func = reinterpret_cast<const void*>(&tile_fused_kernel<4>); break;
        case 5: l.func = reinterpret_cast<const void*>(&tile_fused_kernel<5>); break;
        default: l.func = reinterpret_cast<const void*>(&tile_fused_kernel<6>); break;
    }
    l.block = dim3(kFusedThreads);
    l.grid = dim3((ntiles + 511u) / 512u * 512u);  // whole runs of 8 XCDs x 64 tiles
    l.shared = 0;
    return l;
}

Launch merge_launch(int footprint, int shift, uint32_t ntiles) {
    Launch l;
    l.func = footprint == 3 ? pick_merge<3>(shift, false) : pick_merge<1>(shift, false);
    l.block = dim3(256);
    // workgroups per tile: about 1024 pixels each
    l.grid = dim3(ntiles, shift == 6 ? 4u : 1u);
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

uint32_t tcol_stride(uint32_t num_wg) {
    return (num_wg + kTcolAlign - 1u) / kTcolAlign * kTcolAlign;
}

Launch transpose_launch(uint32_t ntiles, uint32_t num_wg) {
    Launch l;
    l.func = reinterpret_cast<const void*>(&transpose_kernel);
    l.block = dim3(256);
    const uint32_t groups = (ntiles + 1u + 63u) / 64u;
    const uint32_t row_groups = (num_wg + kTransRows - 1u) / kTransRows;
    l.grid = dim3(groups * ((row_groups + 7u) / 8u * 8u));  // row groups padded to 8
    l.shared = 0;
    return l;
}

Launch plan_launch() {
    Launch l;
    l.func = reinterpret_cast<const void*>(&plan_kernel);
    l.block = dim3(1024);
    l.grid = dim3(1);
    l.shared = 0;
    return l;
}

template <int FOOT>
const void* pick_tile_list(int shift) {
    switch (shift) {
        case 4: return reinterpret_cast<const void*>(&tile_list_kernel<FOOT, 4>);
        case 5: return reinterpret_cast<const void*>(&tile_list_kernel<FOOT, 5>);
        default: return reinterpret_cast<const void*>(&tile_list_kernel<FOOT, 6>);
    }
}

Launch tile_list_launch(int footprint, int shift, uint32_t grid_blocks) {
    Launch l;
    l.func = footprint == 3 ? pick_tile_list<3>(shift) : pick_tile_list<1>(shift);
    l.block = dim3(kTileThreads);
    l.grid = dim3(grid_blocks);
    l.shared = 0;
    return l;
}

Launch batch_tile_launch(int footprint, int shift, uint32_t items, uint32_t grid_blocks) {
    Launch l;
    l.func = footprint == 3 ? pick_tile<3>(shift, true) : pick_tile<1>(shift, true);
    l.block = dim3(kBatchThreads);
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
