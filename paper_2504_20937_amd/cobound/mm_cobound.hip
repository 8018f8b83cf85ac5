// Co-bounds of the two passes of a binned frame, each timed without the rest
// of the frame.
//
// Bin pass (integer/FP32 ALU): the per-point arithmetic of a frame (the
// Philox4x32-10 draw; the draw, the displacement and the projection) without
// the position traffic. The launch has the shape of the plain bin kernel at
// its default tuning (1024-thread workgroups, 8 points per thread); each
// thread folds its results into one 4-byte store so the compiler keeps all of
// the work. A kernel with only the index arithmetic and that store gives the
// launch and store overhead.
//
// Bin pass (memory): the same launch moving only the bin kernel's bytes per
// point, with its access kinds: the position read and written in place
// (12-byte non-temporal accesses) and an 8-byte record write, coalesced,
// with no arithmetic and no sort; what the HBM traffic of the pass costs by
// itself (the table row, 1.5% of the bytes at 1080p, is left out).
//
// Tile pass (one CU's record stream): a dense tile is taken by one 1024-thread
// workgroup on one CU, which streams the tile's 8-byte records in 64-record
// windows per wave. The stream probe runs one such workgroup per CU (dynamic
// LDS keeps a second one off the CU), each reading its own contiguous range
// of 8-byte words with U windows in flight per lane and no other work, and
// stores the device clock at each workgroup's start and end. Workgroup 0 can
// take a longer range (the heaviest tile) than the others (the mean tile).
// Last, every workgroup reads the heaviest tile's words contiguously, and as
// the tile pass meets them: short runs at scattered, misaligned offsets.
//
//   mm_cobound [log2 points = 24] [launches = 50]
//
// prints one JSON line with the mean time per launch of each probe.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mm_device.h"

namespace {

using namespace mm;
using namespace mm::dev;

constexpr uint32_t kThreads = 1024;
constexpr int kPpt = 8;

__global__ __launch_bounds__(kThreads) void index_probe(uint32_t* out, uint32_t salt) {
    const uint32_t base = blockIdx.x * (kThreads * kPpt);
    uint32_t acc = salt;
#pragma unroll
    for (int k = 0; k < kPpt; ++k) acc ^= base + k * kThreads + threadIdx.x;
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void philox_probe(uint32_t* out, CloudArgs c) {
    const uint32_t base = blockIdx.x * (kThreads * kPpt);
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kPpt; ++k) {
        const uint4 r = philox4x32_10(c.step, kTagDisplace, base + k * kThreads + threadIdx.x, 0u,
                                      c.seed_lo, c.seed_hi);
        acc ^= r.x ^ r.y ^ r.z;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// Positions synthesised from the index in [0, 1)^3, then one frame's
// displacement and projection.
__global__ __launch_bounds__(kThreads) void point_probe(uint32_t* out, CloudArgs c, ViewGeom g) {
    const uint32_t base = blockIdx.x * (kThreads * kPpt);
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kPpt; ++k) {
        const uint32_t i = base + k * kThreads + threadIdx.x;
        float x = static_cast<float>(i & 0xFFFu) * 0x1p-12f;
        float y = static_cast<float>((i >> 12) & 0xFFFu) * 0x1p-12f;
        float z = static_cast<float>(i >> 24) * 0x1p-8f;
        displace<3, false>(c, c.step, i, x, y, z);
        int32_t px, py;
        uint32_t bits;
        if (project<3>(g, x, y, z, px, py, bits))
            acc ^= bits ^ (static_cast<uint32_t>(px) << 16) ^ static_cast<uint32_t>(py);
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void traffic_probe(float* pos, uint64_t* rec) {
    const uint32_t base = blockIdx.x * (kThreads * kPpt);
    float x[kPpt], y[kPpt], z[kPpt];
#pragma unroll
    for (int k = 0; k < kPpt; ++k) load_point<3>(pos, base + k * kThreads + threadIdx.x, x[k], y[k], z[k]);
#pragma unroll
    for (int k = 0; k < kPpt; ++k) {
        const uint32_t i = base + k * kThreads + threadIdx.x;
        store_point<3>(pos, i, x[k], y[k], z[k]);
        rec[i] = (static_cast<uint64_t>(__float_as_uint(z[k])) << 32) | i;
    }
}

// The tile pass reads a tile's records as one run per bin workgroup: at
// 2^24 points and 1080p the heaviest tile's 150,000 records come in runs of
// about 73 (150,000 over 2,048 bin workgroups), each starting anywhere in
// its cache line. LAYOUT 1 reads word f of a workgroup's stream as word
// f mod kRunLen of run f / kRunLen, the runs kRunGap words apart at
// misaligned offsets; LAYOUT 2 the same with every run starting on a 1 KB
// boundary; LAYOUT 0 reads the words contiguously.
constexpr uint32_t kRunLen = 73, kRunGap = 128;

// Workgroup b reads n_b words of src from word b * stride on (n_b = heavy
// for b = 0 and mean otherwise; the layout keeps every word below
// (b + 1) * stride); slot 2 b and 2 b + 1 of clk get the device clock at its
// start and end.
template <int U, int LAYOUT>
__global__ __launch_bounds__(kThreads) void stream_probe(const uint64_t* src, uint32_t* out,
                                                         uint64_t* clk, uint32_t stride,
                                                         uint32_t mean, uint32_t heavy) {
    extern __shared__ uint32_t hold[];  // sized by the launch only: one workgroup per CU
    if (threadIdx.x == 0) clk[2 * blockIdx.x] = wall_clock64();
    const uint32_t n = blockIdx.x == 0 ? heavy : mean;
    const uint64_t* p = src + static_cast<uint64_t>(blockIdx.x) * stride;
    uint64_t acc = 0;
    for (uint32_t w = threadIdx.x; w < n; w += kThreads * U) {
        uint64_t r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = w + static_cast<uint32_t>(u) * kThreads;
            uint32_t a = i;
            if constexpr (LAYOUT != 0) {
                const uint32_t run = i / kRunLen, pos = i - run * kRunLen;
                const uint32_t off = LAYOUT == 1 ? (run * 37u) % (kRunGap - kRunLen) : 0u;
                a = run * kRunGap + off + pos;
            }
            r[u] = i < n ? p[a] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= r[u];
    }
    out[blockIdx.x * kThreads + threadIdx.x] = static_cast<uint32_t>(acc ^ (acc >> 32));
    __syncthreads();
    if (threadIdx.x == 0) clk[2 * blockIdx.x + 1] = wall_clock64();
}

#define CHECK(call)                                                                      \
    do {                                                                                 \
        const hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));       \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

}  // namespace

int main(int argc, char** argv) {
    const int log2n = argc > 1 ? std::atoi(argv[1]) : 24;
    const int launches = argc > 2 ? std::atoi(argv[2]) : 50;
    if (log2n < 13 || log2n > 30 || launches < 1 || launches > 10000) {
        std::fprintf(stderr, "usage: mm_cobound [log2 points in 13..30] [launches in 1..10000]\n");
        return 2;
    }
    const uint32_t blocks = (1u << log2n) / (kThreads * kPpt);
    uint32_t* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(uint32_t) * blocks * kThreads));
    CloudArgs c{};
    c.n = blocks * kThreads * kPpt;
    c.seed_lo = 7u;
    c.amp = 0.001f;
    c.fold_lim = 1e30f;
    ViewGeom g{};  // a perspective camera in front of the unit cube
    g.width = 1920;
    g.height = 1080;
    g.half_w = 960.0f;
    g.half_h = 540.0f;
    g.fwidth = 1920.0f;
    g.fheight = 1080.0f;
    const float m[12] = {1.2f, 0.0f, -0.3f, -0.4f, 0.0f, 1.7f, 0.0f, -0.85f, 0.2f, 0.0f, 0.9f, 2.0f};
    for (int k = 0; k < 12; ++k) g.m[k] = m[k];
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char* names[3] = {"index_store_us", "philox_us", "displace_project_us"};
    float us[3] = {0, 0, 0};
    for (int which = 0; which < 3; ++which) {
        for (int pass = 0; pass < 2; ++pass) {  // the first pass warms up
            CHECK(hipEventRecord(e0, nullptr));
            for (int it = 0; it < launches; ++it) {
                c.step = static_cast<uint32_t>(it);
                if (which == 0)
                    hipLaunchKernelGGL(index_probe, dim3(blocks), dim3(kThreads), 0, nullptr, out,
                                       static_cast<uint32_t>(it));
                else if (which == 1)
                    hipLaunchKernelGGL(philox_probe, dim3(blocks), dim3(kThreads), 0, nullptr, out, c);
                else
                    hipLaunchKernelGGL(point_probe, dim3(blocks), dim3(kThreads), 0, nullptr, out, c, g);
            }
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, nullptr));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            us[which] = 1000.0f * ms / static_cast<float>(launches);
        }
    }
    // the bin pass's bytes alone: positions in place and one record per point
    float* pos = nullptr;
    uint64_t* rec = nullptr;
    CHECK(hipMalloc(&pos, 12ull * c.n));
    CHECK(hipMalloc(&rec, 8ull * c.n));
    CHECK(hipMemset(pos, 0, 12ull * c.n));
    float traffic_us = 0.0f;
    for (int pass = 0; pass < 2; ++pass) {
        CHECK(hipEventRecord(e0, nullptr));
        for (int it = 0; it < launches; ++it)
            hipLaunchKernelGGL(traffic_probe, dim3(blocks), dim3(kThreads), 0, nullptr, pos, rec);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, nullptr));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        traffic_us = 1000.0f * ms / static_cast<float>(launches);
    }
    CHECK(hipFree(pos));
    CHECK(hipFree(rec));

    uint32_t probe = 0;
    CHECK(hipMemcpy(&probe, out, sizeof probe, hipMemcpyDeviceToHost));
    std::printf("{\"points\": %u, \"threads\": %u, \"points_per_thread\": %d, \"launches\": %d",
                c.n, kThreads, kPpt, launches);
    for (int k = 0; k < 3; ++k) std::printf(", \"%s\": %.2f", names[k], us[k]);
    std::printf(", \"check\": %u, \"traffic_us\": %.2f, \"traffic_bytes\": %llu", probe, traffic_us,
                32ull * c.n);

    // The tile pass's record stream: one workgroup per CU. The mean and
    // heaviest ranges are those of the 1x1 tile pass at 2^24 points and
    // 1920x1080 (about 65,000 and 150,000 records per active tile).
    int dev = 0, cus = 0, khz = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const uint32_t mean = 65536, heavy = 150000;
    // room for the heaviest stream in runs: every word read stays below the next workgroup's
    const uint32_t stride = (heavy + kRunLen - 1) / kRunLen * kRunGap;
    uint64_t* src = nullptr;
    uint64_t* clk = nullptr;
    uint32_t* sout = nullptr;
    CHECK(hipMalloc(&src, sizeof(uint64_t) * stride * static_cast<size_t>(cus)));
    CHECK(hipMalloc(&clk, sizeof(uint64_t) * 2 * static_cast<size_t>(cus)));
    CHECK(hipMalloc(&sout, sizeof(uint32_t) * kThreads * static_cast<size_t>(cus)));
    CHECK(hipMemset(src, 0x5a, sizeof(uint64_t) * stride * static_cast<size_t>(cus)));
    int lds_max = 0;
    CHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // of 160 KB of LDS per CU, 96 KB leave no room for a second workgroup
    const size_t hold = std::min<size_t>(96 * 1024, static_cast<size_t>(lds_max));
    std::vector<uint64_t> t(2 * static_cast<size_t>(cus));
    std::printf(", \"stream\": {\"cus\": %d, \"lds_hold\": %zu, \"mean_words\": %u, \"heavy_words\": %u",
                cus, hold, mean, heavy);
    for (int which = 0; which < 4; ++which) {
        const uint32_t hv = which & 1 ? heavy : mean;
        const int U = which < 2 ? 12 : 24;
        float ms = 0.0f;
        double first = 0.0, rest = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            CHECK(hipEventRecord(e0, nullptr));
            for (int it = 0; it < launches; ++it) {
                if (U == 12)
                    hipLaunchKernelGGL((stream_probe<12, 0>), dim3(cus), dim3(kThreads), hold, nullptr, src,
                                       sout, clk, stride, mean, hv);
                else
                    hipLaunchKernelGGL((stream_probe<24, 0>), dim3(cus), dim3(kThreads), hold, nullptr, src,
                                       sout, clk, stride, mean, hv);
            }
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, nullptr));
            CHECK(hipEventSynchronize(e1));
            CHECK(hipEventElapsedTime(&ms, e0, e1));
        }
        // workgroup durations of the last launch, in microseconds
        CHECK(hipMemcpy(t.data(), clk, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost));
        first = static_cast<double>(t[1] - t[0]) * 1000.0 / khz;
        for (int b = 1; b < cus; ++b) rest += static_cast<double>(t[2 * b + 1] - t[2 * b]) * 1000.0 / khz;
        rest /= cus - 1;
        std::printf(", \"%s_u%d\": {\"launch_us\": %.2f, \"wg0_us\": %.2f, \"wg_mean_us\": %.2f}",
                    which & 1 ? "heavy" : "even", U, 1000.0f * ms / static_cast<float>(launches), first,
                    rest);
    }
    // every workgroup the heaviest tile's words, contiguous or in runs
    const char* layouts[3] = {"contiguous", "runs", "aligned_runs"};
    std::printf(", \"layout_words\": %u", heavy);
    for (int layout = 0; layout < 3; ++layout) {
        double mean_us = 0.0;
        for (int it = 0; it < launches; ++it) {
            if (layout == 0)
                hipLaunchKernelGGL((stream_probe<12, 0>), dim3(cus), dim3(kThreads), hold, nullptr, src, sout,
                                   clk, stride, heavy, heavy);
            else if (layout == 1)
                hipLaunchKernelGGL((stream_probe<12, 1>), dim3(cus), dim3(kThreads), hold, nullptr, src, sout,
                                   clk, stride, heavy, heavy);
            else
                hipLaunchKernelGGL((stream_probe<12, 2>), dim3(cus), dim3(kThreads), hold, nullptr, src, sout,
                                   clk, stride, heavy, heavy);
            CHECK(hipGetLastError());
            CHECK(hipMemcpy(t.data(), clk, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost));
            double m = 0.0;
            for (int b = 0; b < cus; ++b) m += static_cast<double>(t[2 * b + 1] - t[2 * b]) * 1000.0 / khz;
            if (it > 0 || launches == 1) mean_us += m / cus;  // the first launch warms up
        }
        mean_us /= launches > 1 ? launches - 1 : 1;
        std::printf(", \"%s_wg_us\": %.2f", layouts[layout], mean_us);
    }
    std::printf("}}\n");
    CHECK(hipFree(src));
    CHECK(hipFree(clk));
    CHECK(hipFree(sout));
    CHECK(hipFree(out));
    return 0;
}
