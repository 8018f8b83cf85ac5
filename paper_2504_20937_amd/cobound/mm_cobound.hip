// Integer/FP32 ALU co-bound of the bin pass: the per-point arithmetic of a
// frame (the Philox4x32-10 draw; the draw, the displacement and the
// projection) timed without the position traffic. The launch has the shape of
// the plain bin kernel at its default tuning (1024-thread workgroups, 8
// points per thread); each thread folds its results into one 4-byte store so
// the compiler keeps all of the work. A kernel with only the index arithmetic
// and that store gives the launch and store overhead.
//
//   mm_cobound [log2 points = 24] [launches = 50]
//
// prints one JSON line with the mean time per launch of each probe.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

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
    uint32_t probe = 0;
    CHECK(hipMemcpy(&probe, out, sizeof probe, hipMemcpyDeviceToHost));
    std::printf("{\"points\": %u, \"threads\": %u, \"points_per_thread\": %d, \"launches\": %d",
                c.n, kThreads, kPpt, launches);
    for (int k = 0; k < 3; ++k) std::printf(", \"%s\": %.2f", names[k], us[k]);
    std::printf(", \"check\": %u}\n", probe);
    CHECK(hipFree(out));
    return 0;
}
