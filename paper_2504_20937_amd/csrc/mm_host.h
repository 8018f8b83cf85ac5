// Host-side pieces shared by the C ABI translation units: the handle
// structs of instances and allocations, error reporting, and the mapping of
// public descriptions onto kernel argument blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>
#include <set>
#include <string>

#include "mm.h"
#include "mm_internal.h"

struct mm_alloc_s {
    mm_instance inst;
    void* ptr;
    size_t bytes;
    bool owned;
    uint32_t users;  // views, batches and servers referring to it
};

struct mm_instance_s {
    int device;
    hipStream_t stream;
    bool owns_stream;
    std::set<mm_alloc> allocs;
    std::set<mm_view> views;
    std::set<mm_batch> batches;
    std::set<mm_server> servers;
    std::set<mm_grid> grids;
    std::set<mm_edges> edges;
    // compute sections (mm_prepare_views / mm_update_views), created on first use
    hipEvent_t prep_ev = nullptr;
    hipEvent_t upd_ev = nullptr;
};

namespace mmh {

// Sets the thread-local message of mm_last_error and returns st.
mm_status fail(mm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

inline mm_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? MM_ERR_OUT_OF_MEMORY : MM_ERR_HIP, "%s failed: %s",
                what, hipGetErrorString(e));
}

#define MM_HIP(call)                                                                        \
    do {                                                                                    \
        const hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                               \
            return ::mmh::fail(e_ == hipErrorOutOfMemory ? MM_ERR_OUT_OF_MEMORY : MM_ERR_HIP, \
                               "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                               __FILE__, __LINE__);                                         \
    } while (0)

#define MM_TRY(expr)                       \
    do {                                   \
        const mm_status s_ = (expr);       \
        if (s_ != MM_OK) return s_;        \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;
};

inline bool amplitude_ok(float a) {
    return a == 0.0f || (std::isfinite(a) && a >= 0x1p-64f && a <= 0x1p64f);
}

inline uint32_t shift_of(uint32_t side) {
    return side == 16 ? 4u : side == 32 ? 5u : side == 64 ? 6u : 0u;
}

inline uint32_t tiles_of(uint32_t width, uint32_t height, uint32_t side) {
    return ((width + side - 1) / side) * ((height + side - 1) / side);
}

// Largest tile table a bin workgroup holds in LDS.
constexpr uint32_t kMaxTiles = 4096;

inline void set_camera_rows(mm::ViewGeom& g, const float m[16]) {
    const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) g.m[4 * r + c] = m[4 * rows[r] + c];
}

inline mm::CloudArgs cloud_args(void* pos, uint64_t n, uint64_t seed, float amp) {
    mm::CloudArgs c{};
    c.pos = static_cast<float*>(pos);
    c.n = static_cast<uint32_t>(n);
    c.seed_lo = static_cast<uint32_t>(seed);
    c.seed_hi = static_cast<uint32_t>(seed >> 32);
    c.step = 0;
    c.amp = amp;
    c.fold_lim = std::numeric_limits<float>::infinity();
    return c;
}

inline mm::ViewGeom view_geom(uint32_t width, uint32_t height, const float m[16]) {
    mm::ViewGeom g{};
    g.width = width;
    g.height = height;
    g.half_w = static_cast<float>(width / 2u);
    g.half_h = static_cast<float>(height / 2u);
    g.fwidth = static_cast<float>(width);
    g.fheight = static_cast<float>(height);
    set_camera_rows(g, m);
    return g;
}

inline hipKernelNodeParams node_params(const mm::Launch& l, void** args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(l.func);
    p.gridDim = l.grid;
    p.blockDim = l.block;
    p.sharedMemBytes = l.shared;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

inline hipError_t launch(const mm::Launch& l, void* arg, hipStream_t s) {
    if (l.grid.x == 0) return hipSuccess;
    void* args[] = {arg};
    return hipLaunchKernel(l.func, l.grid, l.block, args, l.shared, s);
}

// Every device and pinned host allocation of the library goes through these,
// so that a test can make one of them fail (mm_debug_fail_allocations).
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t pinned_malloc(void** p, size_t bytes);

template <typename T>
hipError_t alloc_n(T** p, uint64_t n) {
    return dev_malloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T));
}

// Checks a cloud: format, count against its alloc, amplitude and wrap.
mm_status validate_cloud(mm_instance inst, const mm_cloud_desc& c, mm_domain domain,
                         const char* what);

// Checks a screen size: even, in [2, 16384].
mm_status validate_screen(uint32_t width, uint32_t height, const char* what);

mm_status validate_camera(const float m[16], const char* what);

}  // namespace mmh

namespace mmh {

// Autotuning cache: a text file named by the environment variable
// MM_TUNE_CACHE, one "key v0 .. v6" line per tuned shape; later lines win.
// Without the variable nothing is read or written.
constexpr int kTuneValues = 7;
bool tune_cache_lookup(const std::string& key, uint32_t out[kTuneValues]);
void tune_cache_store(const std::string& key, const uint32_t v[kTuneValues]);
// gcnArchName of a device (e.g. "gfx950:sramecc+:xnack-"), "" on failure.
std::string device_arch(int device);

// Mean time per call of fn over `frames` calls after one warm-up call, from
// HIP events on stream s; negative on error.
template <typename F>
float time_frames(hipStream_t s, uint32_t frames, F fn) {
    hipEvent_t a = nullptr, b = nullptr;
    // timing only: no system-scope fence per event
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return -1.0f;
    if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.0f;
    }
    float ms = -1.0f;
    bool ok = fn() == MM_OK && hipEventRecord(a, s) == hipSuccess;
    for (uint32_t k = 0; ok && k < frames; ++k) ok = fn() == MM_OK;
    if (ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
        hipEventElapsedTime(&ms, a, b) == hipSuccess)
        ms /= static_cast<float>(frames);
    else
        ms = -1.0f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

}  // namespace mmh
