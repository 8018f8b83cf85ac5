// A frame that allocates nothing (mm_step_render_static): the direct
// splat's displace + project + atomicMin pass and its resolve, on the
// caller's positions, frame and stream, with the per-pixel depth keys in a
// file-scope device array instead of memory the library allocates.
//
// The keys must be empty (kEmptyKey) when a frame starts. The resolve leaves
// every key it reads empty again, so once the array has been filled with
// empty keys (the first call on a device, and any call after a launch that
// failed), each completed call leaves it ready for the next. Calls on one
// device share the array: calls that overlap on a device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "mm_host.h"

namespace {

// Largest screen of a call: 2^22 pixels (up to 2048 x 2048), 32 MiB of keys
// held by every device the library runs on until the process ends.
constexpr uint64_t kStaticMaxPixels = 1ull << 22;

// The depth keys. In host code this name is a host-side stand-in, not a
// device address: kernels take the address hipGetSymbolAddress returns for
// the current device (StaticKeys::ptr).
static __device__ __align__(256) uint64_t scratch[kStaticMaxPixels];

struct StaticKeys {
    uint64_t* ptr = nullptr;  // this device's copy of `scratch`
    bool empty = false;       // every key holds kEmptyKey
};

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
StaticKeys g_static[kMaxDevices];

}  // namespace

using namespace mmh;

extern "C" {

mm_status mm_step_render_static(const mm_static_frame_desc* d) {
    if (!d || !d->dev_positions || !d->dev_rgba)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: null argument");
    if (d->domain != MM_DOMAIN_2D && d->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: domain %d is not 2D/3D", (int)d->domain);
    if (d->element_count < 1 || d->element_count > 0xFFFFFFFFull)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: element_count %llu outside [1, 2^32-1]",
                    (unsigned long long)d->element_count);
    MM_TRY(validate_screen(d->width, d->height, "step_render_static"));
    const uint64_t npix = static_cast<uint64_t>(d->width) * d->height;
    if (npix > kStaticMaxPixels)
        return fail(MM_ERR_BUDGET, "step_render_static: %ux%u is %llu pixels, more than the %llu the "
                    "static key array holds", d->width, d->height, (unsigned long long)npix,
                    (unsigned long long)kStaticMaxPixels);
    if (d->footprint != 1 && d->footprint != 3)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: footprint %u is not 1 or 3", d->footprint);
    if (!amplitude_ok(d->amplitude))
        return fail(MM_ERR_INVALID_ARG, "step_render_static: amplitude %g outside {0} U [2^-64, 2^64]",
                    (double)d->amplitude);
    if (d->wrap != 0 && d->wrap != 1)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: wrap must be 0 or 1");
    if (d->wrap && d->amplitude > 1.0f)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: wrap needs amplitude <= 1");
    if (d->domain == MM_DOMAIN_3D) MM_TRY(validate_camera(d->view_proj, "step_render_static"));
    if (reinterpret_cast<uintptr_t>(d->dev_positions) % 4 != 0 ||
        reinterpret_cast<uintptr_t>(d->dev_rgba) % 4 != 0)
        return fail(MM_ERR_INVALID_ARG, "step_render_static: device pointers must be 4-byte aligned");
    int dev = 0;
    MM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MM_ERR_UNSUPPORTED, "step_render_static: device %d", dev);
    hipStream_t s = static_cast<hipStream_t>(d->stream);

    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticKeys& k = g_static[dev];
    if (!k.ptr) {  // once per device, with the device current
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MM_ERR_HIP, "step_render_static: hipGetSymbolAddress failed: %s",
                        hipGetErrorString(e));
        }
        k.ptr = static_cast<uint64_t*>(p);
        k.empty = false;
    }
    if (!k.empty) {
        const hipError_t e = mm::launch_fill(k.ptr, kStaticMaxPixels, mm::kEmptyKey, s);
        if (e != hipSuccess) return hip_fail(e, "step_render_static: clearing the keys");
        k.empty = true;
    }
    mm::PointArgs a{};
    a.c = cloud_args(d->dev_positions, d->element_count, d->seed, d->amplitude);
    a.c.step = d->step;
    a.g = view_geom(d->width, d->height, d->view_proj);
    a.depth = k.ptr;
    const int dim = static_cast<int>(d->domain), foot = static_cast<int>(d->footprint);
    hipError_t e = mm::launch_point(a, dim, foot, d->wrap != 0, mm::kDisplaceRender, s);
    if (e == hipSuccess) {
        const mm::ResolveArgs r{k.ptr, d->dev_rgba, npix, a.c.seed_lo, a.c.seed_hi, mm::Palette{}};
        e = mm::launch_resolve(r, s);
    }
    if (e != hipSuccess) {
        k.empty = false;  // the keys may hold a partial frame: fill them again next time
        return hip_fail(e, "step_render_static: launch");
    }
    return MM_OK;
}

}  // extern "C"
