// C ABI runtime: instances, allocations, views and the per-frame graph.
//
// A frame is one hipGraph: [point kernel: displace+project+splat] ->
// [resolve kernel: colour + clear]. The graph is built once per view; per
// frame only the point kernel's argument block (step, camera) is replaced
// with hipGraphExecKernelNodeSetParams before hipGraphLaunch, so a frame
// costs two host calls and no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "mm.h"
#include "mm_internal.h"

struct mm_alloc_s {
    mm_instance inst;
    void* ptr;
    size_t bytes;
    bool owned;
    uint32_t users;  // views referring to it
};

struct mm_view_s {
    mm_instance inst;
    mm_alloc position;
    mm_view_desc desc;
    uint64_t* depth = nullptr;
    uint32_t* colour = nullptr;
    mm::PointArgs args{};
    mm::ResolveArgs rargs{};
    // frame graph: plain, and a timed variant with event-record nodes
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t point_node = nullptr;
    hipGraph_t tgraph = nullptr;
    hipGraphExec_t texec = nullptr;
    hipGraphNode_t tpoint_node = nullptr;
    hipGraphNode_t tevent_node[3] = {nullptr, nullptr, nullptr};
    mm::Launch point_l{}, resolve_l{};
    // profiling ring
    std::vector<hipEvent_t> events;  // 3 per frame
    uint32_t prof_cap = 0, prof_count = 0;
    bool profiling = false;
};

struct mm_instance_s {
    int device;
    hipStream_t stream;
    bool owns_stream;
    std::set<mm_alloc> allocs;
    std::set<mm_view> views;
};

namespace {

thread_local std::string g_last_error;

mm_status fail(mm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define MM_HIP(call)                                                                        \
    do {                                                                                    \
        const hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? MM_ERR_OUT_OF_MEMORY : MM_ERR_HIP,       \
                        "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                          \
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
};

bool finite_positive_pow2_range(float a) {
    return std::isfinite(a) && a >= 0x1p-64f && a <= 0x1p64f;
}

void fill_point_args(mm_view v) {
    const mm_view_desc& d = v->desc;
    mm::PointArgs& a = v->args;
    a.pos = static_cast<float*>(v->position->ptr);
    a.depth = v->depth;
    a.n = static_cast<uint32_t>(d.element_count);
    a.width = d.width;
    a.height = d.height;
    a.half_w = static_cast<float>(d.width / 2u);
    a.half_h = static_cast<float>(d.height / 2u);
    a.fwidth = static_cast<float>(d.width);
    a.fheight = static_cast<float>(d.height);
    a.seed_lo = static_cast<uint32_t>(d.seed);
    a.seed_hi = static_cast<uint32_t>(d.seed >> 32);
    a.step = 0;
    a.amp = d.amplitude;
    const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) a.m[4 * r + c] = d.view_proj[4 * rows[r] + c];
    mm::ResolveArgs& r = v->rargs;
    r.depth = v->depth;
    r.colour = v->colour;
    r.npix = static_cast<uint64_t>(d.width) * d.height;
    r.seed_lo = a.seed_lo;
    r.seed_hi = a.seed_hi;
}

hipKernelNodeParams node_params(const mm::Launch& l, void** args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(l.func);
    p.gridDim = l.grid;
    p.blockDim = l.block;
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

// Builds the frame graph of a view. With timed set, event-record nodes
// bracket each kernel: ev0 -> point -> ev1 -> resolve -> ev2.
mm_status build_graph(mm_view v, bool timed, hipGraph_t* g_out, hipGraphExec_t* e_out,
                      hipGraphNode_t* point_out, hipGraphNode_t* ev_out) {
    hipGraph_t g = nullptr;
    MM_HIP(hipGraphCreate(&g, 0));
    void* pargs[] = {&v->args};
    void* rargs[] = {&v->rargs};
    hipKernelNodeParams pp = node_params(v->point_l, pargs);
    hipKernelNodeParams rp = node_params(v->resolve_l, rargs);
    hipGraphNode_t pn = nullptr, rn = nullptr, e0 = nullptr, e1 = nullptr, e2 = nullptr;
    hipError_t err = hipSuccess;
    if (!timed) {
        err = hipGraphAddKernelNode(&pn, g, nullptr, 0, &pp);
        if (err == hipSuccess) err = hipGraphAddKernelNode(&rn, g, &pn, 1, &rp);
    } else {
        err = hipGraphAddEventRecordNode(&e0, g, nullptr, 0, v->events[0]);
        if (err == hipSuccess) err = hipGraphAddKernelNode(&pn, g, &e0, 1, &pp);
        if (err == hipSuccess) err = hipGraphAddEventRecordNode(&e1, g, &pn, 1, v->events[1]);
        if (err == hipSuccess) err = hipGraphAddKernelNode(&rn, g, &e1, 1, &rp);
        if (err == hipSuccess) err = hipGraphAddEventRecordNode(&e2, g, &rn, 1, v->events[2]);
    }
    hipGraphExec_t e = nullptr;
    if (err == hipSuccess) err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(MM_ERR_HIP, "building the frame graph failed: %s", hipGetErrorString(err));
    }
    *g_out = g;
    *e_out = e;
    *point_out = pn;
    if (ev_out) {
        ev_out[0] = e0;
        ev_out[1] = e1;
        ev_out[2] = e2;
    }
    return MM_OK;
}

mm_status validate_desc(mm_instance inst, const mm_view_desc* d) {
    if (!d->position) return fail(MM_ERR_INVALID_ARG, "view: position alloc is null");
    if (d->position->inst != inst)
        return fail(MM_ERR_INVALID_ARG, "view: position alloc belongs to another instance");
    if (d->format != MM_FLOAT2 && d->format != MM_FLOAT3)
        return fail(MM_ERR_INVALID_ARG, "view: format %d is not MM_FLOAT2/MM_FLOAT3",
                    (int)d->format);
    if (d->domain != MM_DOMAIN_2D && d->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "view: domain %d is not 2D/3D", (int)d->domain);
    if ((int)d->format != (int)d->domain)
        return fail(MM_ERR_UNSUPPORTED, "view: format float%d with a %dD domain",
                    (int)d->format, (int)d->domain);
    if (d->element_count < 1 || d->element_count > 0xFFFFFFFFull)
        return fail(MM_ERR_INVALID_ARG, "view: element_count %llu outside [1, 2^32-1]",
                    (unsigned long long)d->element_count);
    const uint64_t stride = 4ull * (uint64_t)d->format;
    if (d->element_count > d->position->bytes / stride)
        return fail(MM_ERR_INVALID_ARG, "view: %llu points of %llu B exceed the %zu-byte alloc",
                    (unsigned long long)d->element_count, (unsigned long long)stride,
                    d->position->bytes);
    if (d->width < 2 || d->height < 2 || d->width > 16384 || d->height > 16384 ||
        (d->width & 1u) || (d->height & 1u))
        return fail(MM_ERR_INVALID_ARG, "view: screen %ux%u must be even and in [2, 16384]",
                    d->width, d->height);
    if (d->footprint != 1 && d->footprint != 3)
        return fail(MM_ERR_INVALID_ARG, "view: footprint %u is not 1 or 3", d->footprint);
    if (!(d->amplitude == 0.0f || finite_positive_pow2_range(d->amplitude)))
        return fail(MM_ERR_INVALID_ARG, "view: amplitude %g outside {0} U [2^-64, 2^64]",
                    (double)d->amplitude);
    if (d->wrap != 0 && d->wrap != 1)
        return fail(MM_ERR_INVALID_ARG, "view: wrap must be 0 or 1");
    if (d->wrap && d->amplitude > 1.0f)
        return fail(MM_ERR_INVALID_ARG, "view: wrap needs amplitude <= 1");
    if (d->domain == MM_DOMAIN_3D)
        for (int k = 0; k < 16; ++k)
            if (!std::isfinite(d->view_proj[k]))
                return fail(MM_ERR_INVALID_ARG, "view: view_proj[%d] is not finite", k);
    return MM_OK;
}

void destroy_view_resources(mm_view v) {
    if (v->exec) (void)hipGraphExecDestroy(v->exec);
    if (v->graph) (void)hipGraphDestroy(v->graph);
    if (v->texec) (void)hipGraphExecDestroy(v->texec);
    if (v->tgraph) (void)hipGraphDestroy(v->tgraph);
    for (hipEvent_t e : v->events) (void)hipEventDestroy(e);
    v->events.clear();
    if (v->depth) (void)hipFree(v->depth);
    if (v->colour) (void)hipFree(v->colour);
}

}  // namespace

extern "C" {

int32_t mm_version(void) { return 100; }

const char* mm_last_error(void) { return g_last_error.c_str(); }

const char* mm_status_string(mm_status s) {
    switch (s) {
        case MM_OK: return "MM_OK";
        case MM_ERR_INVALID_ARG: return "MM_ERR_INVALID_ARG";
        case MM_ERR_OUT_OF_MEMORY: return "MM_ERR_OUT_OF_MEMORY";
        case MM_ERR_HIP: return "MM_ERR_HIP";
        case MM_ERR_BUDGET: return "MM_ERR_BUDGET";
        case MM_ERR_IN_USE: return "MM_ERR_IN_USE";
        case MM_ERR_UNSUPPORTED: return "MM_ERR_UNSUPPORTED";
        case MM_ERR_NOT_READY: return "MM_ERR_NOT_READY";
        default: return "MM_ERR_UNKNOWN";
    }
}

mm_status mm_create_instance(const mm_instance_desc* desc, mm_instance* out) {
    if (!desc || !out) return fail(MM_ERR_INVALID_ARG, "create_instance: null argument");
    int count = 0;
    MM_HIP(hipGetDeviceCount(&count));
    if (desc->device < 0 || desc->device >= count)
        return fail(MM_ERR_INVALID_ARG, "create_instance: device %d of %d", desc->device, count);
    DeviceGuard guard(desc->device);
    hipStream_t s = static_cast<hipStream_t>(desc->stream);
    bool owns = false;
    if (!s) {
        MM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        owns = true;
    }
    mm_instance inst = new (std::nothrow) mm_instance_s{desc->device, s, owns, {}, {}};
    if (!inst) {
        if (owns) (void)hipStreamDestroy(s);
        return fail(MM_ERR_OUT_OF_MEMORY, "create_instance: host allocation");
    }
    *out = inst;
    return MM_OK;
}

mm_status mm_synchronize(mm_instance inst) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "synchronize: null instance");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    return MM_OK;
}

mm_status mm_destroy_view(mm_view v);

mm_status mm_destroy_instance(mm_instance inst) {
    if (!inst) return fail(MM_ERR_INVALID_ARG, "destroy_instance: null instance");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    std::vector<mm_view> views(inst->views.begin(), inst->views.end());
    for (mm_view v : views) mm_destroy_view(v);
    for (mm_alloc a : inst->allocs) {
        if (a->owned) (void)hipFree(a->ptr);
        delete a;
    }
    if (inst->owns_stream) (void)hipStreamDestroy(inst->stream);
    delete inst;
    return MM_OK;
}

mm_status mm_alloc_linear(mm_instance inst, size_t bytes, void** dev_ptr, mm_alloc* out) {
    if (!inst || !dev_ptr || !out) return fail(MM_ERR_INVALID_ARG, "alloc_linear: null argument");
    if (bytes == 0) return fail(MM_ERR_INVALID_ARG, "alloc_linear: zero bytes");
    DeviceGuard guard(inst->device);
    void* p = nullptr;
    MM_HIP(hipMalloc(&p, bytes));
    mm_alloc a = new (std::nothrow) mm_alloc_s{inst, p, bytes, true, 0};
    if (!a) {
        (void)hipFree(p);
        return fail(MM_ERR_OUT_OF_MEMORY, "alloc_linear: host allocation");
    }
    inst->allocs.insert(a);
    *dev_ptr = p;
    *out = a;
    return MM_OK;
}

mm_status mm_alloc_wrap(mm_instance inst, void* dev_ptr, size_t bytes, mm_alloc* out) {
    if (!inst || !dev_ptr || !out) return fail(MM_ERR_INVALID_ARG, "alloc_wrap: null argument");
    if (bytes == 0) return fail(MM_ERR_INVALID_ARG, "alloc_wrap: zero bytes");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 4 != 0)
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: pointer not 4-byte aligned");
    hipPointerAttribute_t attr{};
    const hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != inst->device) {
        (void)hipGetLastError();
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: %p is not device memory of device %d",
                    dev_ptr, inst->device);
    }
    // the whole range must lie inside one device allocation
    hipDeviceptr_t base = nullptr;
    size_t range = 0;
    if (hipMemGetAddressRange(&base, &range, dev_ptr) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: no allocation contains %p", dev_ptr);
    }
    const uintptr_t lo = reinterpret_cast<uintptr_t>(base);
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(dev_ptr);
    if (p0 < lo || bytes > range - (p0 - lo))
        return fail(MM_ERR_INVALID_ARG, "alloc_wrap: %zu bytes at %p overrun the %zu-byte allocation",
                    bytes, dev_ptr, range);
    mm_alloc a = new (std::nothrow) mm_alloc_s{inst, dev_ptr, bytes, false, 0};
    if (!a) return fail(MM_ERR_OUT_OF_MEMORY, "alloc_wrap: host allocation");
    inst->allocs.insert(a);
    *out = a;
    return MM_OK;
}

mm_status mm_free(mm_alloc a) {
    if (!a) return fail(MM_ERR_INVALID_ARG, "free: null alloc");
    if (a->users) return fail(MM_ERR_IN_USE, "free: %u view(s) still use this alloc", a->users);
    mm_instance inst = a->inst;
    DeviceGuard guard(inst->device);
    if (a->owned) {
        MM_HIP(hipStreamSynchronize(inst->stream));
        MM_HIP(hipFree(a->ptr));
    }
    inst->allocs.erase(a);
    delete a;
    return MM_OK;
}

mm_status mm_create_view(mm_instance inst, const mm_view_desc* desc, mm_view* out) {
    if (!inst || !desc || !out) return fail(MM_ERR_INVALID_ARG, "create_view: null argument");
    if (!desc->position || inst->allocs.count(desc->position) == 0)
        return fail(MM_ERR_INVALID_ARG, "create_view: position is not an alloc of this instance");
    const mm_status vs = validate_desc(inst, desc);
    if (vs != MM_OK) return vs;
    DeviceGuard guard(inst->device);
    mm_view v = new (std::nothrow) mm_view_s();
    if (!v) return fail(MM_ERR_OUT_OF_MEMORY, "create_view: host allocation");
    v->inst = inst;
    v->position = desc->position;
    v->desc = *desc;
    const uint64_t npix = static_cast<uint64_t>(desc->width) * desc->height;
    hipError_t e = hipMalloc(&v->depth, npix * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&v->colour, npix * sizeof(uint32_t));
    if (e == hipSuccess) e = mm::launch_fill(v->depth, npix, inst->stream);
    if (e == hipSuccess) e = hipMemsetAsync(v->colour, 0, npix * sizeof(uint32_t), inst->stream);
    if (e != hipSuccess) {
        destroy_view_resources(v);
        delete v;
        return fail(e == hipErrorOutOfMemory ? MM_ERR_OUT_OF_MEMORY : MM_ERR_HIP,
                    "create_view: device buffers: %s", hipGetErrorString(e));
    }
    fill_point_args(v);
    const int dim = static_cast<int>(desc->domain);
    v->point_l = mm::point_launch(dim, static_cast<int>(desc->footprint), desc->wrap != 0,
                                  mm::kDisplaceRender, v->args.n);
    v->resolve_l = mm::resolve_launch(npix);
    const mm_status gs = build_graph(v, false, &v->graph, &v->exec, &v->point_node, nullptr);
    if (gs != MM_OK) {
        destroy_view_resources(v);
        delete v;
        return gs;
    }
    desc->position->users++;
    inst->views.insert(v);
    *out = v;
    return MM_OK;
}

mm_status mm_destroy_view(mm_view v) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "destroy_view: null view");
    mm_instance inst = v->inst;
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    destroy_view_resources(v);
    v->position->users--;
    inst->views.erase(v);
    delete v;
    return MM_OK;
}

mm_status mm_set_camera(mm_view v, const float m[16]) {
    if (!v || !m) return fail(MM_ERR_INVALID_ARG, "set_camera: null argument");
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(m[k])) return fail(MM_ERR_INVALID_ARG, "set_camera: m[%d] not finite", k);
    std::memcpy(v->desc.view_proj, m, sizeof(float) * 16);
    const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) v->args.m[4 * r + c] = m[4 * rows[r] + c];
    return MM_OK;
}

mm_status mm_step(mm_view v, uint32_t step) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "step: null view");
    DeviceGuard guard(v->inst->device);
    v->args.step = step;
    MM_HIP(mm::launch_point(v->args, static_cast<int>(v->desc.domain),
                            static_cast<int>(v->desc.footprint), v->desc.wrap != 0,
                            mm::kDisplace, v->inst->stream));
    return MM_OK;
}

mm_status mm_render(mm_view v) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "render: null view");
    DeviceGuard guard(v->inst->device);
    MM_HIP(mm::launch_point(v->args, static_cast<int>(v->desc.domain),
                            static_cast<int>(v->desc.footprint), v->desc.wrap != 0,
                            mm::kRender, v->inst->stream));
    MM_HIP(mm::launch_resolve(v->rargs, v->inst->stream));
    return MM_OK;
}

mm_status mm_step_render(mm_view v, uint32_t step) {
    if (!v) return fail(MM_ERR_INVALID_ARG, "step_render: null view");
    DeviceGuard guard(v->inst->device);
    v->args.step = step;
    void* pargs[] = {&v->args};
    hipKernelNodeParams pp = node_params(v->point_l, pargs);
    if (v->profiling && v->prof_count < v->prof_cap) {
        const uint32_t k = v->prof_count++;
        for (int j = 0; j < 3; ++j)
            MM_HIP(hipGraphExecEventRecordNodeSetEvent(v->texec, v->tevent_node[j],
                                                       v->events[3 * k + j]));
        MM_HIP(hipGraphExecKernelNodeSetParams(v->texec, v->tpoint_node, &pp));
        MM_HIP(hipGraphLaunch(v->texec, v->inst->stream));
        return MM_OK;
    }
    MM_HIP(hipGraphExecKernelNodeSetParams(v->exec, v->point_node, &pp));
    MM_HIP(hipGraphLaunch(v->exec, v->inst->stream));
    return MM_OK;
}

mm_status mm_frame_device_ptr(mm_view v, const uint32_t** dev_rgba) {
    if (!v || !dev_rgba) return fail(MM_ERR_INVALID_ARG, "frame_device_ptr: null argument");
    *dev_rgba = v->colour;
    return MM_OK;
}

mm_status mm_read_frame(mm_view v, void* host_rgba, size_t bytes) {
    if (!v || !host_rgba) return fail(MM_ERR_INVALID_ARG, "read_frame: null argument");
    const size_t need = static_cast<size_t>(v->desc.width) * v->desc.height * sizeof(uint32_t);
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipMemcpyAsync(host_rgba, v->colour, need, hipMemcpyDeviceToHost, v->inst->stream));
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    return MM_OK;
}

mm_status mm_profile_begin(mm_view v, uint32_t capacity) {
    if (!v || capacity == 0 || capacity > (1u << 20))
        return fail(MM_ERR_INVALID_ARG, "profile_begin: null view or capacity outside [1, 2^20]");
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    if (v->texec) (void)hipGraphExecDestroy(v->texec);
    if (v->tgraph) (void)hipGraphDestroy(v->tgraph);
    v->texec = nullptr;
    v->tgraph = nullptr;
    for (hipEvent_t e : v->events) (void)hipEventDestroy(e);
    v->events.assign(3ull * capacity, nullptr);
    for (auto& e : v->events) MM_HIP(hipEventCreate(&e));
    const mm_status gs = build_graph(v, true, &v->tgraph, &v->texec, &v->tpoint_node, v->tevent_node);
    if (gs != MM_OK) return gs;
    v->prof_cap = capacity;
    v->prof_count = 0;
    v->profiling = true;
    return MM_OK;
}

mm_status mm_profile_end(mm_view v, float* splat_ms, float* resolve_ms, float* frame_ms,
                         uint32_t* count) {
    if (!v || !count) return fail(MM_ERR_INVALID_ARG, "profile_end: null argument");
    if (!v->profiling) return fail(MM_ERR_INVALID_ARG, "profile_end: no profile_begin");
    DeviceGuard guard(v->inst->device);
    MM_HIP(hipStreamSynchronize(v->inst->stream));
    for (uint32_t k = 0; k < v->prof_count; ++k) {
        float t = 0.0f;
        hipEvent_t* e = &v->events[3ull * k];
        if (splat_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[0], e[1]));
            splat_ms[k] = t;
        }
        if (resolve_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[1], e[2]));
            resolve_ms[k] = t;
        }
        if (frame_ms) {
            MM_HIP(hipEventElapsedTime(&t, e[0], e[2]));
            frame_ms[k] = t;
        }
    }
    *count = v->prof_count;
    v->profiling = false;
    return MM_OK;
}

}  // extern "C"
