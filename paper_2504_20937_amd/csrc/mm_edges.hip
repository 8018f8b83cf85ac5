// Edges view: segments between indexed vertices of a point cloud (the
// paper's edge views of triangle meshes and Delaunay triangulations), drawn
// into a key buffer with the same (depth bits << 32 | id) minimum as points,
// then resolved to RGBA8. One thread per primitive (a vertex pair, or a
// triangle's three sides); a segment is sampled at n + 1 points, n the
// ceiling of its longer screen extent (at most kMaxSteps), each interpolated
// in binary32 from the first vertex in a fixed order, so the frame is exact.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "mm_device.h"
#include "mm_host.h"

namespace {

using namespace mm;
using namespace mm::dev;

constexpr uint32_t kMaxSteps = 32768;

struct EdgesArgs {
    const float* pos;
    const uint32_t* idx;
    uint64_t* depth;
    uint32_t n;          // vertices
    uint32_t nprim;      // primitives
    uint32_t prim;       // 2: vertex pairs, 3: triangles
    ViewGeom g;
};

// Screen position before the pixel floor and clip w (3D) of a vertex, in the
// point projection's operation order; false when the near test culls it.
template <int DIM>
__device__ __forceinline__ bool screen_of(const ViewGeom& a, const float* pos, uint32_t i,
                                          float& sx, float& sy, float& w) {
    if constexpr (DIM == 2) {
        const float x = pos[2ull * i], y = pos[2ull * i + 1];
        sx = (x + 1.0f) * a.half_w;
        sy = (y + 1.0f) * a.half_h;
        w = 0.0f;
        return true;
    } else {
        const float x = pos[3ull * i], y = pos[3ull * i + 1], z = pos[3ull * i + 2];
        float cx = a.m[0] * x;
        cx = cx + a.m[1] * y;
        cx = cx + a.m[2] * z;
        cx = cx + a.m[3];
        float cy = a.m[4] * x;
        cy = cy + a.m[5] * y;
        cy = cy + a.m[6] * z;
        cy = cy + a.m[7];
        float cw = a.m[8] * x;
        cw = cw + a.m[9] * y;
        cw = cw + a.m[10] * z;
        cw = cw + a.m[11];
        if (!(cw > 0.1f)) return false;
        const float iw = 1.0f / cw;
        sx = (cx * iw + 1.0f) * a.half_w;
        sy = (cy * iw + 1.0f) * a.half_h;
        w = cw;
        return true;
    }
}

template <int DIM>
__device__ void draw_segment(const EdgesArgs& a, uint32_t va, uint32_t vb, uint32_t e) {
    if (va >= a.n || vb >= a.n) return;
    float ax, ay, aw, bx, by, bw;
    if (!screen_of<DIM>(a.g, a.pos, va, ax, ay, aw)) return;
    if (!screen_of<DIM>(a.g, a.pos, vb, bx, by, bw)) return;
    const float dx = bx - ax, dy = by - ay, dw = bw - aw;
    const float len = fmaxf(fabsf(dx), fabsf(dy));
    const uint32_t steps = len >= static_cast<float>(kMaxSteps) ? kMaxSteps
                                                                 : static_cast<uint32_t>(ceilf(len));
    for (uint32_t k = 0; k <= steps; ++k) {
        const float t = steps == 0u ? 0.0f : static_cast<float>(k) / static_cast<float>(steps);
        const float x = ax + t * dx;
        const float y = ay + t * dy;
        const float w = aw + t * dw;
        if (!(x >= 0.0f && x < a.g.fwidth && y >= 0.0f && y < a.g.fheight)) continue;
        const int32_t px = static_cast<int32_t>(floorf(x));
        const int32_t py = static_cast<int32_t>(a.g.height) - 1 - static_cast<int32_t>(floorf(y));
        const uint64_t key = (static_cast<uint64_t>(DIM == 2 ? 0u : __float_as_uint(w)) << 32) | e;
        uint64_t* slot = a.depth + static_cast<uint64_t>(py) * a.g.width + static_cast<uint32_t>(px);
        if (key < *slot) atomic_min_global(slot, key);
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void edges_kernel(EdgesArgs a) {
    const uint32_t q = blockIdx.x * 256u + threadIdx.x;
    if (q >= a.nprim) return;
    if (a.prim == 2u) {
        draw_segment<DIM>(a, a.idx[2ull * q], a.idx[2ull * q + 1], q);
    } else {
        const uint32_t v0 = a.idx[3ull * q], v1 = a.idx[3ull * q + 1], v2 = a.idx[3ull * q + 2];
        draw_segment<DIM>(a, v0, v1, 3u * q);
        draw_segment<DIM>(a, v1, v2, 3u * q + 1u);
        draw_segment<DIM>(a, v2, v0, 3u * q + 2u);
    }
}

}  // namespace

struct mm_edges_s {
    mm_instance inst;
    mm_alloc position, indices;
    mm_domain domain;
    uint32_t* colour;
    EdgesArgs args;
    ResolveArgs rargs;
};

using namespace mmh;

extern "C" {

mm_status mm_create_edges(mm_instance inst, const mm_edges_desc* d, mm_edges* out) {
    if (!inst || !d || !out) return fail(MM_ERR_INVALID_ARG, "create_edges: null argument");
    if (d->domain != MM_DOMAIN_2D && d->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "create_edges: domain %d is not 2D/3D", (int)d->domain);
    const mm_cloud_desc c{d->position, d->element_count, d->format, d->seed, 0.0f, 0};
    MM_TRY(validate_cloud(inst, c, d->domain, "create_edges"));
    MM_TRY(validate_screen(d->width, d->height, "create_edges"));
    if (d->domain == MM_DOMAIN_3D) MM_TRY(validate_camera(d->view_proj, "create_edges"));
    if (d->vertices_per_primitive != 2 && d->vertices_per_primitive != 3)
        return fail(MM_ERR_INVALID_ARG, "create_edges: vertices_per_primitive %u is not 2 or 3",
                    d->vertices_per_primitive);
    const uint64_t edges = d->primitive_count * d->vertices_per_primitive / (d->vertices_per_primitive == 2 ? 2 : 1);
    if (d->primitive_count < 1 || edges > 0xFFFFFFFFull)
        return fail(MM_ERR_INVALID_ARG, "create_edges: %llu primitives (1 .. 2^32 - 1 edges)",
                    (unsigned long long)d->primitive_count);
    if (!d->indices || !inst->allocs.count(d->indices))
        return fail(MM_ERR_INVALID_ARG, "create_edges: indices is not an alloc of this instance");
    if (d->primitive_count * d->vertices_per_primitive > d->indices->bytes / 4)
        return fail(MM_ERR_INVALID_ARG, "create_edges: %llu vertex indices exceed the %zu-byte alloc",
                    (unsigned long long)(d->primitive_count * d->vertices_per_primitive), d->indices->bytes);
    DeviceGuard guard(inst->device);
    const uint64_t npix = static_cast<uint64_t>(d->width) * d->height;
    uint32_t* colour = nullptr;
    uint64_t* depth = nullptr;
    hipError_t e = alloc_n(&colour, npix);
    if (e == hipSuccess) e = alloc_n(&depth, npix);
    if (e == hipSuccess) e = hipMemsetAsync(colour, 0, npix * 4, inst->stream);
    if (e == hipSuccess) e = launch_fill(depth, npix, kEmptyKey, inst->stream);
    if (e != hipSuccess) {
        if (colour) (void)hipFree(colour);
        if (depth) (void)hipFree(depth);
        return hip_fail(e, "create_edges: frame buffers");
    }
    EdgesArgs a{};
    a.pos = static_cast<const float*>(d->position->ptr);
    a.idx = static_cast<const uint32_t*>(d->indices->ptr);
    a.depth = depth;
    a.n = static_cast<uint32_t>(d->element_count);
    a.nprim = static_cast<uint32_t>(d->primitive_count);
    a.prim = d->vertices_per_primitive;
    a.g = view_geom(d->width, d->height, d->view_proj);
    ResolveArgs r{depth, colour, npix, static_cast<uint32_t>(d->seed), static_cast<uint32_t>(d->seed >> 32),
                  Palette{}};
    mm_edges g = new (std::nothrow) mm_edges_s{inst, d->position, d->indices, d->domain, colour, a, r};
    if (!g) {
        (void)hipFree(colour);
        (void)hipFree(depth);
        return fail(MM_ERR_OUT_OF_MEMORY, "create_edges: host allocation");
    }
    d->position->users++;
    d->indices->users++;
    inst->edges.insert(g);
    *out = g;
    return MM_OK;
}

mm_status mm_destroy_edges(mm_edges g) {
    if (!g) return fail(MM_ERR_INVALID_ARG, "destroy_edges: null view");
    mm_instance inst = g->inst;
    if (!inst->edges.count(g)) return fail(MM_ERR_INVALID_ARG, "destroy_edges: unknown view");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    (void)hipFree(g->colour);
    (void)hipFree(g->args.depth);
    g->position->users--;
    g->indices->users--;
    inst->edges.erase(g);
    delete g;
    return MM_OK;
}

mm_status mm_edges_set_camera(mm_edges g, const float m[16]) {
    if (!g || !m) return fail(MM_ERR_INVALID_ARG, "edges_set_camera: null argument");
    MM_TRY(validate_camera(m, "edges_set_camera"));
    set_camera_rows(g->args.g, m);
    return MM_OK;
}

mm_status mm_edges_render(mm_edges g) {
    if (!g) return fail(MM_ERR_INVALID_ARG, "edges_render: null view");
    DeviceGuard guard(g->inst->device);
    const void* f = g->domain == MM_DOMAIN_2D ? reinterpret_cast<const void*>(&edges_kernel<2>)
                                              : reinterpret_cast<const void*>(&edges_kernel<3>);
    EdgesArgs a = g->args;
    void* args[] = {&a};
    MM_HIP(hipLaunchKernel(f, dim3((a.nprim + 255u) / 256u), dim3(256), args, 0, g->inst->stream));
    MM_HIP(launch_resolve(g->rargs, g->inst->stream));
    return MM_OK;
}

mm_status mm_edges_frame_device_ptr(mm_edges g, const uint32_t** dev_rgba) {
    if (!g || !dev_rgba) return fail(MM_ERR_INVALID_ARG, "edges_frame_device_ptr: null argument");
    *dev_rgba = g->colour;
    return MM_OK;
}

mm_status mm_edges_read_frame(mm_edges g, void* host_rgba, size_t bytes) {
    if (!g || !host_rgba) return fail(MM_ERR_INVALID_ARG, "edges_read_frame: null argument");
    const size_t need = static_cast<size_t>(g->args.g.width) * g->args.g.height * 4;
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "edges_read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(g->inst->device);
    MM_HIP(hipMemcpyAsync(host_rgba, g->colour, need, hipMemcpyDeviceToHost, g->inst->stream));
    MM_HIP(hipStreamSynchronize(g->inst->stream));
    return MM_OK;
}

}  // extern "C"
