// Structured-grid view: a cols x rows lattice of cells, each drawn as the
// palette entry of its cell value, filling the screen (the paper's voxel view
// of a 2D structured domain, as used for the Potts-model lattice, with colour
// from a colormap through the cell's index). Each thread takes four pixels of
// a row: the cell under each pixel centre by integer arithmetic, an index
// load, a palette load and a non-temporal colour store per pixel.
#include <hip/hip_runtime.h>

#include <new>

#include "mm_host.h"

namespace {

struct GridArgs {
    const void* index;       // cols * rows cell values, row-major, row 0 at the bottom
    const uint32_t* palette;
    uint32_t* colour;        // width * height RGBA8, row 0 at the top
    uint32_t cols, rows, width, height;
    uint32_t palette_size, index_size;
};

// Cell column of pixel column px: floor((px + 1/2) * cols / width), exactly.
// (2 px + 1) * cells < 32769 * 65536 < 2^32, so 32-bit arithmetic is exact.
__device__ __forceinline__ uint32_t cell_of(uint32_t p, uint32_t cells, uint32_t pixels) {
    return (2u * p + 1u) * cells / (2u * pixels);
}

// Four pixels per thread, 256 apart, so their loads are in flight together.
constexpr uint32_t kGridPix = 4;

__device__ __forceinline__ uint32_t cell_value(const GridArgs& a, uint64_t cell) {
    if (a.index_size == 1) return static_cast<const uint8_t*>(a.index)[cell];
    if (a.index_size == 2) return static_cast<const uint16_t*>(a.index)[cell];
    return static_cast<const uint32_t*>(a.index)[cell];
}

__global__ __launch_bounds__(256) void grid_kernel(GridArgs a) {
    const uint32_t py = blockIdx.y;
    const uint32_t cy = cell_of(a.height - 1u - py, a.rows, a.height);  // y up; uniform per block
    const uint64_t row = static_cast<uint64_t>(cy) * a.cols;
    const uint32_t x0 = blockIdx.x * (256u * kGridPix) + threadIdx.x;
    uint32_t v[kGridPix];
#pragma unroll
    for (uint32_t k = 0; k < kGridPix; ++k) {
        const uint32_t px = min(x0 + k * 256u, a.width - 1u);  // tail lanes repeat the last pixel
        v[k] = cell_value(a, row + cell_of(px, a.cols, a.width));
    }
    uint32_t c[kGridPix];
#pragma unroll
    for (uint32_t k = 0; k < kGridPix; ++k) c[k] = v[k] < a.palette_size ? a.palette[v[k]] : 0u;
    uint32_t* out = a.colour + static_cast<uint64_t>(py) * a.width;
#pragma unroll
    for (uint32_t k = 0; k < kGridPix; ++k) {
        const uint32_t px = x0 + k * 256u;
        if (px < a.width) __builtin_nontemporal_store(c[k], out + px);
    }
}

}  // namespace

struct mm_grid_s {
    mm_instance inst;
    mm_alloc palette, indices;
    GridArgs args;
};

using namespace mmh;

extern "C" {

mm_status mm_create_grid(mm_instance inst, const mm_grid_desc* d, mm_grid* out) {
    if (!inst || !d || !out) return fail(MM_ERR_INVALID_ARG, "create_grid: null argument");
    if (d->cols < 1 || d->rows < 1 || d->cols > 65536 || d->rows > 65536)
        return fail(MM_ERR_INVALID_ARG, "create_grid: lattice %ux%u outside [1, 65536]^2", d->cols, d->rows);
    MM_TRY(validate_screen(d->width, d->height, "create_grid"));
    if (!d->palette || !inst->allocs.count(d->palette))
        return fail(MM_ERR_INVALID_ARG, "create_grid: palette is not an alloc of this instance");
    if (d->palette_size < 1 || d->palette_size > d->palette->bytes / 4)
        return fail(MM_ERR_INVALID_ARG, "create_grid: %u palette entries do not fit the %zu-byte alloc",
                    d->palette_size, d->palette->bytes);
    if (!d->indices || !inst->allocs.count(d->indices))
        return fail(MM_ERR_INVALID_ARG, "create_grid: indices is not an alloc of this instance");
    if (d->index_size != 1 && d->index_size != 2 && d->index_size != 4)
        return fail(MM_ERR_INVALID_ARG, "create_grid: index_size %u is not 1, 2 or 4", d->index_size);
    const uint64_t cells = static_cast<uint64_t>(d->cols) * d->rows;
    if (cells > d->indices->bytes / d->index_size)
        return fail(MM_ERR_INVALID_ARG, "create_grid: %llu cells of %u B exceed the %zu-byte alloc",
                    (unsigned long long)cells, d->index_size, d->indices->bytes);
    DeviceGuard guard(inst->device);
    const uint64_t npix = static_cast<uint64_t>(d->width) * d->height;
    uint32_t* colour = nullptr;
    hipError_t e = alloc_n(&colour, npix);
    if (e == hipSuccess) e = hipMemsetAsync(colour, 0, npix * 4, inst->stream);
    if (e != hipSuccess) {
        if (colour) (void)hipFree(colour);
        return hip_fail(e, "create_grid: frame buffer");
    }
    mm_grid g = new (std::nothrow) mm_grid_s{inst, d->palette, d->indices,
                                             GridArgs{d->indices->ptr, static_cast<const uint32_t*>(d->palette->ptr),
                                                      colour, d->cols, d->rows, d->width, d->height,
                                                      d->palette_size, d->index_size}};
    if (!g) {
        (void)hipFree(colour);
        return fail(MM_ERR_OUT_OF_MEMORY, "create_grid: host allocation");
    }
    d->palette->users++;
    d->indices->users++;
    inst->grids.insert(g);
    *out = g;
    return MM_OK;
}

mm_status mm_destroy_grid(mm_grid g) {
    if (!g) return fail(MM_ERR_INVALID_ARG, "destroy_grid: null grid");
    mm_instance inst = g->inst;
    if (!inst->grids.count(g)) return fail(MM_ERR_INVALID_ARG, "destroy_grid: unknown grid");
    DeviceGuard guard(inst->device);
    MM_HIP(hipStreamSynchronize(inst->stream));
    (void)hipFree(g->args.colour);
    g->palette->users--;
    g->indices->users--;
    inst->grids.erase(g);
    delete g;
    return MM_OK;
}

mm_status mm_grid_render(mm_grid g) {
    if (!g) return fail(MM_ERR_INVALID_ARG, "grid_render: null grid");
    DeviceGuard guard(g->inst->device);
    const dim3 grid((g->args.width + 256u * kGridPix - 1u) / (256u * kGridPix), g->args.height);
    GridArgs a = g->args;
    void* args[] = {&a};
    MM_HIP(hipLaunchKernel(reinterpret_cast<const void*>(&grid_kernel), grid, dim3(256), args, 0,
                           g->inst->stream));
    return MM_OK;
}

mm_status mm_grid_frame_device_ptr(mm_grid g, const uint32_t** dev_rgba) {
    if (!g || !dev_rgba) return fail(MM_ERR_INVALID_ARG, "grid_frame_device_ptr: null argument");
    *dev_rgba = g->args.colour;
    return MM_OK;
}

mm_status mm_grid_read_frame(mm_grid g, void* host_rgba, size_t bytes) {
    if (!g || !host_rgba) return fail(MM_ERR_INVALID_ARG, "grid_read_frame: null argument");
    const size_t need = static_cast<size_t>(g->args.width) * g->args.height * 4;
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "grid_read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(g->inst->device);
    MM_HIP(hipMemcpyAsync(host_rgba, g->args.colour, need, hipMemcpyDeviceToHost, g->inst->stream));
    MM_HIP(hipStreamSynchronize(g->inst->stream));
    return MM_OK;
}

}  // extern "C"
