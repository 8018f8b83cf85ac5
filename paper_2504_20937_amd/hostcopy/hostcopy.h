/*
 * hostcopy.h: the host-copy comparison path's renderer (host memory in,
 * RGBA8 frame out, all host cores). Not part of the device path: the
 * benchmark times it beside the device frame.
 */
#ifndef MM_HOSTCOPY_H
#define MM_HOSTCOPY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Renders n points (AoS float2 when dim == 2, float3 when dim == 3) held in
 * host memory into rgba (width * height uint32, row 0 = top), as the device
 * path draws them: view_proj is the row-major camera (3D), footprint 1 or 3,
 * seed keys the colour hash. threads <= 0 uses every core OpenMP offers.
 * Allocates threads * width * height * 8 bytes of host scratch for the call.
 * Returns 0, -1 for an invalid argument, -2 when the scratch cannot be
 * allocated. */
int hc_render(const float* pos, uint64_t n, int dim, const float view_proj[16], uint32_t width,
              uint32_t height, uint32_t footprint, uint64_t seed, uint32_t* rgba, int threads);

/* Threads hc_render uses by default. */
int hc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
