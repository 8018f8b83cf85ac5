/*
 * mm.h: C ABI of the MI355X displace+render library.
 *
 * The calls follow the three stages the Mimir paper gives its interface
 * (section "Interface"): initialise an instance and allocate memory from it,
 * describe a view of that memory, and render. Allocation mirrors the paper's
 * allocLinear, which takes the same arguments as the native allocator and
 * hands back a plain device pointer plus a handle (section "Allocations").
 * A view is described by a plain struct, as the paper's ViewDescription
 * (section "Views", listing "C++ Library usage example"): the position
 * source, element count, format, domain, and here also the camera, the
 * screen and the per-step displacement of the benchmark (section
 * "Performance Benchmark"). There is no window and no graphics API: frames
 * stay in device memory and are copied to the host only on request.
 *
 * Conventions for every call:
 *  - The return value is an mm_status: MM_OK (0) or a negative error code.
 *    On error, out-parameters are left untouched, what the call allocated
 *    is freed, and mm_last_error() gives a thread-local message. A call that
 *    reshapes an object (mm_set_tuning, mm_set_frame_overlap,
 *    mm_batch_set_tuning) and fails puts back the shape the object had.
 *  - Pointers named dev_* are device addresses; every other pointer is host
 *    memory owned by the caller and only read or written during the call.
 *  - Calls on one instance (and on its views, batches) must be serialised
 *    by the caller. The server object (mm_server_*) is internally locked.
 *  - All device work is enqueued on the instance's stream, in call order.
 *    Calls return without waiting unless stated ("synchronises").
 *  - Positions are AoS float32: float2 (x, y) or float3 (x, y, z).
 *  - Frames are RGBA8 packed in uint32 little-endian (R in the low byte),
 *    row-major, row 0 = top of the screen; 0 = background.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_instance_s* mm_instance;
typedef struct mm_alloc_s* mm_alloc;
typedef struct mm_view_s* mm_view;
typedef struct mm_batch_s* mm_batch;
typedef struct mm_server_s* mm_server;
typedef struct mm_grid_s* mm_grid;
typedef struct mm_edges_s* mm_edges;

typedef int32_t mm_status;
#define MM_OK 0
#define MM_ERR_INVALID_ARG (-1)   /* a null handle/pointer or an out-of-range field */
#define MM_ERR_OUT_OF_MEMORY (-2) /* device or host allocation failed */
#define MM_ERR_HIP (-3)           /* a HIP runtime call failed (message has the call) */
#define MM_ERR_BUDGET (-4)        /* a request exceeds a configured memory budget */
#define MM_ERR_IN_USE (-5)        /* the object is still referenced (e.g. alloc by a view) */
#define MM_ERR_UNSUPPORTED (-6)   /* valid but not supported (format/domain combination) */
#define MM_ERR_NOT_READY (-7)     /* a polled result is not available yet */

typedef enum { MM_FLOAT2 = 2, MM_FLOAT3 = 3 } mm_format;
typedef enum { MM_DOMAIN_2D = 2, MM_DOMAIN_3D = 3 } mm_domain;

/* ---------------------------------------------------------------- instance
 * Section "Initialization": the instance binds one device. Here it also
 * binds one stream. */
typedef struct {
    int32_t device; /* HIP device ordinal */
    void* stream;   /* hipStream_t to enqueue on (e.g. torch's current stream); NULL:
                       the library creates a default-priority stream and owns it */
} mm_instance_desc;

/* Creates an instance on desc->device. *out receives the handle. */
mm_status mm_create_instance(const mm_instance_desc* desc, mm_instance* out);

/* Waits for the stream, destroys every view still alive, frees every
 * allocation the instance owns (not wrapped ones), then the stream if it
 * owns it. The handle is invalid afterwards. */
mm_status mm_destroy_instance(mm_instance inst);

/* Waits until all work enqueued on the instance's stream has finished. */
mm_status mm_synchronize(mm_instance inst);

/* Compute sections, the paper's prepareViews / updateViews (section
 * "Synchronization": a simulation's writes to the viewed allocations are
 * bracketed so that display never reads a half-written state). For a
 * simulation that writes positions (or other viewed data) on a HIP stream of
 * its own, `stream` (NULL: the null stream):
 *   mm_prepare_views: `stream` waits until the work enqueued so far on the
 *     instance (frames, batches, grids, edge views) has finished, so the
 *     simulation may then overwrite what that work reads;
 *   mm_update_views: the instance's later work waits until the work enqueued
 *     so far on `stream` has finished, so the next frames see the writes.
 * Work enqueued on the instance between the two calls runs beside the
 * simulation: the paper's ping-pong scheme, one buffer rendered while the
 * other is written (two views on two allocations, rendered alternately).
 * Both calls only enqueue events (no host wait). Servers run on streams of
 * their own and are not covered. */
mm_status mm_prepare_views(mm_instance inst, void* stream);
mm_status mm_update_views(mm_instance inst, void* stream);

/* ------------------------------------------------------------- allocations
 * Section "Allocations": allocLinear takes the native allocator's
 * arguments and returns a plain device pointer that kernels use as usual,
 * plus a handle that views refer to. */

/* Allocates bytes (> 0) of device memory owned by the instance, 256-byte
 * aligned. *dev_ptr receives the device address, *out the handle. */
mm_status mm_alloc_linear(mm_instance inst, size_t bytes, void** dev_ptr, mm_alloc* out);

/* Wraps caller-owned device memory (e.g. a torch CUDA/HIP tensor) of
 * `bytes` bytes at dev_ptr (4-byte aligned, on the instance's device). The
 * library never frees it; the caller keeps it alive while views use it. */
mm_status mm_alloc_wrap(mm_instance inst, void* dev_ptr, size_t bytes, mm_alloc* out);

/* Releases the handle (and the memory, for mm_alloc_linear). Returns
 * MM_ERR_IN_USE while a view still refers to it. */
mm_status mm_free(mm_alloc alloc);

/* ------------------------------------------------------------------- views
 * Section "Views": a view describes how raw memory is drawn. Here a view
 * draws a point cloud as markers of one size (section "Performance
 * Benchmark": every point the same size), and also carries the benchmark's
 * per-timestep displacement of that cloud. */
typedef struct {
    mm_alloc position;      /* source of the positions: element_count points, AoS */
    uint64_t element_count; /* N, 1 <= N <= 2^32 - 1; N * stride must fit the alloc */
    mm_format format;       /* MM_FLOAT2 with MM_DOMAIN_2D, MM_FLOAT3 with MM_DOMAIN_3D */
    mm_domain domain;
    uint32_t width;         /* screen size in pixels, each even and in [2, 16384] */
    uint32_t height;
    uint32_t footprint;     /* marker side in pixels: 1 or 3 */
    uint64_t seed;          /* key of the displacement draw and of the colour hash */
    float amplitude;        /* per-coordinate offset is uniform on [-a, a); a == 0 or
                               2^-64 <= a <= 2^64 (a <= 1 when wrap is set) */
    int32_t wrap;           /* 1: fold each coordinate into [-1, 1) after the step */
    float view_proj[16];    /* row-major float32 clip-from-world matrix; 3D only */
} mm_view_desc;

/* Creates a view: validates desc, allocates its RGBA8 frame (4 B per pixel,
 * zero) and the scratch buffers of its splat strategy (MM_SPLAT_AUTO, see
 * mm_set_tuning), and builds its per-frame graph. The view refers to
 * desc->position until destroyed. */
mm_status mm_create_view(mm_instance inst, const mm_view_desc* desc, mm_view* out);

/* Frees the view's buffers and graph (after the stream has drained). */
mm_status mm_destroy_view(mm_view view);

/* Replaces the view's 3D camera (row-major, 16 floats) for later frames. */
mm_status mm_set_camera(mm_view view, const float view_proj[16]);

/* Displacement only: every point i moves by the draw keyed by (seed, i,
 * step), as the benchmark's per-timestep kernel. */
mm_status mm_step(mm_view view, uint32_t step);

/* Render only: splat the current positions and resolve them into the
 * view's frame. */
mm_status mm_render(mm_view view);

/* One frame: displace with `step`, then splat and resolve, as one graph
 * launch on the stream. Equivalent to mm_step then mm_render. */
mm_status mm_step_render(mm_view view, uint32_t step);

/* `count` frames in one graph launch (1 <= count <= 64): frame i displaces
 * with step first_step + i and, when view_proj is not NULL, renders with the
 * camera view_proj[16 i .. 16 i + 15] (row-major, count * 16 floats; NULL:
 * the view's camera for every frame). The same frames as mm_set_camera then
 * mm_step_render per frame, bit for bit, without the gap a device leaves
 * between graph launches (section "Performance Benchmark" runs its time
 * steps back to back); the frame buffer holds the last one, and the view's
 * camera is left at the last camera. With frame overlap the frames are
 * enqueued one by one. Frame marks mark every frame; a profile samples at
 * most the first frame of a launch. The first call for a count builds and
 * keeps that count's graph. */
mm_status mm_step_render_frames(mm_view view, uint32_t first_step, uint32_t count,
                                const float* view_proj);

/* Colour of a view's points (section "Views": a colour property read per
 * element, or through an index description into a table, as value mapping
 * with a colormap; a default when the property is absent). */
typedef struct {
    mm_alloc palette;      /* RGBA8 entries (uint32 each, red in the low byte, stored
                              as given, alpha included); NULL: the default colour,
                              a hash of the point index with opaque alpha */
    uint32_t palette_size; /* entries, >= 1; without indices, >= the view's points */
    mm_alloc indices;      /* per-point unsigned palette index of index_size bytes;
                              NULL: point i takes palette entry i */
    uint32_t index_size;   /* 1, 2 or 4 */
} mm_colour_desc;

/* Sets the view's colour source for later frames (desc NULL: the default
 * hash colour). A pixel's colour is that of the point that wins its depth
 * test; an index at or past palette_size gives colour 0 (the point still
 * hides what lies behind it). The view keeps the allocations in use (mm_free
 * refuses them) until another colour source is set or the view is
 * destroyed; their contents are read at every frame. Rebuilds the frame
 * graph and synchronises. */
mm_status mm_set_colour(mm_view view, const mm_colour_desc* desc);

/* Frame overlap, the device form of the paper's ping-pong scheme (section
 * "Synchronization": one buffer is displayed while the other is written)
 * with the two sides unsynchronised (the study of section "Performance
 * Benchmark" with synchronization disabled). With on = 1 (binned splat only), frame f is
 * displaced, projected and binned into one of two record sets on the
 * instance stream while frame f - 1 is drawn from the other set on a render
 * stream of the view's own, so the two passes of consecutive frames run
 * side by side. mm_step_render then leaves the frame buffer one frame
 * behind: after the call for step f it holds (or will hold) frame f - 1, and
 * frames are still bit-identical to the serial path's. Every tile not drawn
 * in a frame is cleared. on = 0 returns to the serial frame graph.
 * Reallocates the view's scratch (a second set of records, table and tile
 * stamps) and synchronises. A view whose splat was left on auto switches to
 * the binned splat (auto shapes); MM_ERR_UNSUPPORTED when the direct splat
 * was asked for; mm_set_tuning to a direct splat is refused while it is on.
 * On failure the view keeps its mode and tuning, as mm_set_tuning. */
mm_status mm_set_frame_overlap(mm_view view, uint32_t on);

/* Overlapped views: draws the frame of the last mm_step_render (the pending
 * frame) and makes the instance stream wait for it, so the frame buffer
 * holds the last frame for work after it in stream order. Does not
 * synchronise the host. A no-op for views without overlap. */
mm_status mm_flush_frame(mm_view view);

/* *dev_rgba receives the device address of the view's frame (width *
 * height uint32). It stays valid until the view is destroyed; its content
 * is that of the last frame in stream order (with frame overlap, of the
 * last frame drawn: call mm_flush_frame before reading it on the stream). */
mm_status mm_frame_device_ptr(mm_view view, const uint32_t** dev_rgba);

/* Copies the frame to host memory (bytes >= width * height * 4) after all
 * enqueued work (with frame overlap: the last frame drawn; the pending frame
 * is drawn by mm_flush_frame or the next mm_step_render). Synchronises. */
mm_status mm_read_frame(mm_view view, void* host_rgba, size_t bytes);

/* Splat strategy of a view (all give the same frames, bit for bit).
 *  MM_SPLAT_DIRECT: 64-bit atomicMin of each point's key into a full-screen
 *    key buffer (skipped when a plain load already shows a smaller key),
 *    then a resolve pass over the screen.
 *  MM_SPLAT_BINNED: each workgroup sorts its points by screen tile in LDS
 *    and writes 8-byte records; then `splits` workgroups per tile take the
 *    per-pixel minimum of their share in LDS, a merge pass combines them and
 *    writes RGBA8 directly (3x3 footprints merge tile seams in a last pass;
 *    a 1x1 footprint with one split resolves each tile in the same pass).
 *    No global atomics.
 *  MM_SPLAT_AUTO: direct for a cloud of at most 2^18 points on a screen of
 *    at most 2^21 pixels (the binned path's fixed cost per frame dominates
 *    there), else binned when the screen fits the tile table, else direct. */
#define MM_SPLAT_AUTO 0u
#define MM_SPLAT_DIRECT 1u
#define MM_SPLAT_BINNED 2u

typedef struct {
    uint32_t splat;             /* MM_SPLAT_* */
    uint32_t tile;              /* binned tile side: 16, 32 or 64 pixels; 0 = auto */
    uint32_t points_per_thread; /* binned: 4, 8 or 16 points per bin thread; 0 = auto */
    uint32_t splits;            /* binned: workgroups per tile in the depth test, 1, 2, 4
                                   or 8 (each takes a share of the points); with the 1x1
                                   footprint, 1 resolves each tile in the same pass (no
                                   merge pass); 0 = auto (1x1: 1; 3x3: 2 from 256 bin
                                   workgroups, else 1) */
    uint32_t bin_threads;       /* binned: threads of a bin workgroup, 256, 512 or 1024
                                   (a chunk is bin_threads * points_per_thread points);
                                   0 = auto */
    uint32_t piece_records;     /* binned: 1024 .. 2^20 balances the depth test by
                                   load: every tile is cut into pieces of about this
                                   many records (at least points / 65535), taken by a
                                   persistent grid; MM_PIECES_STATIC: `splits`
                                   workgroups per tile; 0 = auto (static when
                                   splits is set or below 8192 bin workgroups,
                                   else balanced by load) */
    uint32_t occlusion_cull;    /* binned 3D views with the 1x1 footprint, one static
                                   split per tile and no frame overlap: MM_CULL_ON drops
                                   the records that points of the same frame provably
                                   hide. The points that won each pixel in the previous
                                   frame are moved and projected as this frame's are;
                                   a record deeper than such a point at its pixel's 8x8
                                   block cannot win. Frames are unchanged; fewer records
                                   are written and read. MM_CULL_OFF: every record is
                                   kept. 0 = auto (off). With ON and bin_threads /
                                   points_per_thread left 0, a bin workgroup is 512
                                   threads of 16 points. mm_get_tuning reports ON or
                                   OFF. */
} mm_tuning;

#define MM_PIECES_STATIC 0xFFFFFFFFu
#define MM_CULL_AUTO 0u
#define MM_CULL_ON 1u
#define MM_CULL_OFF 2u

/* Chooses the splat strategy and its shape for later frames; reallocates the
 * view's scratch buffers and rebuilds its graph. Synchronises. Returns
 * MM_ERR_UNSUPPORTED for a shape the screen cannot use (more than 4096 tiles, or
 * a bin workgroup whose LDS, 8 * bin_threads * points_per_thread + 4 * (tiles + 1)
 * bytes, exceeds 160 KiB). On any failure the view keeps the tuning it had;
 * only if that tuning's scratch cannot be had again either is the view left
 * without a splat (its frames then return MM_ERR_INVALID_ARG) until a later
 * mm_set_tuning succeeds. */
mm_status mm_set_tuning(mm_view view, const mm_tuning* tuning);

/* The resolved strategy and shape in use (never MM_SPLAT_AUTO; fields a
 * strategy does not use are 0: splits when balanced by load, piece_records
 * is MM_PIECES_STATIC with static splits). */
mm_status mm_get_tuning(mm_view view, mm_tuning* out);

/* Autotuning: times every supported strategy and shape on `frames` whole
 * frames (mm_step_render with step 0, after one warm-up frame; frames in
 * [1, 1000]) and keeps the fastest, which *out receives (resolved). The
 * positions are saved first and restored afterwards, so the cloud is left as
 * it was; the frame holds the last timed frame. When the environment
 * variable MM_TUNE_CACHE names a file, a shape found before for the same
 * device architecture, point count, screen, domain and footprint is taken
 * from it without timing, and new results are appended to it.
 * Synchronises. */
mm_status mm_autotune(mm_view view, uint32_t frames, mm_tuning* out);

/* Per-kernel timing of the next frames, for measurement. mm_profile_begin
 * makes the view's next `capacity` calls of mm_step_render record HIP
 * events inside the frame graph: before and after the point pass (displace,
 * project and splat or bin: the direct point kernel or the bin kernel) and
 * after the last node. mm_profile_end synchronises and writes, per recorded
 * frame k, the point pass time splat_ms[k], the time of the remaining
 * passes (resolve, or tile + seam) resolve_ms[k] and the whole frame graph
 * frame_ms[k] (arrays of `capacity`, any may be NULL),
 * and *count; recording then stops. */
mm_status mm_profile_begin(mm_view view, uint32_t capacity);

/* Sampling of the profile: from the next mm_profile_begin on, events are
 * recorded on the first of every `every` calls (1 <= every <= 1000; default
 * 1, every call) and the other calls launch the plain graph. Re-pointing the
 * timed graph's event nodes costs host time per recorded frame; sampling
 * keeps that cost out of the rate of a tight frame loop. */
mm_status mm_profile_every(mm_view view, uint32_t every);
mm_status mm_profile_end(mm_view view, float* splat_ms, float* resolve_ms, float* frame_ms,
                         uint32_t* count);

/* Frame marks, for the latency of every frame of a loop: from
 * mm_mark_begin on, each of the next `capacity` calls of mm_step_render
 * marks its frame: the frame's first kernel stores the device's constant-rate
 * clock (wall_clock64) as it starts, from inside the frame graph, so a mark
 * adds no work to the stream between frames. mm_mark_end stops marking; if
 * marks are left it enqueues one more after the last frame (drawing a
 * pending overlapped frame first). It does not wait. mm_mark_read waits for
 * the stream and writes to interval_ms (an array of `capacity` - 1; may be
 * NULL) the time between consecutive marks: frame k's span on the device,
 * from the start of frame k to the start of the next frame (or the closing
 * mark), idle gaps included, and to *count the number of intervals;
 * MM_ERR_HIP if a mark was not written. A loop of K frames takes capacity
 * K + 1. 2 <= capacity <= 2^20. */
mm_status mm_mark_begin(mm_view view, uint32_t capacity);
mm_status mm_mark_end(mm_view view);
mm_status mm_mark_read(mm_view view, float* interval_ms, uint32_t* count);

/* ------------------------------------------------------- structured grids
 * The paper's voxel view of a 2D structured domain (section "Potts model":
 * an L x L lattice drawn from the simulation's cell array, its states mapped
 * to colours): a cols x rows lattice of cells fills the screen, and the
 * pixel whose centre lies in cell (cx, cy) takes the palette entry of that
 * cell's value. Cell column of pixel column px: floor((px + 1/2) * cols /
 * width); cell row of pixel row py (row 0 at the top): floor((height - 1 -
 * py + 1/2) * rows / height), so cell row 0 is the bottom row, as y points
 * up in the point views. A value at or past palette_size draws 0. */
typedef struct {
    uint32_t cols, rows;    /* lattice cells, each in [1, 65536] */
    uint32_t width, height; /* screen, each even and in [2, 16384] */
    mm_alloc palette;       /* RGBA8 entries (uint32, stored as given) */
    uint32_t palette_size;  /* >= 1 */
    mm_alloc indices;       /* cols * rows unsigned cell values of index_size bytes,
                               row-major from the bottom row; read at every render */
    uint32_t index_size;    /* 1, 2 or 4 */
} mm_grid_desc;

/* Creates a grid view with a zeroed RGBA8 frame of its own; it keeps both
 * allocations in use until destroyed. */
mm_status mm_create_grid(mm_instance inst, const mm_grid_desc* desc, mm_grid* out);
/* Frees the frame after the instance stream has drained. */
mm_status mm_destroy_grid(mm_grid grid);
/* Draws the current cell values into the frame (one kernel on the instance
 * stream; no host synchronisation). */
mm_status mm_grid_render(mm_grid grid);
mm_status mm_grid_frame_device_ptr(mm_grid grid, const uint32_t** dev_rgba);
/* Copies the frame to host memory (bytes >= width * height * 4); synchronises. */
mm_status mm_grid_read_frame(mm_grid grid, void* host_rgba, size_t bytes);

/* ------------------------------------------------------------------ edges
 * The paper's edge views (triangle meshes, the Delaunay edges of its colloid
 * sample): segments between indexed vertices of a point cloud, depth-tested
 * with the same (depth bits << 32 | id) minimum as points and resolved with
 * the hash colour of the winning edge id. Segment e from vertex a to b: both
 * must pass the near test of the point projection; with (dx, dy, dw) the
 * screen and clip-w differences b - a, it takes n = ceil(max(|dx|, |dy|))
 * steps (at most 32768) and samples t = k / n, k = 0..n (t = 0 alone when
 * n = 0): x = ax + t dx, y = ay + t dy, w = aw + t dw in binary32, each
 * rounded as written; every sample on the screen keys its pixel like a point
 * (2D: depth bits 0). Edge ids: pair e, or side j of triangle t as 3t + j
 * (joining its vertices j and (j + 1) mod 3). A vertex index past the vertex
 * count skips the segment. */
typedef struct {
    mm_alloc position;               /* vertices, AoS, as a view's positions */
    uint64_t element_count;          /* vertices, 1 .. 2^32 - 1 */
    mm_format format;
    mm_domain domain;
    mm_alloc indices;                /* uint32 vertex indices, primitive_count * vpp */
    uint64_t primitive_count;        /* pairs or triangles (edge ids must fit 32 bits) */
    uint32_t vertices_per_primitive; /* 2: vertex pairs, 3: triangles */
    uint32_t width, height;          /* screen, each even and in [2, 16384] */
    uint64_t seed;                   /* key of the colour hash */
    float view_proj[16];             /* row-major float32 clip-from-world; 3D only */
} mm_edges_desc;

/* Creates an edges view with its own key buffer and RGBA8 frame; it keeps
 * both allocations in use until destroyed. */
mm_status mm_create_edges(mm_instance inst, const mm_edges_desc* desc, mm_edges* out);
mm_status mm_destroy_edges(mm_edges view);
mm_status mm_edges_set_camera(mm_edges view, const float view_proj[16]);
/* Draws the segments of the current vertex positions and indices (two
 * kernels on the instance stream: segments, then resolve). */
mm_status mm_edges_render(mm_edges view);
mm_status mm_edges_frame_device_ptr(mm_edges view, const uint32_t** dev_rgba);
/* Copies the frame to host memory (bytes >= width * height * 4); synchronises. */
mm_status mm_edges_read_frame(mm_edges view, void* host_rgba, size_t bytes);

/* ----------------------------------------------------------------- batches
 * Many point clouds, each drawn into one or more views, rendered together
 * with one launch per pass of the binned splat (the per-frame loop of
 * section "Synchronization" over many views at once). A bin work item is a
 * chunk of one cloud: it is displaced once and then binned into every view
 * of its cloud. Each (cloud, view) frame is bit-identical to the frame of a
 * plain view (mm_view_desc with the cloud's fields and the view's screen
 * and camera) after the same steps. */
typedef struct {
    mm_alloc position;      /* element_count points, AoS; no two clouds of a batch
                               may share an alloc */
    uint64_t element_count; /* 1 <= N <= 2^32 - 1; N * stride must fit the alloc */
    mm_format format;       /* MM_FLOAT2 with MM_DOMAIN_2D, MM_FLOAT3 with MM_DOMAIN_3D */
    uint64_t seed;          /* key of the displacement draw and of the colour hash */
    float amplitude;        /* as mm_view_desc.amplitude */
    int32_t wrap;           /* as mm_view_desc.wrap */
} mm_cloud_desc;

typedef struct {
    uint32_t cloud;         /* index into mm_batch_desc.clouds */
    uint32_t width;         /* even, in [2, 16384]; at most 4096 tiles of 64 px */
    uint32_t height;
    float view_proj[16];    /* row-major float32 clip-from-world matrix; 3D only */
} mm_batch_view_desc;

typedef struct {
    mm_domain domain;       /* of every cloud */
    uint32_t footprint;     /* marker side of every view: 1 or 3 */
    uint32_t n_clouds;      /* >= 1 */
    const mm_cloud_desc* clouds;
    uint32_t n_views;       /* >= 1; a cloud may have no view (it is only displaced) */
    const mm_batch_view_desc* views;
} mm_batch_desc;

/* Creates a batch: validates desc, allocates one RGBA8 frame (zero) per view
 * and the binned-splat scratch of every view, writes the work tables to
 * device memory and builds the batch's frame graph. Views are addressed by
 * their index in desc->views. The batch refers to the clouds' allocs until
 * destroyed. */
mm_status mm_create_batch(mm_instance inst, const mm_batch_desc* desc, mm_batch* out);

/* Frees the batch (after the stream has drained). */
mm_status mm_destroy_batch(mm_batch batch);

/* Replaces the camera of view `view` for later frames. */
mm_status mm_batch_set_camera(mm_batch batch, uint32_t view, const float view_proj[16]);

/* Replaces the cameras of views first .. first + count - 1 from count
 * consecutive row-major 4x4 matrices (16 * count floats). */
mm_status mm_batch_set_cameras(mm_batch batch, uint32_t first, uint32_t count,
                               const float* view_proj);

/* One frame of the whole batch: every cloud is displaced with `step`, then
 * every view is splatted and resolved. One graph launch (after a small
 * host-to-device copy of the per-frame cameras and steps). */
mm_status mm_batch_step_render(mm_batch batch, uint32_t step);

/* Render only (no displacement), launched kernel by kernel. */
mm_status mm_batch_render(mm_batch batch);

/* Device address of view `view`'s frame, valid until the batch is destroyed. */
mm_status mm_batch_frame_device_ptr(mm_batch batch, uint32_t view, const uint32_t** dev_rgba);

/* Copies view `view`'s frame to host memory (bytes >= width * height * 4).
 * Synchronises. */
mm_status mm_batch_read_frame(mm_batch batch, uint32_t view, void* host_rgba, size_t bytes);

typedef struct {
    uint32_t tile;              /* tile side of every view: 16, 32 or 64; 0 = auto */
    uint32_t points_per_thread; /* 4, 8 or 16; 0 = auto */
    uint32_t splits;            /* workgroups per tile: 1, 2, 4 or 8 for every view;
                                   0 = per view by its cloud's points per tile
                                   (n / tiles: 2 from 4096 or from 256 bin
                                   workgroups, 4 from 8192, 8 from 16384) */
    uint32_t grid_blocks;       /* 0: one workgroup per work item; else a persistent
                                   grid of that many workgroups per pass, each
                                   looping over work items */
    uint32_t bin_threads;       /* 256, 512 or 1024; 0 = auto */
} mm_batch_tuning;

/* Chooses the shape for later frames; reallocates scratch and rebuilds the
 * graph. Synchronises. On failure the batch keeps the shape it had (or, if
 * that cannot be set up again, has none until a later call succeeds). */
mm_status mm_batch_set_tuning(mm_batch batch, const mm_batch_tuning* tuning);
mm_status mm_batch_get_tuning(mm_batch batch, mm_batch_tuning* out);

/* Autotuning of a batch, as mm_autotune: every supported tile, points per
 * thread, splits and grid shape is timed on `frames` whole batch frames and
 * the fastest is kept; every cloud's positions are restored afterwards.
 * The cache key is the device architecture and a hash of the cloud sizes,
 * the views' clouds and screens, the domain and the footprint. */
mm_status mm_batch_autotune(mm_batch batch, uint32_t frames, mm_batch_tuning* out);

/* Frame timing of the next `capacity` calls of mm_batch_step_render: HIP
 * events before the per-frame upload and after the frame graph. */
mm_status mm_batch_profile_begin(mm_batch batch, uint32_t capacity);
mm_status mm_batch_profile_end(mm_batch batch, float* frame_ms, uint32_t* count);

/* ------------------------------------------------------------------ server
 * Served rendering (the remote-rendering direction the paper names as
 * future work, section "Conclusions and limitations"): clients submit
 * requests (session, cloud, camera, screen); a scheduler thread packs the
 * pending requests of many sessions into batched launches (continuous
 * batching over a few streams) and admits a session only while its frame
 * buffer fits the memory budget.
 *
 * Order and results: every cloud added to the server has a step counter.
 * Requests on one cloud are served in submission order, and the k-th
 * request on a cloud (k from 0) displaces the cloud with step k and then
 * renders it. Its frame therefore equals the plain frame of that cloud
 * after steps 0..k, whatever else is queued or in flight.
 *
 * Streams: up to two launches are in flight on each stream. A cloud's (or
 * a session's) requests in flight are all on one stream, and its next
 * request goes into the next launch on that stream, behind the previous one
 * in stream order, so saturated clouds share every launch while the next
 * one is prepared on the host. Requests with nothing in flight go to a
 * stream that is idle, so independent requests run side by side.
 *
 * A session's frame buffer is its RGBA8 frame (4 B per pixel) plus the
 * per-tile scratch of the depth test; its screen is fixed by its first
 * request. It is held from admission until the session is closed, or until
 * the scheduler evicts it (least recently used first) while it is idle and
 * the budget is needed by a waiting session; an evicted session's frame is
 * lost. A session evicted with requests still queued is admitted again
 * when its next request's turn comes.
 *
 * Failure: if a launch fails (or cannot be sent), or a frame buffer within
 * the budget cannot be allocated even after every other one is given up,
 * the server stops scheduling: that launch's requests and every queued one
 * are dropped (mm_server_poll and mm_server_wait return an error for them,
 * stats.dropped counts them) and later submissions fail with MM_ERR_HIP.
 * The server's calls may come from any thread. */
typedef struct {
    uint64_t fb_budget_bytes;   /* frame-buffer bytes the admitted sessions may hold */
    uint32_t streams;           /* streams the launches run on: 1..4 (two launches each) */
    uint32_t max_batch;         /* requests per launch: 1..4096 */
    mm_domain domain;           /* of every cloud */
    uint32_t footprint;         /* 1 or 3 */
    mm_batch_tuning tuning;     /* tile (0: 64), points_per_thread (0: 16), splits,
                                   grid_blocks, bin_threads (0: 256) */
} mm_server_desc;

typedef struct {
    uint64_t submitted;
    uint64_t completed;          /* requests whose frame is complete */
    uint64_t launches;
    uint64_t admitted_sessions;  /* sessions holding a frame buffer now */
    uint64_t admissions, evictions;
    uint64_t fb_bytes_in_use;    /* held by admitted sessions and kept for reuse */
    uint64_t queued;             /* submitted, not yet launched */
    uint64_t dropped;            /* requests that will not complete (failure, shutdown) */
    uint64_t max_in_flight;      /* most launches sent and not yet retired at one time */
    uint64_t max_batch;          /* most requests in one launch */
} mm_server_stats;

/* Creates the server and starts its scheduler thread. Its streams are
 * created by the server (default priority, non-blocking). */
mm_status mm_create_server(mm_instance inst, const mm_server_desc* desc, mm_server* out);

/* Stops the scheduler after the launches in flight; queued requests are
 * dropped. Frees every buffer of the server. */
mm_status mm_destroy_server(mm_server server);

/* Registers a cloud (the server refers to its alloc until destroyed);
 * *cloud_id receives its index (0, 1, ...). Its step counter starts at 0. */
mm_status mm_server_add_cloud(mm_server server, const mm_cloud_desc* cloud, uint32_t* cloud_id);

/* Queues one displace+render request and returns at once. dev_out: NULL
 * renders into the session's frame; else the device address of width *
 * height uint32 owned by the caller, which receives the frame instead.
 * MM_ERR_BUDGET if the session's frame buffer alone exceeds the budget;
 * MM_ERR_INVALID_ARG for a screen other than the session's. */
mm_status mm_server_submit(mm_server server, uint32_t session, uint32_t cloud,
                           const float view_proj[16], uint32_t width, uint32_t height,
                           uint32_t* dev_out, uint64_t* request_id);

/* *done = 1 once the request's frame is complete on the device, with
 * *latency_s the time from submission to completion (may be NULL). */
mm_status mm_server_poll(mm_server server, uint64_t request_id, int32_t* done,
                         double* latency_s);

/* Blocks until the request is complete. MM_ERR_NOT_READY if it will not
 * complete: the server stopped, or failed (see below). */
mm_status mm_server_wait(mm_server server, uint64_t request_id, double* latency_s);

/* Copies the session's frame (its last completed request drawn into it) to
 * host memory. MM_ERR_NOT_READY if the session holds no frame buffer. */
mm_status mm_server_read_frame(mm_server server, uint32_t session, void* host_rgba,
                               size_t bytes);

/* The session's frame buffer is released once its queued requests are done. */
mm_status mm_server_close_session(mm_server server, uint32_t session);

mm_status mm_server_stats_get(mm_server server, mm_server_stats* out);

/* ------------------------------------------------- frames that allocate nothing
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): one frame of the
 * direct splat (as mm_step_render with MM_SPLAT_DIRECT) on the caller's
 * positions, frame and stream, with no instance, view or allocation. The
 * per-pixel depth keys live in a file-scope device array of 2^22 keys
 * (32 MiB, held by every device the library runs on until the process
 * ends), so width * height may not exceed 2^22 (MM_ERR_BUDGET). The first
 * call on a device fills the keys with the empty key; every frame leaves
 * them empty. All calls on one device share the array: calls that overlap
 * on a device (two streams, or two threads) race and may draw each other's
 * points. Calls no hipMalloc or hipFree. Returns once the work is enqueued
 * on `stream` (NULL: the null stream) of the current device. */
typedef struct {
    void* dev_positions;    /* element_count AoS points, displaced in place */
    uint64_t element_count; /* 1 <= N <= 2^32 - 1 */
    mm_domain domain;       /* MM_DOMAIN_2D: float2, MM_DOMAIN_3D: float3 */
    uint32_t width;         /* even, in [2, 16384], width * height <= 2^22 */
    uint32_t height;
    uint32_t footprint;     /* 1 or 3 */
    uint64_t seed;          /* as mm_view_desc */
    float amplitude;
    int32_t wrap;
    uint32_t step;          /* displacement step of this frame */
    float view_proj[16];    /* row-major clip-from-world; 3D only */
    uint32_t* dev_rgba;     /* width * height RGBA8 words, written */
    void* stream;           /* hipStream_t */
} mm_static_frame_desc;

mm_status mm_step_render_static(const mm_static_frame_desc* desc);

/* ---------------------------------------------------------------- testing
 * For tests of the error paths: the next `after` device or pinned host
 * allocations the library makes succeed and the one after them fails as if
 * memory were short (MM_ERR_OUT_OF_MEMORY from the call that made it), once;
 * negative: no allocation is made to fail (the default). Process-wide. */
mm_status mm_debug_fail_allocations(int64_t after);

/* ------------------------------------------------------------ diagnostics */
const char* mm_status_string(mm_status status);
const char* mm_last_error(void);
/* Library version as major * 10000 + minor * 100 + patch. */
int32_t mm_version(void);

#ifdef __cplusplus
}
#endif
#endif
