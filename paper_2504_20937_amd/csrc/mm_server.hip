// Served rendering: a scheduler thread packs the requests of many sessions
// into batched binned-splat launches on a few streams (continuous batching),
// admits sessions by frame-buffer bytes, and serves every cloud's requests in
// submission order.
//
// Per launch, at most one request per cloud (its displacement step must
// follow the previous request's) and per session (one frame buffer). Views
// are full-clear: a session's frame buffer carries no frame-to-frame tile
// history, so every tile not drawn is cleared. Per-cloud scratch (records
// and table rows) lives with the cloud, per-view scratch with the session.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mm_batch.h"
#include "mm_sched.h"

using namespace mmh;

namespace {

struct FrameBuf {
    uint32_t width = 0, height = 0;
    uint64_t bytes = 0;
    void* base = nullptr;  // one allocation, split below
    uint32_t* colour = nullptr;
    uint64_t* part = nullptr;
    uint64_t* border = nullptr;
    uint64_t* apron = nullptr;
    uint32_t* active = nullptr;
    bool fresh = false;    // new memory: its tile stamps are zeroed by its first launch
    // Stamp of the launch that drew its frame (0: none, or the frame is not
    // known to be whole). Every tile is then either drawn by that launch or
    // clear, so the next frame clears only the tiles drawn then and not now
    // instead of every tile it does not draw.
    uint32_t last_stamp = 0;
};

struct SCloud {
    mm::CloudArgs args{};
    uint64_t n = 0;
    mm_alloc alloc = nullptr;
    uint32_t num_wg = 0;
    uint64_t* seg = nullptr;
    uint16_t* table = nullptr;
};

using Sched = mms::Scheduler<FrameBuf>;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char* dev = nullptr;   // device copy of the table images
    size_t dev_bytes = 0;
    unsigned char* pinned = nullptr;   // host-coherent staging of the table images
    void* pinned_dev = nullptr;        // its device address
    size_t pinned_bytes = 0;
    uint32_t* stamp_slot = nullptr;
    mmb::TableImage img;
    mm::BatchBinArgs b{};
    mm::BatchTileArgs t{}, m{};
    std::vector<mmb::Node> nodes;
};

}  // namespace

struct mm_server_s : Sched::Backend {
    mm_instance inst = nullptr;
    mm_server_desc desc{};
    uint32_t side = 64, shift = 6, ppt = 16, threads = 256, P = 4096, splits_cap = 2;
    std::mutex mu;
    std::condition_variable cv;     // scheduler wake-up
    std::condition_variable done_cv;  // request completion
    std::thread worker;
    bool stop = false;
    std::vector<SCloud> clouds;
    std::vector<hipStream_t> streams;
    std::vector<Slot> slots;  // kSlotsPerStream per stream, slot k on stream k / kSlotsPerStream
    Sched* sched = nullptr;
    uint32_t stamp = 0;
    uint32_t* stamps = nullptr;     // one device word per slot
    // Two launches can be queued on a stream: the next one is packed and
    // staged on the host while the previous one runs, and takes the clouds
    // in flight there (stream order runs their steps one after the other).
    static constexpr uint32_t kSlotsPerStream = 2;

    uint64_t fb_bytes(uint32_t w, uint32_t h) const override;
    bool alloc_buf(uint32_t w, uint32_t h, FrameBuf& out) override;
    void free_buf(FrameBuf& b) override;
    bool launch(uint32_t slot, const std::vector<Sched::Item>& items) override;
    int query(uint32_t slot) override;
    mm_status launch_slot(Slot& slot, const std::vector<Sched::Item>& items);
    void run();
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

uint64_t mm_server_s::fb_bytes(uint32_t w, uint32_t h) const {
    const uint64_t nt = tiles_of(w, h, side);
    const uint64_t a = desc.footprint == 3 ? side + 2 : side;
    uint64_t b = align_up(static_cast<uint64_t>(w) * h * 4, 256);
    b += align_up(nt * splits_cap * a * a * 8, 256);
    b += align_up(nt * 4, 256);
    if (desc.footprint == 3) {
        b += align_up(nt * 4 * side * 8, 256);
        b += align_up(nt * (4 * side + 4) * 8, 256);
    }
    return b;
}

bool mm_server_s::alloc_buf(uint32_t w, uint32_t h, FrameBuf& out) {
    FrameBuf b;
    b.width = w;
    b.height = h;
    b.bytes = fb_bytes(w, h);
    hipError_t e = dev_malloc(&b.base, b.bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        hip_fail(e, "server: allocating a frame buffer");
        return false;
    }
    const uint64_t nt = tiles_of(w, h, side);
    const uint64_t a = desc.footprint == 3 ? side + 2 : side;
    unsigned char* p = static_cast<unsigned char*>(b.base);
    b.colour = reinterpret_cast<uint32_t*>(p);
    p += align_up(static_cast<uint64_t>(w) * h * 4, 256);
    b.part = reinterpret_cast<uint64_t*>(p);
    p += align_up(nt * splits_cap * a * a * 8, 256);
    b.active = reinterpret_cast<uint32_t*>(p);
    p += align_up(nt * 4, 256);
    if (desc.footprint == 3) {
        b.border = reinterpret_cast<uint64_t*>(p);
        p += align_up(nt * 4 * side * 8, 256);
        b.apron = reinterpret_cast<uint64_t*>(p);
    }
    // the tile stamps must read older than any launch's stamp: the first
    // launch drawing into this buffer zeroes them on its own stream (a
    // synchronous clear here would wait for the launches in flight); the
    // frame and the partial tiles are written before they are read
    b.fresh = true;
    out = b;
    return true;
}

void mm_server_s::free_buf(FrameBuf& b) {
    if (b.base) (void)hipFree(b.base);
    b = FrameBuf{};
}

int mm_server_s::query(uint32_t k) {
    const hipError_t q = hipEventQuery(slots[k].done);
    if (q == hipErrorNotReady) return 0;
    if (q == hipSuccess) return 1;
    fail(MM_ERR_HIP, "server: a launch failed: %s", hipGetErrorString(q));
    return -1;
}

bool mm_server_s::launch(uint32_t k, const std::vector<Sched::Item>& items) {
    Slot& sl = slots[k];
    if (launch_slot(sl, items) == MM_OK) return true;
    (void)hipStreamSynchronize(sl.stream);
    return false;
}

mm_status mm_server_s::launch_slot(Slot& sl, const std::vector<Sched::Item>& items) {
    if (stamp + 1u == 0u) {
        // every older stamp must read as "not this launch": once no launch
        // reads them, clear all of them; each buffer's next frame then clears
        // every tile it does not draw
        for (hipStream_t st : streams) MM_HIP(hipStreamSynchronize(st));
        mm_status st = MM_OK;
        sched->for_each_buf([&](FrameBuf& b) {
            const hipError_t e = hipMemset(b.active, 0, tiles_of(b.width, b.height, side) * 4);
            if (e != hipSuccess && st == MM_OK) st = hip_fail(e, "server: resetting tile stamps");
            b.last_stamp = 0;
        });
        MM_TRY(st);
        stamp = 0;
    }
    const uint32_t launch_stamp = stamp + 1u;
    std::vector<mmb::Cloud> cl;
    std::vector<mmb::PlanView> views;
    for (const Sched::Item& it : items) {
        const Sched::Request& r = *it.req;
        const SCloud& c = clouds[r.cloud];
        const FrameBuf& buf = it.session->buf;
        mmb::Cloud x;
        x.args = c.args;
        x.args.step = r.step;
        x.n = c.n;
        cl.push_back(x);
        mmb::PlanView v;
        v.cloud = static_cast<uint32_t>(cl.size() - 1);
        v.width = r.width;
        v.height = r.height;
        std::memcpy(v.view_proj, r.m, sizeof v.view_proj);
        // a request into the caller's buffer, a 3x3 footprint (whose edges
        // the seam pass writes across tile borders) or a buffer without a
        // known frame: every tile not drawn is cleared
        v.full_clear = r.dev_out != nullptr || desc.footprint == 3 || buf.last_stamp == 0;
        v.prev_stamp = v.full_clear ? 0u : buf.last_stamp;
        v.colour = r.dev_out ? r.dev_out : buf.colour;
        v.seg = c.seg;
        v.table = c.table;
        v.part = buf.part;
        v.border = buf.border;
        v.apron = buf.apron;
        v.active = buf.active;
        views.push_back(v);
    }
    // frame buffers hold splits_cap partial blocks per tile (fb_bytes)
    mmb::shape_views(views, cl, side, P, desc.tuning.splits, splits_cap);
    for (const mmb::PlanView& v : views)
        if (v.splits > splits_cap)
            return fail(MM_ERR_HIP, "server: %u splits for a frame buffer of %u", v.splits, splits_cap);
    MM_TRY(mmb::build_tables(cl, views, P, desc.footprint, sl.img));
    const size_t stat = sl.img.stat.size(), frame = sl.img.frame.size();
    const size_t total = stat + frame;
    if (total > sl.dev_bytes) {
        if (sl.dev) (void)hipFree(sl.dev);
        sl.dev = nullptr;
        sl.dev_bytes = 0;
        MM_HIP(dev_malloc(reinterpret_cast<void**>(&sl.dev), total * 2));
        sl.dev_bytes = total * 2;
    }
    if (total > sl.pinned_bytes) {
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        sl.pinned_dev = nullptr;
        sl.pinned_bytes = 0;
        MM_HIP(pinned_malloc(reinterpret_cast<void**>(&sl.pinned), total * 2));
        MM_HIP(hipHostGetDevicePointer(&sl.pinned_dev, sl.pinned, 0));
        sl.pinned_bytes = total * 2;
    }
    for (const Sched::Item& it : items) {
        FrameBuf& b = it.session->buf;
        if (!b.fresh) continue;
        MM_HIP(hipMemsetAsync(b.active, 0, tiles_of(b.width, b.height, side) * 4, sl.stream));
        b.fresh = false;
    }
    std::memcpy(sl.pinned, sl.img.stat.data(), stat);
    std::memcpy(sl.pinned + stat, sl.img.frame.data(), frame);
    // a kernel reads the staged tables: the slot's stream stays on the compute queue
    MM_HIP(mm::launch_upload(sl.dev, sl.pinned_dev, total, sl.stream));
    mmb::bind_args(sl.img, sl.dev, sl.dev + stat, sl.stamp_slot, shift, P, sl.b, sl.t, sl.m);
    stamp = launch_stamp;
    sl.b.stamp = stamp;
    // the session's buffer now holds this frame, unless the frame went to the
    // caller's buffer (the stamps then no longer describe the buffer's frame)
    for (const Sched::Item& it : items) it.session->buf.last_stamp = it.req->dev_out ? 0u : stamp;
    sl.nodes = mmb::make_nodes(desc.domain, desc.footprint, shift, ppt, threads, sl.img,
                               desc.tuning.grid_blocks, &sl.b, &sl.t, &sl.m);
    for (const mmb::Node& n : sl.nodes) MM_HIP(mmh::launch(n.l, n.arg, sl.stream));
    MM_HIP(hipEventRecord(sl.done, sl.stream));
    return MM_OK;
}

void mm_server_s::run() {
    (void)hipSetDevice(inst->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = sched->retire();
        if (progressed) done_cv.notify_all();
        if (stop && !sched->in_flight()) break;
        if (!stop && sched->schedule()) {
            progressed = true;
            done_cv.notify_all();  // a launch that did not go out dropped requests
        }
        if (progressed) continue;
        if (sched->in_flight())
            cv.wait_for(lk, std::chrono::microseconds(20));
        else
            cv.wait(lk, [&] { return stop || (sched->has_pending() && !sched->failed()); });
    }
}

namespace {

mm_status server_ok(mm_server s, const char* what) {
    if (!s) return fail(MM_ERR_INVALID_ARG, "%s: null server", what);
    return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_create_server(mm_instance inst, const mm_server_desc* desc, mm_server* out) {
    if (!inst || !desc || !out) return fail(MM_ERR_INVALID_ARG, "create_server: null argument");
    if (desc->streams < 1 || desc->streams > 4)
        return fail(MM_ERR_INVALID_ARG, "create_server: streams %u outside [1, 4]", desc->streams);
    if (desc->max_batch < 1 || desc->max_batch > 4096)
        return fail(MM_ERR_INVALID_ARG, "create_server: max_batch %u outside [1, 4096]", desc->max_batch);
    if (desc->domain != MM_DOMAIN_2D && desc->domain != MM_DOMAIN_3D)
        return fail(MM_ERR_INVALID_ARG, "create_server: domain %d is not 2D/3D", (int)desc->domain);
    if (desc->footprint != 1 && desc->footprint != 3)
        return fail(MM_ERR_INVALID_ARG, "create_server: footprint %u is not 1 or 3", desc->footprint);
    if (desc->fb_budget_bytes == 0) return fail(MM_ERR_INVALID_ARG, "create_server: zero budget");
    const mm_batch_tuning& t = desc->tuning;
    const uint32_t side = t.tile ? t.tile : 64u;
    const uint32_t ppt = t.points_per_thread ? t.points_per_thread : 16u;
    const uint32_t threads = t.bin_threads ? t.bin_threads : 256u;
    if (!mm::binned_shape_ok(static_cast<int>(shift_of(side)), static_cast<int>(ppt), threads,
                             t.splits == 0 ? 1u : t.splits))
        return fail(MM_ERR_INVALID_ARG, "create_server: tuning %u / %u / %u not supported", side, ppt,
                    t.splits);
    if (t.grid_blocks != 0 && (t.grid_blocks % 8 != 0 || t.grid_blocks > (1u << 20)))
        return fail(MM_ERR_INVALID_ARG, "create_server: grid_blocks %u", t.grid_blocks);
    DeviceGuard guard(inst->device);
    mm_server srv = new (std::nothrow) mm_server_s();
    if (!srv) return fail(MM_ERR_OUT_OF_MEMORY, "create_server: host allocation");
    srv->inst = inst;
    srv->desc = *desc;
    srv->side = side;
    srv->shift = shift_of(side);
    srv->ppt = ppt;
    srv->threads = threads;
    srv->P = threads * ppt;
    srv->splits_cap = t.splits ? t.splits : 2u;
    srv->desc.tuning = mm_batch_tuning{side, ppt, t.splits, t.grid_blocks, threads};
    const uint32_t nslots = desc->streams * mm_server_s::kSlotsPerStream;
    hipError_t e = dev_malloc(reinterpret_cast<void**>(&srv->stamps), 256 * nslots);
    if (e == hipSuccess) e = hipMemset(srv->stamps, 0, 256 * nslots);
    srv->streams.assign(desc->streams, nullptr);
    for (uint32_t k = 0; k < desc->streams && e == hipSuccess; ++k)
        e = hipStreamCreateWithFlags(&srv->streams[k], hipStreamNonBlocking);
    srv->slots.resize(nslots);
    for (uint32_t k = 0; k < nslots && e == hipSuccess; ++k) {
        Slot& sl = srv->slots[k];
        sl.stream = srv->streams[k / mm_server_s::kSlotsPerStream];
        e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        sl.stamp_slot = srv->stamps + 64 * k;
    }
    auto destroy_streams = [srv] {
        for (Slot& sl : srv->slots)
            if (sl.done) (void)hipEventDestroy(sl.done);
        for (hipStream_t st : srv->streams)
            if (st) (void)hipStreamDestroy(st);
    };
    if (e != hipSuccess) {
        destroy_streams();
        if (srv->stamps) (void)hipFree(srv->stamps);
        delete srv;
        return hip_fail(e, "create_server: streams");
    }
    srv->sched = new (std::nothrow)
        Sched(*srv, desc->fb_budget_bytes, nslots, desc->max_batch, mm_server_s::kSlotsPerStream);
    if (!srv->sched) {
        destroy_streams();
        (void)hipFree(srv->stamps);
        delete srv;
        return fail(MM_ERR_OUT_OF_MEMORY, "create_server: host allocation");
    }
    srv->worker = std::thread([srv] { srv->run(); });
    inst->servers.insert(srv);
    *out = srv;
    return MM_OK;
}

mm_status mm_destroy_server(mm_server srv) {
    MM_TRY(server_ok(srv, "destroy_server"));
    mm_instance inst = srv->inst;
    if (!inst->servers.count(srv)) return fail(MM_ERR_INVALID_ARG, "destroy_server: unknown server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->sched->drop_all_queued();
    }
    srv->cv.notify_all();
    srv->worker.join();
    srv->done_cv.notify_all();
    DeviceGuard guard(inst->device);
    for (hipStream_t st : srv->streams) (void)hipStreamSynchronize(st);
    for (Slot& sl : srv->slots) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        (void)hipEventDestroy(sl.done);
    }
    for (hipStream_t st : srv->streams) (void)hipStreamDestroy(st);
    srv->sched->free_all();
    delete srv->sched;
    for (SCloud& c : srv->clouds) {
        if (c.seg) (void)hipFree(c.seg);
        if (c.table) (void)hipFree(c.table);
        c.alloc->users--;
    }
    (void)hipFree(srv->stamps);
    inst->servers.erase(srv);
    delete srv;
    return MM_OK;
}

mm_status mm_server_add_cloud(mm_server srv, const mm_cloud_desc* c, uint32_t* cloud_id) {
    MM_TRY(server_ok(srv, "server_add_cloud"));
    if (!c || !cloud_id) return fail(MM_ERR_INVALID_ARG, "server_add_cloud: null argument");
    MM_TRY(validate_cloud(srv->inst, *c, srv->desc.domain, "server_add_cloud"));
    std::lock_guard<std::mutex> lk(srv->mu);
    for (const SCloud& o : srv->clouds)
        if (o.alloc == c->position)
            return fail(MM_ERR_INVALID_ARG, "server_add_cloud: the alloc is already a cloud of this server");
    DeviceGuard guard(srv->inst->device);
    SCloud sc;
    sc.args = cloud_args(c->position->ptr, c->element_count, c->seed, c->amplitude);
    sc.args.fold_lim = c->wrap ? 1.0f : std::numeric_limits<float>::infinity();
    sc.n = c->element_count;
    sc.alloc = c->position;
    sc.num_wg = static_cast<uint32_t>((c->element_count + srv->P - 1) / srv->P);
    hipError_t e = alloc_n(&sc.seg, static_cast<uint64_t>(sc.num_wg) * srv->P);
    if (e == hipSuccess) e = alloc_n(&sc.table, static_cast<uint64_t>(sc.num_wg) * (kMaxTiles + 1));
    if (e != hipSuccess) {
        if (sc.seg) (void)hipFree(sc.seg);
        return hip_fail(e, "server_add_cloud: scratch");
    }
    c->position->users++;
    srv->clouds.push_back(std::move(sc));
    *cloud_id = srv->sched->add_cloud();
    return MM_OK;
}

mm_status mm_server_submit(mm_server srv, uint32_t session, uint32_t cloud, const float m[16],
                           uint32_t width, uint32_t height, uint32_t* dev_out, uint64_t* request_id) {
    MM_TRY(server_ok(srv, "server_submit"));
    if (!m || !request_id) return fail(MM_ERR_INVALID_ARG, "server_submit: null argument");
    MM_TRY(validate_screen(width, height, "server_submit"));
    if (srv->desc.domain == MM_DOMAIN_3D) MM_TRY(validate_camera(m, "server_submit"));
    if (tiles_of(width, height, srv->side) > kMaxTiles)
        return fail(MM_ERR_UNSUPPORTED, "server_submit: %ux%u needs more than %u tiles of %u px", width,
                    height, kMaxTiles, srv->side);
    if (dev_out) {
        // the output must be device memory of this device, large enough
        DeviceGuard guard(srv->inst->device);
        hipPointerAttribute_t attr{};
        hipDeviceptr_t base = nullptr;
        size_t range = 0;
        if (hipPointerGetAttributes(&attr, dev_out) != hipSuccess || attr.type != hipMemoryTypeDevice ||
            attr.device != srv->inst->device || hipMemGetAddressRange(&base, &range, dev_out) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MM_ERR_INVALID_ARG, "server_submit: dev_out %p is not device memory", (void*)dev_out);
        }
        const uintptr_t lo = reinterpret_cast<uintptr_t>(base), p0 = reinterpret_cast<uintptr_t>(dev_out);
        if (p0 % 4 != 0 || static_cast<uint64_t>(width) * height * 4 > range - (p0 - lo))
            return fail(MM_ERR_INVALID_ARG, "server_submit: dev_out cannot hold a %ux%u frame", width, height);
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop || srv->sched->failed())
            return fail(MM_ERR_HIP, "server_submit: the server has stopped");
        if (cloud >= srv->clouds.size())
            return fail(MM_ERR_INVALID_ARG, "server_submit: cloud %u of %zu", cloud, srv->clouds.size());
        if (srv->fb_bytes(width, height) > srv->desc.fb_budget_bytes)
            return fail(MM_ERR_BUDGET, "server_submit: a %ux%u frame buffer (%llu B) exceeds the budget",
                        width, height, (unsigned long long)srv->fb_bytes(width, height));
        uint64_t id = 0;
        const mm_status st = srv->sched->submit(session, cloud, m, width, height, dev_out, &id);
        if (st == MM_ERR_INVALID_ARG) {
            const Sched::Session* s = srv->sched->session(session);
            return fail(st, "server_submit: session %u is %ux%u, not %ux%u", session, s ? s->width : 0u,
                        s ? s->height : 0u, width, height);
        }
        if (st != MM_OK) return fail(st, "server_submit: refused");
        *request_id = id;
    }
    srv->cv.notify_all();
    return MM_OK;
}

mm_status mm_server_poll(mm_server srv, uint64_t id, int32_t* done, double* latency_s) {
    MM_TRY(server_ok(srv, "server_poll"));
    if (!done) return fail(MM_ERR_INVALID_ARG, "server_poll: null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    const Sched::Request* r = srv->sched->request(id);
    if (!r) return fail(MM_ERR_INVALID_ARG, "server_poll: unknown request %llu", (unsigned long long)id);
    if (r->state == mms::kDropped)
        return fail(MM_ERR_HIP, "server_poll: request %llu was dropped", (unsigned long long)id);
    if (latency_s && r->state == mms::kDone)
        *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    *done = r->state == mms::kDone ? 1 : 0;
    return MM_OK;
}

mm_status mm_server_wait(mm_server srv, uint64_t id, double* latency_s) {
    MM_TRY(server_ok(srv, "server_wait"));
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->sched->request(id))
        return fail(MM_ERR_INVALID_ARG, "server_wait: unknown request %llu", (unsigned long long)id);
    // a failed scheduler drops every queued request, so the state settles
    srv->done_cv.wait(lk, [&] {
        const mms::ReqState st = srv->sched->request(id)->state;
        return st == mms::kDone || st == mms::kDropped || srv->stop;
    });
    const Sched::Request* r = srv->sched->request(id);
    if (r->state != mms::kDone)
        return fail(MM_ERR_NOT_READY, "server_wait: request %llu did not complete", (unsigned long long)id);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    return MM_OK;
}

mm_status mm_server_read_frame(mm_server srv, uint32_t session, void* host_rgba, size_t bytes) {
    MM_TRY(server_ok(srv, "server_read_frame"));
    if (!host_rgba) return fail(MM_ERR_INVALID_ARG, "server_read_frame: null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    Sched::Session* s = srv->sched->session(session);
    if (!s) return fail(MM_ERR_INVALID_ARG, "server_read_frame: unknown session %u", session);
    srv->done_cv.wait(lk, [&] { return s->inflight == 0 || srv->stop; });
    if (!s->admitted) return fail(MM_ERR_NOT_READY, "server_read_frame: session %u holds no frame buffer", session);
    const size_t need = static_cast<size_t>(s->width) * s->height * 4;
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "server_read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(srv->inst->device);
    MM_HIP(hipMemcpy(host_rgba, s->buf.colour, need, hipMemcpyDeviceToHost));
    return MM_OK;
}

mm_status mm_server_close_session(mm_server srv, uint32_t session) {
    MM_TRY(server_ok(srv, "server_close_session"));
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->sched->close_session(session))
        return fail(MM_ERR_INVALID_ARG, "server_close_session: unknown session %u", session);
    srv->cv.notify_all();
    return MM_OK;
}

mm_status mm_server_stats_get(mm_server srv, mm_server_stats* out) {
    MM_TRY(server_ok(srv, "server_stats_get"));
    if (!out) return fail(MM_ERR_INVALID_ARG, "server_stats_get: null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->sched->stats();
    return MM_OK;
}

}  // extern "C"
