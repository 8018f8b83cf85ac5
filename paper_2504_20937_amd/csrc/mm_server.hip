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
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mm_batch.h"

using namespace mmh;
using Clock = std::chrono::steady_clock;

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
};

struct Session {
    uint32_t width = 0, height = 0;
    bool has_screen = false;
    bool admitted = false;
    bool busy = false;      // a request in flight
    bool closing = false;
    uint32_t queued = 0;    // requests submitted, not launched
    uint64_t last_use = 0;  // launch counter when last launched (LRU)
    FrameBuf buf;
};

struct SCloud {
    mm::CloudArgs args{};
    uint64_t n = 0;
    mm_alloc alloc = nullptr;
    uint32_t next_step = 0;
    uint32_t num_wg = 0;
    uint64_t* seg = nullptr;
    uint16_t* table = nullptr;
    bool busy = false;
    std::deque<uint64_t> queue;  // request ids in submission order
};

enum ReqState { kQueued = 0, kInFlight = 1, kDone = 2, kDropped = 3 };

struct Request {
    uint32_t session = 0, cloud = 0, step = 0;
    float m[16] = {};
    uint32_t width = 0, height = 0;
    uint32_t* dev_out = nullptr;
    Clock::time_point t_submit, t_done;
    ReqState state = kQueued;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
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

struct mm_server_s {
    mm_instance inst = nullptr;
    mm_server_desc desc{};
    uint32_t side = 64, shift = 6, ppt = 16, threads = 256, P = 4096, splits_cap = 2;
    std::mutex mu;
    std::condition_variable cv;     // scheduler wake-up
    std::condition_variable done_cv;  // request completion
    std::thread worker;
    bool stop = false;
    bool failed = false;
    std::vector<SCloud> clouds;
    std::unordered_map<uint32_t, Session> sessions;
    std::unordered_map<uint64_t, Request> requests;
    std::deque<uint64_t> pending;   // submission order
    std::multimap<uint64_t, FrameBuf> pool;  // kept for reuse, by (width << 32 | height)
    std::vector<Slot> slots;
    uint64_t held = 0;              // bytes of admitted and pooled frame buffers
    uint64_t next_id = 1;
    uint32_t stamp = 0;
    uint32_t* stamps = nullptr;     // one device word per slot
    mm_server_stats stats{};

    uint64_t fb_bytes(uint32_t w, uint32_t h) const;
    mm_status alloc_buf(uint32_t w, uint32_t h, FrameBuf& out);
    void free_buf(FrameBuf& b);
    bool admit(Session& s);
    void release(Session& s);
    bool retire();
    bool schedule();
    mm_status launch(Slot& slot, const std::vector<uint64_t>& batch);
    void run();
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint64_t screen_key(uint32_t w, uint32_t h) { return (static_cast<uint64_t>(w) << 32) | h; }

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

mm_status mm_server_s::alloc_buf(uint32_t w, uint32_t h, FrameBuf& out) {
    FrameBuf b;
    b.width = w;
    b.height = h;
    b.bytes = fb_bytes(w, h);
    MM_HIP(hipMalloc(&b.base, b.bytes));
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
    // zero frame and tile stamps (older than any launch's stamp)
    const hipError_t e = hipMemset(b.base, 0, b.bytes);
    if (e != hipSuccess) {
        (void)hipFree(b.base);
        return hip_fail(e, "server: clearing a frame buffer");
    }
    out = b;
    return MM_OK;
}

void mm_server_s::free_buf(FrameBuf& b) {
    if (b.base) (void)hipFree(b.base);
    b = FrameBuf{};
}

// Gives s a frame buffer: one kept for reuse at its screen size, else a new
// one once the budget allows (freeing kept buffers of other sizes, then
// evicting idle sessions, least recently used first).
bool mm_server_s::admit(Session& s) {
    const uint64_t need = fb_bytes(s.width, s.height);
    const uint64_t key = screen_key(s.width, s.height);
    for (;;) {
        auto it = pool.find(key);
        if (it != pool.end()) {
            s.buf = it->second;
            pool.erase(it);
            break;
        }
        if (held + need <= desc.fb_budget_bytes) {
            FrameBuf b;
            if (alloc_buf(s.width, s.height, b) != MM_OK) return false;
            held += b.bytes;
            s.buf = b;
            break;
        }
        if (!pool.empty()) {  // none of this size: free one kept buffer
            auto p = pool.begin();
            held -= p->second.bytes;
            free_buf(p->second);
            pool.erase(p);
            continue;
        }
        Session* victim = nullptr;
        for (auto& kv : sessions) {
            Session& v = kv.second;
            if (v.admitted && !v.busy && v.queued == 0 && &v != &s &&
                (!victim || v.last_use < victim->last_use))
                victim = &v;
        }
        if (!victim) return false;
        pool.emplace(screen_key(victim->buf.width, victim->buf.height), victim->buf);
        victim->buf = FrameBuf{};
        victim->admitted = false;
        stats.evictions++;
    }
    s.admitted = true;
    stats.admissions++;
    return true;
}

void mm_server_s::release(Session& s) {
    if (!s.admitted) return;
    pool.emplace(screen_key(s.buf.width, s.buf.height), s.buf);
    s.buf = FrameBuf{};
    s.admitted = false;
}

bool mm_server_s::retire() {
    bool any = false;
    for (Slot& sl : slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            failed = true;
            fail(MM_ERR_HIP, "server: a launch failed: %s", hipGetErrorString(q));
        }
        const Clock::time_point now = Clock::now();
        for (uint64_t id : sl.reqs) {
            Request& r = requests[id];
            r.state = q == hipSuccess ? kDone : kDropped;
            r.t_done = now;
            Session& s = sessions[r.session];
            s.busy = false;
            clouds[r.cloud].busy = false;
            stats.completed++;
            if (s.closing && s.queued == 0) {
                release(s);
                s.closing = false;
                s.has_screen = false;
            }
        }
        sl.reqs.clear();
        sl.busy = false;
        any = true;
    }
    if (any) done_cv.notify_all();
    return any;
}

mm_status mm_server_s::launch(Slot& sl, const std::vector<uint64_t>& batch) {
    std::vector<mmb::Cloud> cl;
    std::vector<mmb::PlanView> views;
    for (uint64_t id : batch) {
        const Request& r = requests[id];
        const SCloud& c = clouds[r.cloud];
        Session& s = sessions[r.session];
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
        v.full_clear = true;
        v.colour = r.dev_out ? r.dev_out : s.buf.colour;
        v.seg = c.seg;
        v.table = c.table;
        v.part = s.buf.part;
        v.border = s.buf.border;
        v.apron = s.buf.apron;
        v.active = s.buf.active;
        views.push_back(v);
    }
    mmb::shape_views(views, cl, side, P, desc.tuning.splits);
    MM_TRY(mmb::build_tables(cl, views, P, desc.footprint, sl.img));
    const size_t stat = sl.img.stat.size(), frame = sl.img.frame.size();
    const size_t total = stat + frame;
    if (total > sl.dev_bytes) {
        if (sl.dev) (void)hipFree(sl.dev);
        sl.dev = nullptr;
        sl.dev_bytes = 0;
        MM_HIP(hipMalloc(reinterpret_cast<void**>(&sl.dev), total * 2));
        sl.dev_bytes = total * 2;
    }
    if (total > sl.pinned_bytes) {
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        sl.pinned_dev = nullptr;
        sl.pinned_bytes = 0;
        MM_HIP(hipHostMalloc(reinterpret_cast<void**>(&sl.pinned), total * 2, hipHostMallocCoherent));
        MM_HIP(hipHostGetDevicePointer(&sl.pinned_dev, sl.pinned, 0));
        sl.pinned_bytes = total * 2;
    }
    std::memcpy(sl.pinned, sl.img.stat.data(), stat);
    std::memcpy(sl.pinned + stat, sl.img.frame.data(), frame);
    // a kernel reads the staged tables: the slot's stream stays on the compute queue
    MM_HIP(mm::launch_upload(sl.dev, sl.pinned_dev, total, sl.stream));
    mmb::bind_args(sl.img, sl.dev, sl.dev + stat, sl.stamp_slot, shift, P, sl.b, sl.t, sl.m);
    if (++stamp == 0) {
        // every older stamp must read as "not this launch": clear all of them
        for (Slot& o : slots)
            if (o.busy) MM_HIP(hipStreamSynchronize(o.stream));
        for (auto& kv : sessions)
            if (kv.second.admitted)
                MM_HIP(hipMemset(kv.second.buf.active, 0, tiles_of(kv.second.width, kv.second.height, side) * 4));
        for (auto& kv : pool) (void)hipMemset(kv.second.base, 0, kv.second.bytes);
        stamp = 1;
    }
    sl.b.stamp = stamp;
    sl.nodes = mmb::make_nodes(desc.domain, desc.footprint, shift, ppt, threads, sl.img,
                               desc.tuning.grid_blocks, &sl.b, &sl.t, &sl.m);
    for (const mmb::Node& n : sl.nodes) MM_HIP(mmh::launch(n.l, n.arg, sl.stream));
    MM_HIP(hipEventRecord(sl.done, sl.stream));
    return MM_OK;
}

bool mm_server_s::schedule() {
    Slot* sl = nullptr;
    for (Slot& s : slots)
        if (!s.busy) {
            sl = &s;
            break;
        }
    if (!sl || pending.empty()) return false;
    std::vector<uint64_t> batch;
    for (uint64_t id : pending) {
        Request& r = requests[id];
        SCloud& c = clouds[r.cloud];
        Session& s = sessions[r.session];
        if (c.busy || c.queue.front() != id || s.busy) continue;
        if (!s.admitted && !admit(s)) continue;
        c.busy = true;
        s.busy = true;
        batch.push_back(id);
        if (batch.size() >= desc.max_batch) break;
    }
    if (batch.empty()) return false;
    for (uint64_t id : batch) {
        Request& r = requests[id];
        r.state = kInFlight;
        clouds[r.cloud].queue.pop_front();
        Session& s = sessions[r.session];
        s.queued--;
        s.last_use = stats.launches + 1;
    }
    pending.erase(std::remove_if(pending.begin(), pending.end(),
                                 [&](uint64_t id) { return requests[id].state != kQueued; }),
                  pending.end());
    sl->reqs = batch;
    sl->busy = true;
    stats.launches++;
    if (launch(*sl, batch) != MM_OK) {
        // the launch did not go out: mark its requests dropped
        failed = true;
        (void)hipStreamSynchronize(sl->stream);
        for (uint64_t id : batch) {
            Request& r = requests[id];
            r.state = kDropped;
            r.t_done = Clock::now();
            sessions[r.session].busy = false;
            clouds[r.cloud].busy = false;
        }
        sl->reqs.clear();
        sl->busy = false;
        done_cv.notify_all();
    }
    return true;
}

void mm_server_s::run() {
    (void)hipSetDevice(inst->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = retire();
        bool in_flight = false;
        for (const Slot& s : slots) in_flight = in_flight || s.busy;
        if (stop && !in_flight) break;
        if (!stop && !failed) progressed = schedule() || progressed;
        if (progressed) continue;
        if (in_flight)
            cv.wait_for(lk, std::chrono::microseconds(20));
        else
            cv.wait(lk, [&] { return stop || (!pending.empty() && !failed); });
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
    hipError_t e = hipMalloc(&srv->stamps, 256 * desc->streams);
    if (e == hipSuccess) e = hipMemset(srv->stamps, 0, 256 * desc->streams);
    srv->slots.resize(desc->streams);
    for (uint32_t k = 0; k < desc->streams && e == hipSuccess; ++k) {
        Slot& sl = srv->slots[k];
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        sl.stamp_slot = srv->stamps + 64 * k;
    }
    if (e != hipSuccess) {
        for (Slot& sl : srv->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (srv->stamps) (void)hipFree(srv->stamps);
        delete srv;
        return hip_fail(e, "create_server: streams");
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
        for (auto& kv : srv->requests)
            if (kv.second.state == kQueued) kv.second.state = kDropped;
        srv->pending.clear();
    }
    srv->cv.notify_all();
    srv->worker.join();
    srv->done_cv.notify_all();
    DeviceGuard guard(inst->device);
    for (Slot& sl : srv->slots) {
        (void)hipStreamSynchronize(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : srv->sessions) srv->free_buf(kv.second.buf);
    for (auto& kv : srv->pool) srv->free_buf(kv.second);
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
    *cloud_id = static_cast<uint32_t>(srv->clouds.size() - 1);
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
        if (srv->stop || srv->failed) return fail(MM_ERR_HIP, "server_submit: the server has stopped");
        if (cloud >= srv->clouds.size())
            return fail(MM_ERR_INVALID_ARG, "server_submit: cloud %u of %zu", cloud, srv->clouds.size());
        if (srv->fb_bytes(width, height) > srv->desc.fb_budget_bytes)
            return fail(MM_ERR_BUDGET, "server_submit: a %ux%u frame buffer (%llu B) exceeds the budget",
                        width, height, (unsigned long long)srv->fb_bytes(width, height));
        Session& s = srv->sessions[session];
        if (s.has_screen && (s.width != width || s.height != height))
            return fail(MM_ERR_INVALID_ARG, "server_submit: session %u is %ux%u, not %ux%u", session,
                        s.width, s.height, width, height);
        s.width = width;
        s.height = height;
        s.has_screen = true;
        s.closing = false;
        s.queued++;
        const uint64_t id = srv->next_id++;
        Request& r = srv->requests[id];
        r.session = session;
        r.cloud = cloud;
        r.step = srv->clouds[cloud].next_step++;
        std::memcpy(r.m, m, sizeof r.m);
        r.width = width;
        r.height = height;
        r.dev_out = dev_out;
        r.t_submit = Clock::now();
        srv->pending.push_back(id);
        srv->clouds[cloud].queue.push_back(id);
        srv->stats.submitted++;
        *request_id = id;
    }
    srv->cv.notify_all();
    return MM_OK;
}

mm_status mm_server_poll(mm_server srv, uint64_t id, int32_t* done, double* latency_s) {
    MM_TRY(server_ok(srv, "server_poll"));
    if (!done) return fail(MM_ERR_INVALID_ARG, "server_poll: null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(id);
    if (it == srv->requests.end()) return fail(MM_ERR_INVALID_ARG, "server_poll: unknown request %llu", (unsigned long long)id);
    const Request& r = it->second;
    if (r.state == kDropped) return fail(MM_ERR_HIP, "server_poll: request %llu was dropped", (unsigned long long)id);
    *done = r.state == kDone ? 1 : 0;
    if (latency_s && r.state == kDone) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    return MM_OK;
}

mm_status mm_server_wait(mm_server srv, uint64_t id, double* latency_s) {
    MM_TRY(server_ok(srv, "server_wait"));
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(id);
    if (it == srv->requests.end()) return fail(MM_ERR_INVALID_ARG, "server_wait: unknown request %llu", (unsigned long long)id);
    srv->done_cv.wait(lk, [&] {
        const ReqState st = srv->requests[id].state;
        return st == kDone || st == kDropped || srv->stop;
    });
    const Request& r = srv->requests[id];
    if (r.state != kDone) return fail(MM_ERR_NOT_READY, "server_wait: request %llu did not complete", (unsigned long long)id);
    if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    return MM_OK;
}

mm_status mm_server_read_frame(mm_server srv, uint32_t session, void* host_rgba, size_t bytes) {
    MM_TRY(server_ok(srv, "server_read_frame"));
    if (!host_rgba) return fail(MM_ERR_INVALID_ARG, "server_read_frame: null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end()) return fail(MM_ERR_INVALID_ARG, "server_read_frame: unknown session %u", session);
    Session& s = it->second;
    srv->done_cv.wait(lk, [&] { return !s.busy || srv->stop; });
    if (!s.admitted) return fail(MM_ERR_NOT_READY, "server_read_frame: session %u holds no frame buffer", session);
    const size_t need = static_cast<size_t>(s.width) * s.height * 4;
    if (bytes < need) return fail(MM_ERR_INVALID_ARG, "server_read_frame: %zu bytes < %zu", bytes, need);
    DeviceGuard guard(srv->inst->device);
    MM_HIP(hipMemcpy(host_rgba, s.buf.colour, need, hipMemcpyDeviceToHost));
    return MM_OK;
}

mm_status mm_server_close_session(mm_server srv, uint32_t session) {
    MM_TRY(server_ok(srv, "server_close_session"));
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end()) return fail(MM_ERR_INVALID_ARG, "server_close_session: unknown session %u", session);
    Session& s = it->second;
    if (!s.busy && s.queued == 0) {
        srv->release(s);
        s.closing = false;
        s.has_screen = false;
    } else {
        s.closing = true;
    }
    srv->cv.notify_all();
    return MM_OK;
}

mm_status mm_server_stats_get(mm_server srv, mm_server_stats* out) {
    MM_TRY(server_ok(srv, "server_stats_get"));
    if (!out) return fail(MM_ERR_INVALID_ARG, "server_stats_get: null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    mm_server_stats s = srv->stats;
    s.admitted_sessions = 0;
    for (auto& kv : srv->sessions) s.admitted_sessions += kv.second.admitted ? 1u : 0u;
    s.fb_bytes_in_use = srv->held;
    s.queued = srv->pending.size();
    *out = s;
    return MM_OK;
}

}  // extern "C"
