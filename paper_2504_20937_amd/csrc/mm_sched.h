// Scheduling policy of the served form, free of device code: request queues
// per cloud, admission of sessions by frame-buffer bytes, eviction, packing
// of pending requests into launches over a fixed set of slots (continuous
// batching), completion and failure handling. The server drives it under its
// lock; a backend supplies frame-buffer memory and launches. Nothing here
// calls HIP, so the policy also builds and runs on the host alone.
//
// Order and results: requests on one cloud run in submission order, the
// k-th on a cloud with displacement step k. A launch holds at most one
// request per cloud and per session. Slots come in groups that share a
// stream; a cloud's or a session's requests are in flight on one stream at a
// time, so several of them can be (a cloud's next step runs after the
// previous one's positions are written, in stream order; a session's frame
// buffer is written by one launch after another).
//
// Chaining: a slot on the stream where a cloud is in flight takes that
// cloud's next request, so saturated clouds go out together in every launch,
// one launch queued behind the other, and the next launch is prepared on the
// host while the previous one runs. A launch with no cloud to chain goes to
// a stream with nothing in flight, so independent requests run side by side.
//
// Progress: when no launch is in flight and a request is pending, the next
// schedule() launches one. The earliest pending request leads its cloud's
// queue; with nothing in flight no session is busy, so admission can evict
// every other session (idle ones first, then ones with queued requests,
// least recently used first) and free kept buffers until the frame buffer
// fits (a session whose buffer alone exceeds the budget is refused at
// submission). A session evicted with requests queued is admitted again
// when its turn comes; its frame buffer holds no history to lose.
//
// Failure: a launch that fails (or does not go out), or a frame buffer
// within the budget that cannot be allocated even with every other buffer
// given up, stops the scheduler: the launch's requests and every queued one
// are dropped, so no waiter blocks on them, and later submissions fail.
//
// Buf is the backend's frame-buffer handle; it carries its screen (fields
// width and height), by which kept buffers are matched and counted.
#pragma once

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "mm.h"

namespace mms {

using Clock = std::chrono::steady_clock;

enum ReqState { kQueued = 0, kInFlight = 1, kDone = 2, kDropped = 3 };

template <typename Buf>
class Scheduler {
public:
    struct Request {
        uint32_t session = 0, cloud = 0, step = 0;
        float m[16] = {};
        uint32_t width = 0, height = 0;
        uint32_t* dev_out = nullptr;
        Clock::time_point t_submit, t_done;
        ReqState state = kQueued;
    };

    struct Session {
        uint32_t width = 0, height = 0;
        bool has_screen = false;
        bool admitted = false;
        uint32_t inflight = 0;  // requests in flight (all on stream `stream`)
        uint32_t stream = 0;
        uint64_t mark = 0;      // the launch being packed that holds one of its requests
        bool closing = false;
        uint32_t queued = 0;    // requests submitted, not launched
        uint64_t last_use = 0;  // launch counter when last launched (LRU)
        Buf buf{};
    };

    struct Cloud {
        uint32_t next_step = 0;
        uint32_t inflight = 0;  // requests in flight (all on stream `stream`)
        uint32_t stream = 0;
        uint64_t mark = 0;      // the launch being packed that holds one of its requests
        std::deque<uint64_t> queue;  // request ids not launched, in submission order
    };

    // One request of a launch, with the session that renders it.
    struct Item {
        uint64_t id;
        const Request* req;
        Session* session;
    };

    struct Backend {
        virtual ~Backend() = default;
        virtual uint64_t fb_bytes(uint32_t w, uint32_t h) const = 0;
        // A cleared frame buffer of w x h; false when memory is short.
        virtual bool alloc_buf(uint32_t w, uint32_t h, Buf& out) = 0;
        virtual void free_buf(Buf& b) = 0;
        // Sends the launch out on slot `slot`; false if it did not go out.
        virtual bool launch(uint32_t slot, const std::vector<Item>& items) = 0;
        // State of the slot's launch: 0 running, 1 complete, -1 failed.
        virtual int query(uint32_t slot) = 0;
    };

    // slots / per_stream streams; slot k runs on stream k / per_stream.
    Scheduler(Backend& be, uint64_t budget, uint32_t slots, uint32_t max_batch, uint32_t per_stream = 1)
        : be_(be), budget_(budget), max_batch_(max_batch), per_stream_(per_stream), slots_(slots) {}

    Scheduler(const Scheduler&) = delete;
    Scheduler& operator=(const Scheduler&) = delete;

    // Adds a cloud; returns its id.
    uint32_t add_cloud() {
        clouds_.emplace_back();
        return static_cast<uint32_t>(clouds_.size() - 1);
    }
    size_t clouds() const { return clouds_.size(); }

    // Queues a request. MM_ERR_BUDGET when the session's frame buffer alone
    // exceeds the budget, MM_ERR_INVALID_ARG for a screen other than the
    // session's or an unknown cloud, MM_ERR_HIP once the scheduler failed.
    mm_status submit(uint32_t session, uint32_t cloud, const float m[16], uint32_t w, uint32_t h,
                     uint32_t* dev_out, uint64_t* id_out) {
        if (failed_) return MM_ERR_HIP;
        if (cloud >= clouds_.size()) return MM_ERR_INVALID_ARG;
        if (be_.fb_bytes(w, h) > budget_) return MM_ERR_BUDGET;
        Session& s = sessions_[session];
        if (s.has_screen && (s.width != w || s.height != h)) return MM_ERR_INVALID_ARG;
        s.width = w;
        s.height = h;
        s.has_screen = true;
        s.closing = false;
        s.queued++;
        const uint64_t id = next_id_++;
        Request& r = requests_[id];
        r.session = session;
        r.cloud = cloud;
        r.step = clouds_[cloud].next_step++;
        std::memcpy(r.m, m, sizeof r.m);
        r.width = w;
        r.height = h;
        r.dev_out = dev_out;
        r.t_submit = Clock::now();
        pending_.push_back(id);
        clouds_[cloud].queue.push_back(id);
        stats_.submitted++;
        *id_out = id;
        return MM_OK;
    }

    // Retires every complete launch; true if any was. A failed launch drops
    // its requests and then every queued one.
    bool retire() {
        bool any = false;
        for (uint32_t k = 0; k < slots_.size(); ++k) {
            SlotState& sl = slots_[k];
            if (!sl.busy) continue;
            const int q = be_.query(k);
            if (q == 0) continue;
            const Clock::time_point now = Clock::now();
            for (uint64_t id : sl.reqs) {
                Request& r = requests_[id];
                r.state = q > 0 ? kDone : kDropped;
                r.t_done = now;
                (q > 0 ? stats_.completed : stats_.dropped)++;
                Session& s = sessions_[r.session];
                s.inflight--;
                clouds_[r.cloud].inflight--;
                if (s.closing && s.queued == 0 && s.inflight == 0) close_now(s);
            }
            sl.reqs.clear();
            sl.busy = false;
            in_flight_--;
            any = true;
            if (q < 0) drop_queued();
        }
        return any;
    }

    // Packs pending requests into one launch on a free slot; true if a
    // launch was attempted (sent, or failed and its requests dropped).
    bool schedule() {
        if (failed_ || pending_.empty()) return false;
        const int picked = pick_slot();
        if (picked < 0) return false;
        const uint32_t slot = static_cast<uint32_t>(picked), st = slot / per_stream_;
        const uint64_t tag = ++tag_;
        std::vector<uint64_t> batch;
        bool no_memory = false;
        for (uint64_t id : pending_) {
            Request& r = requests_[id];
            Cloud& c = clouds_[r.cloud];
            Session& s = sessions_[r.session];
            if (c.queue.front() != id || c.mark == tag || s.mark == tag) continue;
            if ((c.inflight != 0 && c.stream != st) || (s.inflight != 0 && s.stream != st)) continue;
            if (!s.admitted) {
                const int a = admit(s);
                if (a < 0) {
                    no_memory = true;
                    break;
                }
                if (a == 0) continue;
            }
            c.mark = tag;
            s.mark = tag;
            c.inflight++;
            c.stream = st;
            s.inflight++;
            s.stream = st;
            batch.push_back(id);
            if (batch.size() >= max_batch_) break;
        }
        if (no_memory) {
            // a frame buffer within the budget cannot be allocated even with
            // every other buffer given up: the server stops as after a failed
            // launch (a request left out would break its cloud's step order)
            for (uint64_t id : batch) {
                sessions_[requests_[id].session].inflight--;
                clouds_[requests_[id].cloud].inflight--;
            }
            drop_queued();
            return true;
        }
        if (batch.empty()) return false;
        std::vector<Item> items;
        items.reserve(batch.size());
        for (uint64_t id : batch) {
            Request& r = requests_[id];
            r.state = kInFlight;
            clouds_[r.cloud].queue.pop_front();
            Session& s = sessions_[r.session];
            s.queued--;
            s.last_use = stats_.launches + 1;
            items.push_back(Item{id, &r, &s});
        }
        erase_from_pending();
        SlotState& sl = slots_[slot];
        sl.reqs = batch;
        sl.busy = true;
        stats_.launches++;
        stats_.max_batch = std::max<uint64_t>(stats_.max_batch, batch.size());
        in_flight_++;
        stats_.max_in_flight = std::max<uint64_t>(stats_.max_in_flight, in_flight_);
        if (!be_.launch(slot, items)) {
            // the launch did not go out: its requests and every queued one are dropped
            const Clock::time_point now = Clock::now();
            for (uint64_t id : batch) {
                Request& r = requests_[id];
                r.state = kDropped;
                r.t_done = now;
                stats_.dropped++;
                sessions_[r.session].inflight--;
                clouds_[r.cloud].inflight--;
            }
            sl.reqs.clear();
            sl.busy = false;
            in_flight_--;
            drop_queued();
        }
        return true;
    }

    // Releases the session's buffer now if it is idle, else once its queued
    // requests are done. false for an unknown session.
    bool close_session(uint32_t session) {
        auto it = sessions_.find(session);
        if (it == sessions_.end()) return false;
        Session& s = it->second;
        if (s.inflight == 0 && s.queued == 0) close_now(s);
        else s.closing = true;
        return true;
    }

    // Every request still queued is dropped (server shutdown).
    void drop_all_queued() {
        for (uint64_t id : pending_) mark_dropped(id);
        pending_.clear();
        for (Cloud& c : clouds_) c.queue.clear();
    }

    // Frees every buffer held by sessions and kept for reuse.
    void free_all() {
        for (auto& kv : sessions_)
            if (kv.second.admitted) be_.free_buf(kv.second.buf);
        for (auto& kv : pool_) be_.free_buf(kv.second);
        pool_.clear();
        held_ = 0;
    }

    // Calls fn(Buf&) on every buffer held (admitted sessions, then kept ones).
    template <typename Fn>
    void for_each_buf(Fn fn) {
        for (auto& kv : sessions_)
            if (kv.second.admitted) fn(kv.second.buf);
        for (auto& kv : pool_) fn(kv.second);
    }

    const Request* request(uint64_t id) const {
        auto it = requests_.find(id);
        return it == requests_.end() ? nullptr : &it->second;
    }
    Session* session(uint32_t id) {
        auto it = sessions_.find(id);
        return it == sessions_.end() ? nullptr : &it->second;
    }
    bool in_flight() const { return in_flight_ != 0; }
    bool has_pending() const { return !pending_.empty(); }
    bool failed() const { return failed_; }
    uint64_t held() const { return held_; }

    mm_server_stats stats() const {
        mm_server_stats s = stats_;
        s.admitted_sessions = 0;
        for (auto& kv : sessions_) s.admitted_sessions += kv.second.admitted ? 1u : 0u;
        s.fb_bytes_in_use = held_;
        s.queued = pending_.size();
        return s;
    }

private:
    int free_slot_on(uint32_t stream) const {
        for (uint32_t k = stream * per_stream_; k < (stream + 1) * per_stream_ && k < slots_.size(); ++k)
            if (!slots_[k].busy) return static_cast<int>(k);
        return -1;
    }

    // The slot of the next launch: a free slot on the stream of a cloud in
    // flight whose next request is pending (that request and the cloud's
    // later steps chain behind it), else a free slot on a stream with nothing
    // in flight, else any free slot; -1 when none is free.
    int pick_slot() {
        for (uint64_t id : pending_) {
            const Request& r = requests_[id];
            const Cloud& c = clouds_[r.cloud];
            if (c.inflight == 0 || c.queue.front() != id) continue;
            const Session& s = sessions_[r.session];
            if (s.inflight != 0 && s.stream != c.stream) continue;
            const int k = free_slot_on(c.stream);
            if (k >= 0) return k;
        }
        int any = -1;
        for (uint32_t k = 0; k < slots_.size(); ++k) {
            if (slots_[k].busy) continue;
            bool idle = true;
            const uint32_t st = k / per_stream_;
            for (uint32_t j = st * per_stream_; j < (st + 1) * per_stream_ && j < slots_.size(); ++j)
                idle = idle && !slots_[j].busy;
            if (idle) return static_cast<int>(k);
            if (any < 0) any = static_cast<int>(k);
        }
        return any;
    }

    struct SlotState {
        bool busy = false;
        std::vector<uint64_t> reqs;
    };

    static uint64_t screen_key(uint32_t w, uint32_t h) { return (static_cast<uint64_t>(w) << 32) | h; }

    // 1: s holds a buffer; 0: not now (the memory is held by sessions in
    // flight); -1: no buffer even with every other buffer given up.
    int admit(Session& s) {
        const uint64_t need = be_.fb_bytes(s.width, s.height);
        const uint64_t key = screen_key(s.width, s.height);
        for (;;) {
            auto it = pool_.find(key);
            if (it != pool_.end()) {
                s.buf = it->second;
                pool_.erase(it);
                break;
            }
            const bool fits = held_ + need <= budget_;
            if (fits) {
                Buf b{};
                if (be_.alloc_buf(s.width, s.height, b)) {
                    held_ += need;
                    s.buf = b;
                    break;
                }
            }
            // over budget, or the device is short of memory: free a kept
            // buffer (none of this size is kept), else evict a session into
            // the pool, where the next round frees or reuses its buffer
            if (!pool_.empty()) {
                auto p = pool_.begin();
                held_ -= be_.fb_bytes(p->second.width, p->second.height);
                be_.free_buf(p->second);
                pool_.erase(p);
                continue;
            }
            if (evict_one(s)) continue;
            return fits && !in_flight_ ? -1 : 0;
        }
        s.admitted = true;
        stats_.admissions++;
        return 1;
    }

    // Moves the buffer of the least recently used session that is neither
    // `s` nor busy into the pool, preferring sessions with nothing queued.
    bool evict_one(const Session& s) {
        Session* victim = nullptr;
        for (auto& kv : sessions_) {
            Session& v = kv.second;
            if (!v.admitted || v.inflight != 0 || &v == &s) continue;
            if (!victim) {
                victim = &v;
                continue;
            }
            const bool v_idle = v.queued == 0, w_idle = victim->queued == 0;
            if (v_idle != w_idle ? v_idle : v.last_use < victim->last_use) victim = &v;
        }
        if (!victim) return false;
        pool_.emplace(screen_key(victim->buf.width, victim->buf.height), victim->buf);
        victim->buf = Buf{};
        victim->admitted = false;
        stats_.evictions++;
        return true;
    }

    void close_now(Session& s) {
        if (s.admitted) {
            pool_.emplace(screen_key(s.buf.width, s.buf.height), s.buf);
            s.buf = Buf{};
            s.admitted = false;
        }
        s.closing = false;
        s.has_screen = false;
    }

    void mark_dropped(uint64_t id) {
        Request& r = requests_[id];
        if (r.state != kQueued) return;
        r.state = kDropped;
        r.t_done = Clock::now();
        stats_.dropped++;
        Session& s = sessions_[r.session];
        s.queued--;
        if (s.closing && s.queued == 0 && s.inflight == 0) close_now(s);
    }

    // After a failed launch nothing more is scheduled: every queued request
    // is dropped so that no waiter blocks on it.
    void drop_queued() {
        failed_ = true;
        drop_all_queued();
    }

    void erase_from_pending() {
        pending_.erase(std::remove_if(pending_.begin(), pending_.end(),
                                      [&](uint64_t id) { return requests_[id].state != kQueued; }),
                       pending_.end());
    }

    Backend& be_;
    uint64_t budget_;
    uint32_t max_batch_;
    uint32_t per_stream_;
    std::vector<SlotState> slots_;
    std::vector<Cloud> clouds_;
    std::unordered_map<uint32_t, Session> sessions_;
    std::unordered_map<uint64_t, Request> requests_;
    std::deque<uint64_t> pending_;       // submission order
    std::multimap<uint64_t, Buf> pool_;  // kept for reuse, by (width << 32 | height)
    uint64_t held_ = 0;                  // bytes of admitted and kept buffers
    uint64_t next_id_ = 1;
    uint32_t in_flight_ = 0;
    uint64_t tag_ = 0;  // launches packed so far (marks)
    bool failed_ = false;
    mm_server_stats stats_{};
};

}  // namespace mms
