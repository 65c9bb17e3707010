// server.cpp -- the request server: LCS requests admitted as they arrive,
// within a device-memory budget, batched, and overlapped on the device.
//
// One dispatcher thread per server.  Requests wait in arrival order.
// Whenever a stream is free, the dispatcher takes the oldest waiting
// request together with the following ones of the same alphabet and
// traceback choice (up to max_batch_pairs), plans them as one batch whose
// device memory is carved out of the server's arena (first fit), uploads
// and launches it on that stream and goes on: requests that arrive while
// earlier batches run are admitted into new batches on the other streams,
// so their work overlaps on the device.  A batch that does not fit the free
// arena is retried with half the requests; a single request that does not
// fit waits for running batches to finish, and fails with LCS_ERR_NOMEM
// only when it does not fit the empty arena.  Finished batches are found by
// polling their completion events; their results are copied into the
// requests and their memory returns to the arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.hpp"
#include "lcs.h"

namespace {

using Clock = std::chrono::steady_clock;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               Clock::now().time_since_epoch())
        .count();
}

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Request {
    uint64_t id = 0;
    std::vector<uint8_t> x, y;
    std::vector<uint8_t> symbols;   // empty: all 256 bytes
    uint16_t alpha_size = 0;
    bool tb = false;
    ReqState state = kQueued;
    lcs_status status = LCS_OK;
    uint64_t len = 0;
    std::vector<uint8_t> lcs;
    uint64_t t_submit = 0, t_start = 0, t_done = 0;

    bool same_group(const Request &o) const {
        return tb == o.tb && alpha_size == o.alpha_size && symbols == o.symbols;
    }
    // small enough for the express stream
    bool small() const { return (uint64_t)x.size() * (uint64_t)y.size() <= kExpressCells; }
    static constexpr uint64_t kExpressCells = 1ull << 24;
};

// First-fit allocator over one device allocation.
class Arena {
  public:
    void init(char *base, size_t size) {
        base_ = base;
        free_.clear();
        used_.clear();
        free_[0] = size;
    }
    void *alloc(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_[off] = bytes;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        return nullptr;
    }
    void release(void *p) {
        const size_t off = (size_t)((char *)p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t size = u->second;
        in_use_ -= size;
        used_.erase(u);
        size_t start = off;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + size) {   // merge with the next block
            size += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {                             // merge with the previous block
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                size += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = size;
    }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }

  private:
    char *base_ = nullptr;
    std::map<size_t, size_t> free_, used_;
    size_t in_use_ = 0, peak_ = 0;
};

void *arena_alloc(void *user, size_t bytes);
void arena_release(void *user, void *p);

}  // namespace

struct lcs_server {
    lcs_ctx *ctx = nullptr;
    int device = 0;
    size_t arena_bytes = 0;
    int nstreams = 4;
    uint32_t max_batch = 4096;
    char *arena_mem = nullptr;
    Arena arena;                      // dispatcher thread only
    std::vector<hipStream_t> streams;

    std::mutex mu;                    // guards everything below
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    lcs_server_stats stats{};

    std::thread worker;
    void run();
};

namespace {

void *arena_alloc(void *user, size_t bytes) { return static_cast<lcs_server *>(user)->arena.alloc(bytes); }
void arena_release(void *user, void *p) { static_cast<lcs_server *>(user)->arena.release(p); }

struct Flight {
    lcs_batch *b = nullptr;
    int stream = 0;
    std::vector<Request *> rs;
    uint64_t t_launch = 0;
};

}  // namespace

void lcs_server::run() {
    (void)hipSetDevice(device);
    std::vector<Flight> flights;
    std::vector<int> free_streams;
    for (int k = nstreams - 1; k >= 0; --k) free_streams.push_back(k);
    uint32_t group_limit = max_batch;
    bool wait_completion = false;   // a lone request waits for memory to come back
    // With two or more streams, stream 0 is an express stream: it only takes
    // batches of small requests (at most 2^24 cells each), so that a burst
    // of long requests occupying the other streams does not hold up the many
    // short ones behind it.
    const int express = nstreams >= 2 ? 0 : -1;
    for (;;) {
        // ---- finished batches ----
        for (size_t f = 0; f < flights.size();) {
            const int q = lcs::batch_query(flights[f].b);
            if (q == 0) {
                ++f;
                continue;
            }
            Flight fl = std::move(flights[f]);
            flights.erase(flights.begin() + (long)f);
            const uint64_t t_found = now_ns();
            std::vector<uint64_t> lens;
            std::vector<std::vector<uint8_t>> strs;
            lcs_status st = q < 0 ? (lcs_status)q
                                  : lcs::batch_results(fl.b, lens, fl.rs[0]->tb ? &strs : nullptr);
            lcs_batch_destroy(fl.b);   // its memory goes back to the arena
            free_streams.push_back(fl.stream);
            wait_completion = false;
            group_limit = max_batch;
            const uint64_t t = now_ns();
            {
                std::lock_guard<std::mutex> lk(mu);
                stats.device_ns += t_found - fl.t_launch;
                stats.collect_ns += t - t_found;
                for (size_t k = 0; k < fl.rs.size(); ++k) {
                    Request *r = fl.rs[k];
                    r->t_done = t;
                    if (st) {
                        r->state = kFailed;
                        r->status = st;
                        ++stats.failed;
                    } else {
                        r->state = kDone;
                        r->len = lens[k];
                        if (r->tb) r->lcs = std::move(strs[k]);
                        ++stats.completed;
                        stats.cells += (uint64_t)r->x.size() * (uint64_t)r->y.size();
                    }
                    r->x.clear();
                    r->x.shrink_to_fit();
                    r->y.clear();
                    r->y.shrink_to_fit();
                }
                stats.arena_peak_bytes = arena.peak();
            }
            cv_done.notify_all();
        }
        // ---- admission ----
        std::vector<Request *> group;
        int si = -1;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && pending.empty() && flights.empty()) break;
            // a free general stream, else the express stream for small ones
            bool express_only = false;
            for (int k : free_streams)
                if (k != express) si = k;
            if (si < 0 && !free_streams.empty()) {
                si = express;
                express_only = true;
            }
            Request *head = nullptr;
            if (!pending.empty() && si >= 0 && !wait_completion) {
                if (!express_only) {
                    head = pending.front();
                } else {
                    for (Request *r : pending)
                        if (r->small()) {
                            head = r;
                            break;
                        }
                }
            }
            if (!head) {
                if (flights.empty()) {
                    cv_work.wait(lk, [&] { return stop || !pending.empty(); });
                } else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                }
                continue;
            }
            // the oldest (small, on the express stream) request and the
            // following ones of its group
            for (auto it = pending.begin(); it != pending.end() && group.size() < group_limit;) {
                if ((*it)->same_group(*head) && (!express_only || (*it)->small())) {
                    group.push_back(*it);
                    it = pending.erase(it);
                } else {
                    ++it;
                }
            }
            const uint64_t t = now_ns();
            for (Request *r : group) {
                r->state = kRunning;
                r->t_start = t;
            }
        }
        // ---- plan, upload and launch (outside the lock) ----
        const uint64_t t_plan = now_ns();
        std::vector<lcs_pair> pairs(group.size());
        for (size_t k = 0; k < group.size(); ++k)
            pairs[k] = lcs_pair{group[k]->x.data(), group[k]->x.size(), group[k]->y.data(),
                                group[k]->y.size()};
        const Request &h = *group[0];
        const lcs_alphabet al{h.alpha_size, h.symbols.empty() ? nullptr : h.symbols.data()};
        const uint32_t flags = h.tb ? LCS_WANT_TRACEBACK : 0u;
        lcs::BatchHooks hooks;
        hooks.stream = streams[si];
        hooks.alloc = arena_alloc;
        hooks.release = arena_release;
        hooks.user = this;
        // a lone traceback request whose full history would not fit even the
        // empty arena runs in rounds sized to it (one that fits waits for
        // memory instead, and a group that does not fit is split: rounds
        // cost a second fill)
        hooks.avail = group.size() == 1 ? arena_bytes : 0;
        lcs_tuning tun{};
        const bool tuned = lcs::tuning_cached(ctx, pairs.data(), pairs.size(), h.alpha_size, flags, &tun);
        lcs_batch *b = nullptr;
        lcs_status st = lcs::batch_create(ctx, pairs.data(), pairs.size(), &al, flags, &tun, &hooks, &b);
        if (!st) {
            st = lcs::batch_launch(b);
            if (st) {
                lcs_batch_destroy(b);
                b = nullptr;
            }
        }
        if (st == LCS_ERR_NOMEM && (group.size() > 1 || !flights.empty())) {
            // back to the queue, in arrival order, ahead of later arrivals
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = group.rbegin(); it != group.rend(); ++it) {
                (*it)->state = kQueued;
                pending.push_front(*it);
            }
            if (group.size() > 1)
                group_limit = std::max<uint32_t>(1, (uint32_t)group.size() / 2);
            else
                wait_completion = true;
            continue;
        }
        if (st) {
            std::lock_guard<std::mutex> lk(mu);
            const uint64_t t = now_ns();
            for (Request *r : group) {
                r->state = kFailed;
                r->status = st;
                r->t_done = t;
                ++stats.failed;
            }
            cv_done.notify_all();
            continue;
        }
        free_streams.erase(std::find(free_streams.begin(), free_streams.end(), si));
        const uint64_t t_launched = now_ns();
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.plan_ns += t_launched - t_plan;
            ++stats.batches;
            if (tuned) ++stats.tuned_batches;
            stats.max_inflight = std::max<uint64_t>(stats.max_inflight, flights.size() + 1);
        }
        Flight fl;
        fl.b = b;
        fl.stream = si;
        fl.t_launch = t_launched;
        fl.rs = std::move(group);
        flights.push_back(std::move(fl));
    }
}

extern "C" lcs_status lcs_server_create(lcs_ctx *ctx, const lcs_server_config *cfg,
                                        lcs_server **out) {
    if (!ctx || !out) return LCS_ERR_ARG;
    lcs_server_config c{};
    if (cfg) c = *cfg;
    if (c.streams < 0 || c.streams > 16 || c.max_batch_pairs < 0) return LCS_ERR_ARG;
    std::unique_ptr<lcs_server> s(new (std::nothrow) lcs_server());
    if (!s) return LCS_ERR_NOMEM;
    s->ctx = ctx;
    s->device = lcs::ctx_device(ctx);
    s->nstreams = c.streams ? c.streams : 4;
    s->max_batch = c.max_batch_pairs ? (uint32_t)c.max_batch_pairs : 4096u;
    size_t want = c.mem_budget_bytes;
    const lcs_status st = lcs::ctx_reserve(ctx, &want, (void **)&s->arena_mem);
    if (st) return st;
    s->arena_bytes = want;
    s->arena.init(s->arena_mem, want);
    if (hipSetDevice(s->device) != hipSuccess) {
        lcs::ctx_unreserve(ctx, s->arena_mem, s->arena_bytes);
        return LCS_ERR_DEVICE;
    }
    for (int k = 0; k < s->nstreams; ++k) {
        hipStream_t h = nullptr;
        if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
            lcs::ctx_unreserve(ctx, s->arena_mem, s->arena_bytes);
            return LCS_ERR_DEVICE;
        }
        s->streams.push_back(h);
    }
    s->stats.arena_bytes = s->arena_bytes;
    lcs_server *sp = s.release();
    sp->worker = std::thread([sp] { sp->run(); });
    *out = sp;
    return LCS_OK;
}

extern "C" void lcs_server_destroy(lcs_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests are dropped; running batches finish
        for (Request *r : s->pending) {
            r->state = kFailed;
            r->status = LCS_ERR_ARG;
        }
        s->pending.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
    lcs::ctx_unreserve(s->ctx, s->arena_mem, s->arena_bytes);
    delete s;
}

extern "C" lcs_status lcs_submit(lcs_server *s, const uint8_t *x, uint64_t m, const uint8_t *y,
                                 uint64_t n, const lcs_alphabet *alphabet, int want_traceback,
                                 uint64_t *ticket) {
    if (!s || !ticket) return LCS_ERR_ARG;
    int sigma = 0;
    const lcs_status st = lcs::alphabet_check(alphabet, x, m, y, n, &sigma);
    if (st) return st;
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return LCS_ERR_NOMEM;
    try {
        r->x.assign(x, x + m);
        r->y.assign(y, y + n);
        if (alphabet->symbols) r->symbols.assign(alphabet->symbols, alphabet->symbols + alphabet->size);
    } catch (const std::bad_alloc &) {
        return LCS_ERR_NOMEM;
    }
    r->alpha_size = alphabet->size;
    r->tb = want_traceback != 0;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return LCS_ERR_ARG;
        r->id = s->next_id++;
        *ticket = r->id;
        s->pending.push_back(r.get());
        s->reqs[r->id] = std::move(r);
        ++s->stats.submitted;
    }
    s->cv_work.notify_one();
    return LCS_OK;
}

static lcs_status state_status(const Request &r) {
    if (r.state == kDone) return LCS_OK;
    if (r.state == kFailed) return r.status;
    return LCS_PENDING;
}

extern "C" lcs_status lcs_poll(lcs_server *s, uint64_t ticket) {
    if (!s) return LCS_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LCS_ERR_ARG;
    return state_status(*it->second);
}

extern "C" lcs_status lcs_wait(lcs_server *s, uint64_t ticket, int64_t timeout_us) {
    if (!s) return LCS_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LCS_ERR_ARG;
    Request *r = it->second.get();
    auto ready = [&] { return r->state == kDone || r->state == kFailed; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, ready);
    else
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    return state_status(*r);
}

extern "C" lcs_status lcs_result(lcs_server *s, uint64_t ticket, uint64_t *len, uint8_t *out,
                                 uint64_t out_cap, uint64_t *latency_ns) {
    if (!s || !len) return LCS_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LCS_ERR_ARG;
    Request *r = it->second.get();
    const lcs_status st = state_status(*r);
    if (st == LCS_PENDING) return st;
    if (st == LCS_OK) {
        if (r->tb) {
            if (out_cap < r->lcs.size()) return LCS_ERR_BUFFER;
            if (!r->lcs.empty()) {
                if (!out) return LCS_ERR_ARG;
                std::memcpy(out, r->lcs.data(), r->lcs.size());
            }
        }
        *len = r->len;
    }
    if (latency_ns) *latency_ns = r->t_done - r->t_submit;
    s->reqs.erase(it);
    return st;
}

extern "C" lcs_status lcs_cancel(lcs_server *s, uint64_t ticket) {
    if (!s) return LCS_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->state != kQueued) return LCS_ERR_ARG;
    auto q = std::find(s->pending.begin(), s->pending.end(), it->second.get());
    if (q != s->pending.end()) s->pending.erase(q);
    s->reqs.erase(it);
    ++s->stats.cancelled;
    return LCS_OK;
}

extern "C" lcs_status lcs_server_stats_get(lcs_server *s, lcs_server_stats *out) {
    if (!s || !out) return LCS_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = s->pending.size();
    return LCS_OK;
}
