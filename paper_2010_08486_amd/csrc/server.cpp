// Serving loop: requests (host frames) arrive at any time; a dispatcher thread
// forms batches from whatever is waiting, bounded by a frame count and by the
// device footprint still free in the admission budget, and hands each batch
// to an idle slot.  Every slot owns a context (workspace, stream, cached
// launch graph) and a worker thread, so batches launched while others are
// running overlap on the device.  Results are kept per ticket with arrival
// and completion times for latency statistics.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "runtime.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Page-locked host buffers for request copies, reused across requests so a
// steady stream allocates nothing.  Beyond `cap` bytes pinned, buffers are
// plain pageable memory (staged by the context instead of DMA'd directly).
class PinnedPool {
public:
    explicit PinnedPool(uint64_t cap) : cap_(cap) {}
    ~PinnedPool()
    {
        for (auto& kv : free_)
            (void)hipHostFree(kv.second);
    }
    // A buffer of at least `bytes`; *pinned tells which kind it is.
    void* get(size_t bytes, size_t* got, bool* pinned)
    {
        const size_t sz = (bytes + kGrain - 1) / kGrain * kGrain;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(sz);
            if (it != free_.end() && it->first <= 2 * sz) {
                void* p = it->second;
                *got = it->first;
                free_.erase(it);
                *pinned = true;
                return p;
            }
            // make room by dropping idle buffers, largest first
            while (total_ + sz > cap_ && !free_.empty()) {
                auto last = std::prev(free_.end());
                (void)hipHostFree(last->second);
                total_ -= last->first;
                free_.erase(last);
            }
            if (!failed_ && total_ + sz <= cap_) {
                void* p = nullptr;
                if (hipHostMalloc(&p, sz, hipHostMallocPortable) == hipSuccess) {
                    total_ += sz;
                    *got = sz;
                    *pinned = true;
                    return p;
                }
                (void)hipGetLastError();
                failed_ = true;  // no more attempts: pageable from now on
            }
        }
        *got = bytes;
        *pinned = false;
        return std::malloc(bytes);
    }
    void put(void* p, size_t bytes, bool pinned)
    {
        if (!p)
            return;
        if (!pinned) {
            std::free(p);
            return;
        }
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(bytes, p);
    }

private:
    static constexpr size_t kGrain = 1u << 20;
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    uint64_t total_ = 0;
    uint64_t cap_;
    bool failed_ = false;
};

struct Request {
    uint64_t ticket = 0;
    const float* data = nullptr;  // pinned/pageable copy (owned) or borrowed device frame
    size_t bytes = 0;             // size of the owned copy
    bool pinned = false;
    bool on_device = false;
    int64_t H = 0, W = 0, stride = 0;
    int64_t t_arrive = 0;
    uint64_t footprint = 0;
};

struct Slot {
    dog_context* ctx = nullptr;
    std::thread th;
    std::vector<Request> batch;
    bool has_work = false;
    // device buffers the slot's context holds (as of its last batch) and the
    // bytes admission counts for it: what it holds while idle, the bound of
    // its batch while running (its context's budget is capped at that bound)
    uint64_t planes_b = 0, input_b = 0, other_b = 0;
    uint64_t commit = 0;
    uint64_t held() const { return planes_b + input_b + other_b; }
};

}  // namespace

struct dog_server {
    dog_params prm{};
    dog_server_opts opts{};
    dog::Plan plan;
    int n_g = 0;
    uint64_t budget = 0;

    std::unique_ptr<PinnedPool> pool;
    std::mutex mu;
    std::condition_variable cv_dispatch;  // queue grew or a slot became idle
    std::condition_variable cv_done;      // a batch completed
    std::deque<Request> queue;
    std::vector<std::unique_ptr<Slot>> slots;
    std::condition_variable cv_slot;      // a slot got work (or stop)
    std::unordered_map<uint64_t, dog_result> done;
    std::unordered_set<uint64_t> pending;  // queued or running
    uint64_t next_ticket = 1;
    uint64_t reserved = 0;                 // sum of the slots' commits
    uint64_t peak_reserved = 0;
    uint64_t peak_held = 0;                // largest sum of the slots' held bytes
    int64_t admission_waits = 0;           // times the oldest request did not fit
    bool stop = false;
    std::thread dispatcher;

    // statistics
    std::vector<double> lat_ms;
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, batch_frames = 0;
    int64_t running = 0;
    int64_t t_first = 0, t_last = 0;
};

namespace {

uint64_t page(uint64_t x) { return (x + 4095) & ~(uint64_t)4095; }

// Device bytes slot sl may hold while it runs `reqs` (plus `extra` when not
// NULL): each workspace buffer grows to the batch's need if that is larger
// than what the slot holds (exact allocation, so no growth slack), and the
// launch tables and candidate buffer add at most overhead_bound to what it
// already holds.  The slot's context budget is set to this figure, so its
// allocations cannot exceed it.
uint64_t slot_commit(const dog_server* sv, const Slot* sl, const std::vector<Request>& reqs,
                     const Request* extra)
{
    uint64_t planes = 0, input = 0;
    std::vector<int64_t> hs, ws;
    auto add = [&](const Request& r) {
        planes += dog::frame_plane_bytes(sv->plan, r.H, r.W);
        if (!r.on_device)
            input += dog::frame_input_bytes(r.H, r.W);
        hs.push_back(r.H);
        ws.push_back(r.W);
    };
    for (const Request& r : reqs)
        add(r);
    if (extra)
        add(*extra);
    if (hs.empty())
        return sl->held();
    return std::max(sl->planes_b, page(planes)) + std::max(sl->input_b, page(input)) + sl->other_b +
           dog::overhead_bound(sv->plan, (int)hs.size(), hs.data(), ws.data());
}

uint64_t sum_commits(const dog_server* sv, const Slot* except)
{
    uint64_t t = 0;
    for (const auto& s : sv->slots)
        if (s.get() != except)
            t += s->commit;
    return t;
}

void release_request(dog_server* sv, Request& r)
{
    if (!r.on_device && r.data)
        sv->pool->put(const_cast<float*>(r.data), r.bytes, r.pinned);
    r.data = nullptr;
}

void run_slot(dog_server* sv, Slot* sl)
{
    for (;;) {
        std::vector<Request> batch;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_slot.wait(lk, [&] { return sl->has_work || sv->stop; });
            if (!sl->has_work)
                return;
            batch.swap(sl->batch);
            if (sl->ctx)
                sl->ctx->budget = sl->commit;  // allocations stay within the commit
        }
        const int n = (int)batch.size();
        std::vector<dog_result> res(n);
        int rc = DOG_OK;
        if (sv->opts.dry_run) {
            double mpx = 0;
            for (const Request& r : batch)
                mpx += (double)r.H * (double)r.W * 1e-6;
            const int64_t us = (int64_t)(sv->opts.dry_run_us_per_mpx * mpx);
            std::this_thread::sleep_for(std::chrono::microseconds(us));
            for (dog_result& r : res)
                std::memset(&r, 0, sizeof(r));
        } else {
            std::vector<dog_frame> fr(n);
            for (int i = 0; i < n; ++i) {
                fr[i].data = batch[i].data;
                fr[i].height = batch[i].H;
                fr[i].width = batch[i].W;
                fr[i].row_stride = batch[i].stride;
                fr[i].on_device = batch[i].on_device ? 1 : (batch[i].pinned ? 2 : 0);
                fr[i].reserved = 0;
            }
            rc = dog::detect_frames(sl->ctx, &sv->prm, n, fr.data(), sl->ctx->stream, res.data());
        }
        for (Request& r : batch)  // uploads have completed: results were read back
            release_request(sv, r);
        const int64_t t_done = now_ns();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (int i = 0; i < n; ++i) {
                dog_result r = res[i];
                if (rc != DOG_OK && r.status == DOG_OK)
                    r.status = rc;
                r.t_arrive_ns = batch[i].t_arrive;
                r.t_done_ns = t_done;
                if (r.status == DOG_OK) {
                    sv->completed += 1;
                    sv->lat_ms.push_back((double)(t_done - batch[i].t_arrive) * 1e-6);
                } else {
                    sv->failed += 1;
                }
                sv->pending.erase(batch[i].ticket);
                sv->done[batch[i].ticket] = r;
            }
            if (sl->ctx) {
                sl->planes_b = sl->ctx->planes.bytes;
                sl->input_b = sl->ctx->input.bytes;
                sl->other_b = sl->ctx->used - sl->planes_b - sl->input_b;
            }
            sl->commit = sl->held();
            sv->reserved = sum_commits(sv, nullptr);
            uint64_t held = 0;
            for (const auto& o : sv->slots)
                held += o->held();
            sv->peak_held = std::max(sv->peak_held, held);
            sv->running -= n;
            sv->t_last = std::max(sv->t_last, t_done);
            sl->has_work = false;
        }
        sv->cv_done.notify_all();
        sv->cv_dispatch.notify_all();
    }
}

// Dispatcher: whenever requests wait and a slot is idle, launch a batch of
// the oldest requests that fit in the free admission budget.
void run_dispatcher(dog_server* sv)
{
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        Slot* idle = nullptr;
        sv->cv_dispatch.wait(lk, [&] {
            if (sv->stop)
                return true;
            if (sv->queue.empty())
                return false;
            for (auto& s : sv->slots)
                if (!s->has_work)
                    return true;
            return false;
        });
        if (sv->stop)
            return;
        // the idle slot holding the most device memory: a batch that fits in
        // its buffers adds nothing to what the slots hold
        for (auto& s : sv->slots)
            if (!s->has_work && (!idle || s->held() > idle->held()))
                idle = s.get();
        // batching window: give a short batch a chance to grow
        if (sv->opts.max_wait_ms > 0.0 && (int)sv->queue.size() < sv->opts.max_batch_frames) {
            const int64_t deadline =
                sv->queue.front().t_arrive + (int64_t)(sv->opts.max_wait_ms * 1e6);
            const int64_t now = now_ns();
            if (now < deadline) {
                sv->cv_dispatch.wait_for(lk, std::chrono::nanoseconds(deadline - now));
                continue;
            }
        }
        // admission: the other slots' commits (what idle slots hold, the
        // bounds of running batches) plus this slot's bound for the batch
        // must stay within the budget
        const uint64_t others = sum_commits(sv, idle);
        std::vector<Request> batch;
        uint64_t commit = idle->held();
        int64_t px = 0;
        while (!sv->queue.empty() && (int)batch.size() < sv->opts.max_batch_frames) {
            const Request& r = sv->queue.front();
            const uint64_t c = slot_commit(sv, idle, batch, &r);
            if (others + c > sv->budget)
                break;  // wait until memory is released
            const int64_t rpx = (int64_t)r.H * (int64_t)r.W;
            if (!batch.empty() && sv->opts.max_batch_pixels > 0 &&
                px + rpx > sv->opts.max_batch_pixels)
                break;  // the batch's planes would outgrow the cache
            px += rpx;
            commit = c;
            batch.push_back(std::move(sv->queue.front()));
            sv->queue.pop_front();
        }
        if (batch.empty()) {
            // the oldest request does not fit.  Idle slots keep their
            // workspaces between batches: release them, other slots first,
            // then this one; otherwise wait for a running batch to finish
            const Request& r = sv->queue.front();
            sv->admission_waits += 1;
            std::vector<Slot*> idle_held;
            for (auto& s : sv->slots)
                if (!s->has_work && s.get() != idle && s->held() > 0)
                    idle_held.push_back(s.get());
            std::sort(idle_held.begin(), idle_held.end(),
                      [](const Slot* a, const Slot* b) { return a->held() > b->held(); });
            if (idle->held() > 0)
                idle_held.push_back(idle);
            bool trimmed = false;
            for (Slot* s : idle_held) {
                if (sum_commits(sv, idle) + slot_commit(sv, idle, {}, &r) <= sv->budget)
                    break;
                if (s->ctx)
                    (void)dog::ctx_trim(s->ctx);
                s->planes_b = s->input_b = s->other_b = 0;
                s->commit = 0;
                trimmed = true;
            }
            sv->reserved = sum_commits(sv, nullptr);
            if (!trimmed)
                sv->cv_done.wait(lk);
            continue;
        }
        idle->commit = commit;
        sv->reserved = sum_commits(sv, nullptr);
        sv->peak_reserved = std::max(sv->peak_reserved, sv->reserved);
        sv->running += (int64_t)batch.size();
        sv->batches += 1;
        sv->batch_frames += (int64_t)batch.size();
        idle->batch = std::move(batch);
        idle->has_work = true;
        sv->cv_slot.notify_all();
    }
}

void destroy_server(dog_server* sv)
{
    if (!sv)
        return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_dispatch.notify_all();
    sv->cv_done.notify_all();
    if (sv->dispatcher.joinable())
        sv->dispatcher.join();
    // slots finish the batch they hold, then exit
    {
        std::lock_guard<std::mutex> lk(sv->mu);
    }
    sv->cv_slot.notify_all();
    for (auto& s : sv->slots) {
        if (s->th.joinable())
            s->th.join();
        if (s->ctx)
            dog_context_destroy(s->ctx);
    }
    for (auto& kv : sv->done)
        std::free(kv.second.blobs);
    for (Request& r : sv->queue)
        release_request(sv, r);
    sv->queue.clear();
    delete sv;
}

}  // namespace

extern "C" {

int dog_server_create(int device, const dog_params* params, const dog_server_opts* opts,
                      dog_server** out)
{
    if (!params || !out) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    *out = nullptr;
    dog::Plan P;
    std::string err;
    int rc = dog::build_plan(*params, &P, &err);
    if (rc != DOG_OK) {
        dog::set_error(err);
        return rc;
    }
    std::unique_ptr<dog_server> sv(new dog_server());
    sv->prm = *params;
    if (opts)
        sv->opts = *opts;
    sv->pool.reset(new PinnedPool(sv->opts.dry_run ? 0 : (4ull << 30)));
    if (sv->opts.max_batch_frames <= 0)
        sv->opts.max_batch_frames = 16;
    if (sv->opts.slots <= 0)
        sv->opts.slots = 3;
    if (sv->opts.max_batch_pixels == 0)
        sv->opts.max_batch_pixels = (int64_t)1 << 20;
    if (sv->opts.queue_capacity <= 0)
        sv->opts.queue_capacity = 4096;
    if (sv->opts.max_wait_ms < 0.0 || sv->opts.dry_run_us_per_mpx < 0.0) {
        dog::set_error("negative batching window or dry-run time");
        return DOG_EINVAL;
    }
    sv->n_g = P.n_g;
    sv->plan = P;
    sv->budget = sv->opts.hbm_budget_bytes;
    if (!sv->opts.dry_run) {
        for (int i = 0; i < sv->opts.slots; ++i) {
            auto sl = std::make_unique<Slot>();
            rc = dog_context_create(device, sv->budget, &sl->ctx);
            // slots already run batches side by side: each batch is one
            // launch sequence, not split again over lanes of its own; every
            // byte a slot allocates is committed by admission
            if (rc == DOG_OK) {
                sl->ctx->group_pixels = 0;
                sl->ctx->exact_alloc = true;
                sl->ctx->room_margin = 0;
            }
            if (rc == DOG_OK && sv->opts.tune_cache) {
                rc = dog_autotune_load(sl->ctx, sv->opts.tune_cache);
                if (rc != DOG_OK)
                    dog_context_destroy(sl->ctx);
            }
            if (rc != DOG_OK) {
                for (auto& s : sv->slots)
                    dog_context_destroy(s->ctx);
                return rc;
            }
            sv->slots.push_back(std::move(sl));
        }
        if (sv->budget == 0)
            sv->budget = sv->slots[0]->ctx->budget;
        for (auto& s : sv->slots)
            s->ctx->budget = 0;  // nothing is allocated before admission
    } else {
        for (int i = 0; i < sv->opts.slots; ++i)
            sv->slots.push_back(std::make_unique<Slot>());
        if (sv->budget == 0)
            sv->budget = 1ull << 40;
    }
    sv->opts.tune_cache = nullptr;  // read above only; the caller's string may go away
    dog_server* raw = sv.release();
    for (auto& s : raw->slots) {
        Slot* sp = s.get();
        sp->th = std::thread(run_slot, raw, sp);
    }
    raw->dispatcher = std::thread(run_dispatcher, raw);
    *out = raw;
    return DOG_OK;
}

int dog_server_submit(dog_server* sv, const dog_frame* frame, uint64_t* ticket)
{
    if (!sv || !frame || !ticket) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    *ticket = 0;
    int rc = dog::check_image(frame->data, frame->height, frame->width, frame->row_stride);
    if (rc != DOG_OK)
        return rc;
    if (frame->on_device != 0 && frame->on_device != 1) {
        dog::set_error("on_device must be 0 (host) or 1 (device) for a server request");
        return DOG_EINVAL;
    }
    Request r;
    r.H = frame->height;
    r.W = frame->width;
    r.on_device = frame->on_device == 1;
    {
        Slot empty;
        r.footprint = slot_commit(sv, &empty, {}, &r);  // the frame alone on a fresh slot
    }
    if (r.footprint > sv->budget) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->rejected += 1;
        dog::set_error("frame footprint exceeds the server's HBM budget");
        return DOG_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if ((int64_t)sv->queue.size() >= sv->opts.queue_capacity) {
            sv->rejected += 1;
            dog::set_error("server queue full");
            return DOG_EBUSY;
        }
    }
    r.t_arrive = now_ns();
    if (r.on_device) {
        r.data = frame->data;
        r.stride = frame->row_stride;
    } else {
        const size_t row_bytes = (size_t)r.W * sizeof(float);
        float* p = static_cast<float*>(sv->pool->get(row_bytes * (size_t)r.H, &r.bytes, &r.pinned));
        if (!p) {
            dog::set_error("out of host memory");
            return DOG_ENOMEM;
        }
        if (frame->row_stride == r.W) {
            std::memcpy(p, frame->data, row_bytes * (size_t)r.H);
        } else {
            for (int64_t y = 0; y < r.H; ++y)
                std::memcpy(p + y * r.W, frame->data + y * frame->row_stride, row_bytes);
        }
        r.data = p;
        r.stride = r.W;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r.ticket = sv->next_ticket++;
        *ticket = r.ticket;
        sv->pending.insert(r.ticket);
        sv->submitted += 1;
        if (sv->t_first == 0)
            sv->t_first = r.t_arrive;
        sv->queue.push_back(std::move(r));
    }
    sv->cv_dispatch.notify_all();
    return DOG_OK;
}

static int take_result(dog_server* sv, uint64_t ticket, dog_result* out)
{
    auto it = sv->done.find(ticket);
    if (it == sv->done.end())
        return sv->pending.count(ticket) ? DOG_EAGAIN : DOG_ENOTFOUND;
    *out = it->second;
    sv->done.erase(it);
    return DOG_OK;
}

int dog_server_poll(dog_server* sv, uint64_t ticket, dog_result* out)
{
    if (!sv || !out) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lk(sv->mu);
    const int rc = take_result(sv, ticket, out);
    if (rc == DOG_ENOTFOUND)
        dog::set_error("unknown ticket");
    return rc;
}

int dog_server_wait(dog_server* sv, uint64_t ticket, dog_result* out)
{
    if (!sv || !out) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        const int rc = take_result(sv, ticket, out);
        if (rc != DOG_EAGAIN) {
            if (rc == DOG_ENOTFOUND)
                dog::set_error("unknown ticket");
            return rc;
        }
        sv->cv_done.wait(lk);
    }
}

int dog_server_drain(dog_server* sv)
{
    if (!sv) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->pending.empty(); });
    return DOG_OK;
}

int dog_server_stats(dog_server* sv, dog_stats* out)
{
    if (!sv || !out) {
        dog::set_error("invalid argument");
        return DOG_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lk(sv->mu);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->failed = sv->failed;
    out->rejected = sv->rejected;
    out->queued = (int64_t)sv->queue.size();
    out->running = sv->running;
    out->batches = sv->batches;
    out->mean_batch_frames = sv->batches ? (double)sv->batch_frames / (double)sv->batches : 0.0;
    out->reserved_bytes = sv->reserved;
    out->peak_reserved_bytes = sv->peak_reserved;
    for (const auto& s : sv->slots)
        out->held_bytes += s->held();
    out->peak_held_bytes = sv->peak_held;
    out->admission_waits = sv->admission_waits;
    if (!sv->lat_ms.empty()) {
        std::vector<double> v = sv->lat_ms;
        std::sort(v.begin(), v.end());
        auto q = [&](double p) {
            // linear interpolation between closest ranks
            const double pos = p * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
        };
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        double s = 0;
        for (double x : v)
            s += x;
        out->mean_ms = s / (double)v.size();
        out->max_ms = v.back();
    }
    if (sv->t_last > sv->t_first && sv->completed > 0)
        out->frames_per_s = (double)sv->completed / ((double)(sv->t_last - sv->t_first) * 1e-9);
    return DOG_OK;
}

void dog_server_destroy(dog_server* sv) { destroy_server(sv); }

}  // extern "C"
