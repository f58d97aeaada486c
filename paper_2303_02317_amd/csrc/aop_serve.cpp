// aop_serve.cpp -- continuous-batching server of libaop (declared in include/aop.h).
//
// A scheduler thread owns a device arena (the HBM budget) and up to
// max_inflight launch slots, each with its own HIP stream, pinned staging
// buffers and completion event.  Whenever a slot is free it forms a batch from
// the pending requests: the oldest request fixes the size class (model,
// ceil(log2 T)), and younger requests of the same class join it in arrival
// order up to max_batch, as long as the batch's workspace fits in one free
// block of the arena (admission by HBM footprint).  The batch is priced by the
// persistent solve kernel on 1/max_inflight of the compute units, so batches
// admitted while others run overlap on the device.  A finished slot's prices
// are handed back with their queueing and total latency, and its arena block
// is freed for the next admissions.
//
// Every option's schedule depends only on that option (never on the batch it
// shares), so its price is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "aop.h"
#include "aop_host.h"
#include "aop_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

double seconds_since(clock_type::time_point t0, clock_type::time_point t)
{
    return std::chrono::duration<double>(t - t0).count();
}

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
  public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
    }
    // Largest free block (the admission bound).
    size_t largest() const
    {
        size_t m = 0;
        for (const auto &b : free_) m = std::max(m, b.second);
        return m;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = aop::ws_align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t noff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = aop::ws_align(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Request {
    aop_option opt;
    uint64_t id;
    clock_type::time_point submitted;
    int klass;     // size class: model * 64 + ceil(log2 T)
    size_t bytes;  // workspace area of the option
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request> reqs;
    std::vector<aop_option> opts;
    aop::Desc *h_desc = nullptr;  // pinned
    double *h_price = nullptr;    // pinned
    aop::Stats *h_stats = nullptr;  // pinned: the batch's work counters
    int cap = 0;
    size_t off = 0, bytes = 0;
    clock_type::time_point launched;
};

int size_class(const aop_option &o)
{
    int l = 0;
    while (l < 62 && (int64_t(1) << l) < o.T) ++l;
    return o.model * 64 + l;
}

}  // namespace

struct aop_server {
    aop_ctx *ctx = nullptr;
    aop_server_config cfg{};
    char *d_arena = nullptr;
    size_t arena_bytes = 0;
    Arena arena;
    std::vector<Slot> slots;
    int wg_per_batch = 1;
    std::vector<aop_class_tuning> tunings;  // per size class (may be empty)

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    std::vector<aop_result> results;
    bool stop = false;
    aop_status error = AOP_OK;
    int64_t submitted = 0, completed = 0, batches = 0, inflight = 0;
    int64_t alg_bytes = 0;  // algorithmic HBM bytes of the finished batches (correlation inputs and outputs)
    std::thread worker;

    void run();
    bool launch(Slot &sl, std::vector<Request> &&batch, size_t bytes);
    void finish(Slot &sl);
};

bool aop_server::launch(Slot &sl, std::vector<Request> &&batch, size_t bytes)
{
    const int64_t n = (int64_t)batch.size();
    sl.reqs = std::move(batch);
    sl.opts.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) sl.opts[(size_t)i] = sl.reqs[(size_t)i].opt;
    std::vector<int32_t> st((size_t)n);
    const size_t need = aop::build_batch(sl.opts.data(), n, cfg.precision, ctx->lambda, sl.h_desc, st.data());
    if (need > bytes) return false;
    char *ws = d_arena + sl.off;
    double *d_price = (double *)(ws + need);  // prices after the batch's own workspace
    // the schedule of the batch's class: the tuned entry nearest in log2 T
    const aop_tuning *tsel = &ctx->tuning;
    int best = 1 << 30;
    for (const auto &e : tunings) {
        if (e.model != sl.opts[0].model || e.precision != cfg.precision) continue;
        const int d = std::abs(e.log2T - (sl.reqs[0].klass & 63));
        if (d < best) {
            best = d;
            tsel = &e.tuning;
        }
    }
    aop::Tune tune = aop::make_tune(*tsel, ctx->tick_hz, wg_per_batch);
    tune.prec = cfg.precision;
    if (hipMemcpyAsync(ws, sl.h_desc, sizeof(aop::Desc) * (size_t)n, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        return false;
    if (aop::launch_solve((const aop::Desc *)ws, n, ws, ctx->d_tw, d_price, nullptr, 0, nullptr, tune, sl.stream) != 0)
        return false;
    if (hipMemcpyAsync(sl.h_price, d_price, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
        return false;
    if (hipMemcpyAsync(sl.h_stats, ws + aop::stats_offset(n), sizeof(aop::Stats) * (size_t)n, hipMemcpyDeviceToHost,
                       sl.stream) != hipSuccess)
        return false;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return false;
    sl.launched = clock_type::now();
    sl.busy = true;
    return true;
}

void aop_server::finish(Slot &sl)
{
    const auto now = clock_type::now();
    std::vector<aop_result> out(sl.reqs.size());
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        aop_result &r = out[i];
        r.id = sl.reqs[i].id;
        r.price = sl.h_price[i];
        r.status = std::isnan(r.price) ? AOP_EDEVICE : AOP_OK;
        r.batch_size = (int32_t)sl.reqs.size();
        r.queue_s = seconds_since(sl.reqs[i].submitted, sl.launched);
        r.latency_s = seconds_since(sl.reqs[i].submitted, now);
    }
    int64_t bytes = 0;
    for (size_t i = 0; i < sl.reqs.size(); ++i)
        bytes += 8 * (sl.h_stats[i].conv_in + sl.h_stats[i].conv_out + sl.h_stats[i].direct_cells);
    arena.release(sl.off, sl.bytes);
    sl.busy = false;
    sl.reqs.clear();
    std::lock_guard<std::mutex> g(mu);
    for (auto &r : out) results.push_back(r);
    completed += (int64_t)out.size();
    alg_bytes += bytes;
    --inflight;
    cv.notify_all();
}

void aop_server::run()
{
    if (hipSetDevice(ctx->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        error = AOP_EDEVICE;
        return;
    }
    for (;;) {
        // completions
        for (auto &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finish(sl);
            } else if (q != hipErrorNotReady) {
                // a device error: report the slot's requests as failed and stop
                for (size_t i = 0; i < sl.reqs.size(); ++i) sl.h_price[i] = NAN;
                finish(sl);
                std::lock_guard<std::mutex> g(mu);
                error = AOP_EDEVICE;
                stop = true;
            }
        }
        // admissions
        std::unique_lock<std::mutex> lk(mu);
        if (stop && (pending.empty() || error != AOP_OK)) {
            bool any = false;
            for (auto &sl : slots) any = any || sl.busy;
            if (!any) break;
        }
        Slot *free_slot = nullptr;
        for (auto &sl : slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        bool launched = false;
        if (!pending.empty() && error == AOP_OK) {
            // a request that cannot fit even alone in the whole arena is refused
            const Request &r0 = pending.front();
            const size_t alone = aop::batch_fixed_bytes(1) + r0.bytes + aop::ws_align(sizeof(double));
            if (aop::ws_align(alone) > arena_bytes) {
                aop_result x{};
                x.id = r0.id;
                x.price = NAN;
                x.status = AOP_ENOMEM;
                x.batch_size = 0;
                results.push_back(x);
                ++completed;
                pending.pop_front();
                cv.notify_all();
                continue;
            }
        }
        if (free_slot && !pending.empty() && error == AOP_OK) {
            const int klass = pending.front().klass;
            const size_t room = arena.largest();
            std::vector<Request> batch;
            std::vector<size_t> taken;
            size_t area = 0;
            for (size_t i = 0; i < pending.size() && (int)batch.size() < cfg.max_batch; ++i) {
                const Request &r = pending[i];
                if (r.klass != klass) continue;
                const size_t need = aop::batch_fixed_bytes((int64_t)batch.size() + 1) + area + r.bytes +
                                    aop::ws_align(sizeof(double) * (batch.size() + 1));
                if (need > room) break;
                area += r.bytes;
                batch.push_back(r);
                taken.push_back(i);
            }
            if (!batch.empty()) {
                for (size_t k = taken.size(); k-- > 0;) pending.erase(pending.begin() + (std::ptrdiff_t)taken[k]);
                const size_t bytes = aop::batch_fixed_bytes((int64_t)batch.size()) + area +
                                     aop::ws_align(sizeof(double) * batch.size());
                ++inflight;
                ++batches;
                lk.unlock();
                size_t off = 0;
                bool ok = arena.alloc(bytes, &off);
                if (ok) {
                    free_slot->off = off;
                    free_slot->bytes = bytes;
                    ok = launch(*free_slot, std::move(batch), bytes);
                    if (!ok) arena.release(off, bytes);
                }
                if (!ok) {
                    std::lock_guard<std::mutex> g(mu);
                    error = AOP_EDEVICE;
                    stop = true;
                    --inflight;
                    for (auto &r : free_slot->reqs.empty() ? batch : free_slot->reqs) {
                        aop_result x{};
                        x.id = r.id;
                        x.price = NAN;
                        x.status = AOP_EDEVICE;
                        results.push_back(x);
                        ++completed;
                    }
                    free_slot->reqs.clear();
                }
                launched = true;
                lk.lock();
            }
        }
        if (!launched) {
            // nothing to start: wait for a submission or poll the device again soon
            bool busy = false;
            for (auto &sl : slots) busy = busy || sl.busy;
            cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 2000));
        }
    }
    // fail whatever is still queued
    std::lock_guard<std::mutex> g(mu);
    for (auto &r : pending) {
        aop_result x{};
        x.id = r.id;
        x.price = NAN;
        x.status = AOP_ECANCELED;
        results.push_back(x);
    }
    pending.clear();
    cv.notify_all();
}

extern "C" {

aop_status aop_server_create(aop_ctx *ctx, const aop_server_config *cfg, aop_server **out)
{
    if (!ctx || !cfg || !out) return AOP_EINVAL;
    *out = nullptr;
    aop_server_config c = *cfg;
    if (c.max_inflight < 1 || c.max_inflight > 16 || c.max_batch < 1 || c.max_batch > 4096 ||
        (c.precision != AOP_FP64 && c.precision != AOP_MIXED) || c.reserved != 0)
        return AOP_EINVAL;
    if (!c.d_arena || (reinterpret_cast<uintptr_t>(c.d_arena) & (aop::WS_ALIGN - 1)) != 0 ||
        c.hbm_budget < aop::WS_ALIGN)
        return AOP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    if (c.n_tunings < 0 || (c.n_tunings > 0 && !c.tunings)) return AOP_EINVAL;
    for (int64_t i = 0; i < c.n_tunings; ++i) {
        aop_tuning t = c.tunings[i].tuning;
        t.workgroups = 1;  // replaced per batch
        if (!aop::tuning_valid(t) || c.tunings[i].reserved != 0) return AOP_EINVAL;
    }
    aop_server *s = new (std::nothrow) aop_server;
    if (!s) return AOP_ENOMEM;
    s->ctx = ctx;
    s->cfg = c;
    s->tunings.assign(c.tunings, c.tunings + c.n_tunings);
    s->cfg.tunings = nullptr;
    s->arena_bytes = c.hbm_budget / aop::WS_ALIGN * aop::WS_ALIGN;
    s->d_arena = (char *)c.d_arena;  // the caller's memory
    s->arena.reset(s->arena_bytes);
    s->wg_per_batch = std::max(1, std::min(aop::MAX_WG, ctx->n_cu / c.max_inflight));
    s->slots.resize((size_t)c.max_inflight);
    aop_status st = AOP_OK;
    for (auto &sl : s->slots) {
        sl.cap = c.max_batch;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_desc, sizeof(aop::Desc) * (size_t)sl.cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_price, sizeof(double) * (size_t)sl.cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_stats, sizeof(aop::Stats) * (size_t)sl.cap, hipHostMallocDefault) != hipSuccess)
            st = AOP_EDEVICE;
    }
    if (st != AOP_OK) {
        aop_server_destroy(s);
        return st;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return AOP_OK;
}

aop_status aop_server_submit(aop_server *s, const aop_option *opts, const uint64_t *ids, int64_t n)
{
    if (!s || n < 0 || (n > 0 && (!opts || !ids))) return AOP_EINVAL;
    const auto now = std::chrono::steady_clock::now();
    std::vector<aop_result> rejected;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return AOP_ECANCELED;
        for (int64_t i = 0; i < n; ++i) {
            const aop_status v = aop_validate(&opts[i], s->ctx->lambda);
            if (v != AOP_OK) {
                aop_result r{};
                r.id = ids[i];
                r.price = NAN;
                r.status = v;
                s->results.push_back(r);
                ++s->completed;
                ++s->submitted;
                continue;
            }
            Request q;
            q.opt = opts[i];
            q.id = ids[i];
            q.submitted = now;
            q.klass = size_class(opts[i]);
            q.bytes = aop::option_area_bytes(opts[i], s->ctx->lambda);
            s->pending.push_back(q);
            ++s->submitted;
        }
    }
    s->cv.notify_all();
    return AOP_OK;
}

aop_status aop_server_poll(aop_server *s, aop_result *out, int64_t max, int64_t *n_out, int32_t wait_us)
{
    if (!s || !n_out || max < 0 || (max > 0 && !out)) return AOP_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && wait_us > 0)
        s->cv.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->results.empty() || s->error; });
    const int64_t k = std::min<int64_t>(max, (int64_t)s->results.size());
    for (int64_t i = 0; i < k; ++i) out[i] = s->results[(size_t)i];
    s->results.erase(s->results.begin(), s->results.begin() + k);
    *n_out = k;
    return s->error;
}

aop_status aop_server_stats(aop_server *s, int64_t *out)
{
    if (!s || !out) return AOP_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    out[0] = s->submitted;
    out[1] = s->completed;
    out[2] = s->batches;
    out[3] = s->inflight;
    out[4] = (int64_t)s->pending.size();
    out[5] = (int64_t)s->arena.peak();
    out[6] = (int64_t)s->arena_bytes;
    out[7] = s->wg_per_batch;
    out[8] = s->alg_bytes;
    return AOP_OK;
}

aop_status aop_server_destroy(aop_server *s)
{
    if (!s) return AOP_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_desc) (void)hipHostFree(sl.h_desc);
        if (sl.h_price) (void)hipHostFree(sl.h_price);
        if (sl.h_stats) (void)hipHostFree(sl.h_stats);
    }
    delete s;  // the arena belongs to the caller
    return AOP_OK;
}

}  // extern "C"
