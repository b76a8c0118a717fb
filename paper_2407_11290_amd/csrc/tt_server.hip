// tt_server.hip -- continuous-batching server for TT-cross solves on one GPU.
//
// Requests arrive through tt_server_submit at any time.  A server thread
// admits them into the batch engine (tt_batch.hip) while others are in
// flight.  A request is admitted when an engine slot is free and a problem
// object of its shape fits the HBM budget.  Problem objects, with all their
// device buffers, are pooled by shape (modes, subtensor grid, sweep
// precision, rank cap), so after warm-up no request allocates device memory.
// When a solve ends, its stats and cores are copied out to the request and
// the problem object goes back to the pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "tt_batch.h"
#include "tt_cross.h"
#include "tt_internal.h"

namespace ttc {

static double wall_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int d = 0;
    int n[TT_MAX_D] = {0};
    double eps = 0;
    int fn_id = 0;
    std::vector<double> params;
    uint64_t seed = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;                // 0 queued, 1 running, 2 done
    bool force64 = false;         // FP32 sweeps missed eps: solve again with FP64 sweeps
    int status = TT_OK;
    tt_stats stats;
    std::vector<double> cores;
    Problem *Q = nullptr;
};

struct PoolEntry {
    std::unique_ptr<tt_cross_s> h;
    bool busy = false;
    size_t bytes = 0;
    double last_used = 0;
};

class Server {
public:
    Server(size_t budget, int slots, const tt_options &o) : budget_(budget), opt_(o), slots_(slots) {}
    ~Server() { stop(); }

    int start()
    {
        HIPCHK(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        const int st = eng_.init(slots_, stream_);
        if (st) return st;
        th_ = std::thread([this] { loop(); });
        return TT_OK;
    }

    void stop()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        if (th_.joinable()) th_.join();
        if (stream_) (void)hipStreamSynchronize(stream_);
        pool_.clear();
        eng_.release();
        if (stream_) { (void)hipStreamDestroy(stream_); stream_ = nullptr; }
    }

    int submit(int d, const int32_t *n, double eps, int fn_id, const double *params, int nparams, uint64_t seed,
               uint64_t *ticket)
    {
        // validate on the caller's thread, so bad requests fail here
        FnHost f;
        int st = build_fn(fn_id, d, n, params, nparams, f);
        if (st) return st;
        if (fn_id == TT_FN_SEPSUM) return set_err(TT_EFN, "the server takes no separable sums (caller-supplied factor tables)");
        if (!(eps >= 0.0) || !(eps < 1.0)) return set_err(TT_EINVAL, "eps must be in [0,1)");
        auto r = std::make_unique<Request>();
        r->d = d;
        for (int j = 0; j < d; ++j) r->n[j] = n[j];
        r->eps = eps;
        r->fn_id = fn_id;
        if (nparams > 0) r->params.assign(params, params + nparams);
        r->seed = seed;
        r->t_submit = wall_s();
        std::memset(&r->stats, 0, sizeof r->stats);
        {
            std::lock_guard<std::mutex> g(mu_);
            if (loop_err_) return set_err(loop_err_, "server stopped after a device error");
            r->ticket = ++next_;
            *ticket = r->ticket;
            queue_.push_back(r.get());
            reqs_[r->ticket] = std::move(r);
        }
        cv_.notify_all();
        return TT_OK;
    }

    int poll(uint64_t t)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return set_err(TT_EINVAL, "unknown ticket");
        if (loop_err_ && it->second->state != 2) return set_err(loop_err_, "server stopped after a device error");
        return it->second->state == 2 ? 1 : 0;
    }

    int wait(uint64_t t, double *latency)
    {
        std::unique_lock<std::mutex> g(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return set_err(TT_EINVAL, "unknown ticket");
        Request *r = it->second.get();
        done_cv_.wait(g, [&] { return r->state == 2 || loop_err_; });
        if (r->state != 2) return set_err(loop_err_, "server stopped after a device error");
        if (latency) *latency = r->t_done - r->t_submit;
        return r->status;
    }

    int64_t result(uint64_t t, tt_stats *st, double *cores, int64_t cap)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return set_err(TT_EINVAL, "unknown ticket");
        Request *r = it->second.get();
        if (r->state != 2) return set_err(TT_ESTATE, "request not finished");
        if (st) *st = r->stats;
        const int64_t len = (int64_t)r->cores.size();
        if (cores) {
            if (cap < len) return set_err(TT_EINVAL, "cap %lld < %lld", (long long)cap, (long long)len);
            std::memcpy(cores, r->cores.data(), sizeof(double) * len);
        }
        return len;
    }

    int release(uint64_t t)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return set_err(TT_EINVAL, "unknown ticket");
        if (it->second->state != 2) return set_err(TT_ESTATE, "request not finished");
        reqs_.erase(it);
        return TT_OK;
    }

    void counters(tt_server_stats *s)
    {
        std::lock_guard<std::mutex> g(mu_);
        std::memset(s, 0, sizeof *s);
        s->submitted = next_;
        s->completed = completed_;
        s->queued = (int64_t)queue_.size();
        s->running = running_;
        s->pool_bytes = (int64_t)pool_bytes_;
        s->pool_objects = (int64_t)pool_.size();
        s->allocations = allocations_;
    }

private:
    // key of the buffers a request needs
    struct Key {
        int d, fp32, rmax;
        int n[TT_MAX_D], grid[TT_MAX_D];
        bool operator<(const Key &o) const { return std::memcmp(this, &o, sizeof(Key)) < 0; }
    };

    Key key_of(const Request &r) const
    {
        Key k;
        std::memset(&k, 0, sizeof k);
        k.d = r.d;
        int prec = opt_.precision;
        if (prec == TT_PREC_AUTO) prec = (r.eps >= 1e-6) ? TT_PREC_FP32 : TT_PREC_FP64;
        if (r.force64) prec = TT_PREC_FP64;
        k.fp32 = (prec == TT_PREC_FP32);
        k.rmax = opt_.r_max;
        for (int j = 0; j < r.d; ++j) {
            k.n[j] = r.n[j];
            k.grid[j] = std::max(1, std::min(opt_.grid[j], r.n[j]));
        }
        return k;
    }

    // a pooled problem for r, or nullptr if none can be had right now.  Only
    // may_grow callers create objects; a shape that already has objects (all
    // busy) waits for one of them rather than evicting other shapes, because
    // freeing device memory stalls the whole device.
    Problem *acquire(const Request &r, int &err, bool may_grow)
    {
        err = TT_OK;
        const Key k = key_of(r);
        auto range = pool_.equal_range(k);
        PoolEntry *pick = nullptr;
        bool have_shape = false;
        for (auto it = range.first; it != range.second; ++it) {
            have_shape = true;
            if (!it->second.busy) { pick = &it->second; break; }
        }
        if (!pick && !may_grow) return nullptr;
        if (!pick) {
            // a new problem object of this shape, after evicting idle ones of
            // other shapes if the budget needs it
            std::unique_ptr<tt_cross_s> h(new (std::nothrow) tt_cross_s());
            if (!h) { err = set_err(TT_ENOMEM, "out of host memory"); return nullptr; }
            Problem &P = h->p;
            if ((err = build_fn(r.fn_id, r.d, r.n, r.params.data(), (int)r.params.size(), P.fn)) != TT_OK) return nullptr;
            P.d = r.d;
            for (int j = 0; j < r.d; ++j) P.n[j] = r.n[j];
            P.eps = r.eps;
            P.opt = opt_;
            P.opt.stream = stream_;
            P.opt.seed = r.seed;
            P.force_fp64 = r.force64;
            P.resolve_geometry();
            const size_t need = P.device_bytes();
            if (need > budget_) { err = set_err(TT_ENOMEM, "request needs %zu B, budget %zu B", need, budget_); return nullptr; }
            if (have_shape && pool_bytes_ + need > budget_) return nullptr;
            while (pool_bytes_ + need > budget_) {
                auto victim = pool_.end();
                for (auto it = pool_.begin(); it != pool_.end(); ++it)
                    if (!it->second.busy && (victim == pool_.end() || it->second.last_used < victim->second.last_used))
                        victim = it;
                if (victim == pool_.end()) return nullptr;      // everything resident is busy: wait
                pool_bytes_ -= victim->second.bytes;
                pool_.erase(victim);
            }
            if ((err = P.prepare()) != TT_OK) return nullptr;
            ++allocations_;
            PoolEntry e;
            e.h = std::move(h);
            e.bytes = need;
            pool_bytes_ += need;
            auto it = pool_.emplace(k, std::move(e));
            pick = &it->second;
        }
        Problem &P = pick->h->p;
        FnHost f;
        if ((err = build_fn(r.fn_id, r.d, r.n, r.params.data(), (int)r.params.size(), f)) != TT_OK) return nullptr;
        P.fn.dev = f.dev;
        P.fn.table.swap(f.table);
        if ((err = upload_fn(P.fn, stream_)) != TT_OK) return nullptr;
        P.hP.F = P.fn.dev;
        P.eps = r.eps;
        P.opt.seed = r.seed;
        P.force_fp64 = r.force64;
        if ((err = P.prepare()) != TT_OK) return nullptr;
        pick->busy = true;
        pick->last_used = wall_s();
        return &P;
    }

    void give_back(Problem *Q)
    {
        for (auto &kv : pool_)
            if (&kv.second.h->p == Q) { kv.second.busy = false; kv.second.last_used = wall_s(); return; }
    }

    void loop()
    {
        std::vector<int> done;
        bool admitted = false;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                if (quit_) break;
                if (queue_.empty() && eng_.idle())
                    cv_.wait_for(g, std::chrono::milliseconds(20), [&] { return quit_ || !queue_.empty(); });
                if (quit_) break;
                // admit in arrival order while slots and budget allow; the
                // oldest request may create a problem object, later ones
                // (within a window) may pass it on idle pooled objects
                admitted = false;
                int scanned = 0;
                for (auto it = queue_.begin(); it != queue_.end() && eng_.free_slots() > 0 && scanned < 256;
                     ++scanned) {
                    Request *r = *it;
                    int err = TT_OK;
                    Problem *Q = acquire(*r, err, it == queue_.begin());
                    if (!Q) {
                        if (err) {          // the request can never run
                            r->status = err;
                            r->state = 2;
                            r->t_done = wall_s();
                            it = queue_.erase(it);
                            ++completed_;
                            done_cv_.notify_all();
                            continue;
                        }
                        ++it;               // waits for an object of its shape
                        continue;
                    }
                    const int slot = eng_.admit(Q, r);
                    if (slot < 0) { give_back(Q); loop_err_ = slot; break; }
                    r->Q = Q;
                    r->state = 1;
                    r->t_admit = wall_s();
                    ++running_;
                    admitted = true;
                    it = queue_.erase(it);
                }
            }
            done.clear();
            const int st = eng_.tick(&done);
            // nothing admitted, launched or finished: wait a little (the
            // engine's runtime queries would compete with its launches)
            if (!st && !eng_.busy_tick && !admitted) std::this_thread::sleep_for(std::chrono::microseconds(20));
            std::lock_guard<std::mutex> g(mu_);
            if (st) {
                loop_err_ = st;
                done_cv_.notify_all();
                break;
            }
            for (int idx : done) {
                const Slot &s = eng_.slot(idx);
                Request *r = (Request *)s.user;
                Problem &Q = *s.Q;
                if (s.escalate) {
                    // a13: back to the head of the queue, to be solved with FP64 sweeps
                    r->force64 = true;
                    r->state = 0;
                    r->Q = nullptr;
                    --running_;
                    give_back(&Q);
                    eng_.retire(idx);
                    queue_.push_front(r);
                    continue;
                }
                r->status = Q.ran ? Q.status : (Q.status ? Q.status : TT_EDEVICE);
                if (Q.ran) {
                    r->cores.resize((size_t)Q.cores_len);
                    if (hipMemcpy(r->cores.data(), Q.d_cores, sizeof(double) * Q.cores_len, hipMemcpyDeviceToHost) !=
                        hipSuccess)
                        r->status = TT_EDEVICE;
                }
                tt_stats &t = r->stats;
                std::memset(&t, 0, sizeof t);
                t.d = Q.d;
                t.status = r->status;
                if (Q.ran) {
                    t.evaluated = Q.evaluated;
                    t.pivoted = Q.pivoted;
                    t.samples = Q.opt.n_samples;
                    t.sweeps = Q.sweeps;
                    t.precision_used = Q.fp32 ? TT_PREC_FP32 : TT_PREC_FP64;
                    for (int k = 0; k <= Q.d; ++k) t.ranks[k] = Q.ranks[k];
                    t.rms = Q.rms;
                    t.tau = Q.tau;
                    t.sweep_alg_bytes = Q.sweep_alg_bytes;
                    t.new_entries = Q.new_entries;
                    for (int u = 0; u < Q.d - 1; ++u) t.last_best[u] = Q.last_best[u];
                }
                t.sampled_err = Q.sampled_err;
                t.escalated = r->force64 ? 1 : 0;
                r->t_done = wall_s();
                t.time_to_eps_s = r->t_done - r->t_admit;
                r->state = 2;
                r->Q = nullptr;
                --running_;
                ++completed_;
                give_back(&Q);
                eng_.retire(idx);
            }
            if (!done.empty()) done_cv_.notify_all();
        }
    }

    size_t budget_;
    tt_options opt_;
    int slots_;
    hipStream_t stream_ = nullptr;
    Engine eng_;
    std::thread th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    bool quit_ = false;
    int loop_err_ = 0;
    uint64_t next_ = 0;
    int64_t completed_ = 0, running_ = 0, allocations_ = 0;
    std::deque<Request *> queue_;
    std::map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::multimap<Key, PoolEntry> pool_;
    size_t pool_bytes_ = 0;
};

}  // namespace ttc

using namespace ttc;

struct tt_server_s {
    Server *s;
};

extern "C" {

tt_server_h tt_server_create(size_t hbm_budget, int max_slots, const tt_options *opt)
{
    if (hbm_budget == 0 || max_slots < 1 || max_slots > 65535) {
        set_err(TT_EINVAL, "bad server budget or slot count");
        return nullptr;
    }
    tt_options o;
    if (opt) o = *opt;
    else {
        tt_options_default(&o);
        o.r_max = 32;
        for (int j = 0; j < TT_MAX_D; ++j) o.grid[j] = 2;
    }
    if (o.pivot_mode != TT_PIVOT_GREEDY) {
        set_err(TT_EINVAL, "served solves use greedy pivoting (rook pivoting runs through tt_cross_run)");
        return nullptr;
    }
    if (o.r_max < 1 || o.r_max > TT_MAX_RANK || o.n_samples < 1) {
        set_err(TT_EINVAL, "bad server options");
        return nullptr;
    }
    for (int j = 0; j < TT_MAX_D; ++j)
        if (o.grid[j] < 1) { set_err(TT_EINVAL, "bad server grid"); return nullptr; }
    tt_server_s *h = new (std::nothrow) tt_server_s();
    if (!h) { set_err(TT_ENOMEM, "out of host memory"); return nullptr; }
    h->s = new (std::nothrow) Server(hbm_budget, max_slots, o);
    if (!h->s || h->s->start() != TT_OK) {
        delete h->s;
        delete h;
        return nullptr;
    }
    return h;
}

int tt_server_submit(tt_server_h h, int d, const int32_t *n, double eps, int fn_id, const double *params,
                     int nparams, uint64_t seed, uint64_t *ticket)
{
    if (!h || !ticket) return set_err(TT_EINVAL, "NULL argument");
    return h->s->submit(d, n, eps, fn_id, params, nparams, seed, ticket);
}

int tt_server_poll(tt_server_h h, uint64_t ticket)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    return h->s->poll(ticket);
}

int tt_server_wait(tt_server_h h, uint64_t ticket, double *latency_s)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    return h->s->wait(ticket, latency_s);
}

int64_t tt_server_result(tt_server_h h, uint64_t ticket, tt_stats *st, double *cores, int64_t cap)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    return h->s->result(ticket, st, cores, cap);
}

int tt_server_release(tt_server_h h, uint64_t ticket)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    return h->s->release(ticket);
}

int tt_server_get_stats(tt_server_h h, tt_server_stats *st)
{
    if (!h || !st) return set_err(TT_EINVAL, "NULL argument");
    h->s->counters(st);
    return TT_OK;
}

void tt_server_destroy(tt_server_h h)
{
    if (!h) return;
    delete h->s;
    delete h;
}

}  // extern "C"
