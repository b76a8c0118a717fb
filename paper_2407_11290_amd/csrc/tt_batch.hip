// tt_batch.hip -- many independent solves resident on one GPU at once.
//
// The engine keeps a table of slots.  Each slot holds one prepared problem
// (its own residual superblocks, index sets and cores) plus a descriptor in
// a device array shared by all slots.  Every launch covers all slots that
// are at the same phase:
//   setup  samples, rms/tau/first pivot and initial superblocks
//   sweep  one search launch and one commit launch per round, over all
//          slots still sweeping (each slot at its own sweep index; the
//          commit reads it from the slot's device state)
//   cores  Alg. 4 for all slots whose sweeps ended
// The host queues sweep rounds ahead of its view of each slot's stop flag,
// which the commits write to mapped host memory.  Slots may be admitted
// while others are sweeping (continuous batching); a finished slot frees its
// entry for the next admission.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstring>
#include <vector>

#include "tt_batch.h"
#include "tt_cross.h"
#include "tt_device.h"
#include "tt_internal.h"
#include "tt_kernels.h"

namespace ttc {

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Engine::~Engine() { release(); }

void Engine::release()
{
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    ev_free.clear();
    // events still held by slots, each destroyed once
    for (auto &eu : ev_users) (void)hipEventDestroy(eu.first);
    ev_users.clear();
    for (Slot &s : slots) s.ev = nullptr;
    if (dPa) (void)hipFree(dPa);
    if (dS) (void)hipFree(dS);
    if (hPa) (void)hipHostFree(hPa);
    if (hS) (void)hipHostFree(hS);
    if (hm) (void)hipHostFree(hm);
    if (hPart) (void)hipHostFree(hPart);
    dPa = nullptr; dS = nullptr; hPa = nullptr; hS = nullptr; dhS = nullptr; hm = nullptr; dhm = nullptr;
    dPart = nullptr; hPart = nullptr;
    shadow.clear();
    shadow_ok.clear();
    slots.clear();
    cap = 0;
}

int Engine::init(int capacity, hipStream_t s)
{
    release();
    if (capacity < 1 || capacity > 65535) return set_err(TT_EINVAL, "engine capacity %d outside [1,65535]", capacity);
    stream = s;
    cap = capacity;
    HIPCHK(hipMalloc(&dPa, sizeof(ProbDev) * cap));
    shadow.assign(cap, ProbDev{});
    shadow_ok.assign(cap, 0);
    HIPCHK(hipMalloc(&dS, sizeof(ProbState) * cap));
    HIPCHK(hipHostMalloc((void **)&hPa, sizeof(ProbDev) * cap, hipHostMallocDefault));
    // finished states and check partials are written by kernels straight
    // into mapped host memory (no copy per problem)
    HIPCHK(hipHostMalloc((void **)&hS, sizeof(ProbState) * cap, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&dhS, hS, 0));
    HIPCHK(hipHostMalloc((void **)&hm, sizeof(HostMirror) * cap, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&dhm, hm, 0));
    HIPCHK(hipHostMalloc((void **)&hPart, sizeof(double) * 2 * NBV * cap, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&dPart, hPart, 0));
    std::memset(hm, 0, sizeof(HostMirror) * cap);
    slots.assign(cap, Slot());
    for (int i = 0; i < cap; ++i) slots[i].idx = i;
    return TT_OK;
}

int Engine::free_slots() const
{
    int f = 0;
    for (const Slot &s : slots) f += (s.phase == Slot::FREE) ? 1 : 0;
    return f;
}

int Engine::busy() const { return cap - free_slots(); }

int Engine::admit(Problem *Q, void *user)
{
    int i = -1;
    for (int j = 0; j < cap; ++j)
        if (slots[j].phase == Slot::FREE) { i = j; break; }
    if (i < 0) return set_err(TT_ESTATE, "no free slot");
    if (!Q->allocated) return set_err(TT_ESTATE, "problem not prepared");
    Slot &s = slots[i];
    s = Slot();
    s.idx = i;
    s.Q = Q;
    s.user = user;
    s.phase = Slot::SETUP;
    s.t_admit = now_s();
    for (int k = 0; k <= Q->d; ++k) s.rub[k] = s.rst[k] = 1;
    s.verify_R = Q->verify_samples();
    s.can_escalate = Q->auto_fp32();
    Q->sampled_err = -1.0;
    Q->escalated = Q->force_fp64 ? 1 : 0;
    ProbDev &D = hPa[i];
    D = Q->hP;
    D.S = dS + i;
    D.hm = dhm + i;
    D.run.seed = Q->opt.seed;
    D.run.eps = Q->eps;
    D.run.ns = Q->opt.n_samples;
    D.run.vals = Q->d_vals;
    D.run.spart = Q->d_spart;
    D.run.cores = Q->d_cores;
    D.run.verify_R = s.verify_R;
    std::memset(&hm[i], 0, sizeof(HostMirror));
    // the descriptor goes to the device with the others of its setup launch
    Q->ran = false;
    return i;
}

// Copies entries ids of a per-slot array between host and device on the
// engine's stream: one copy over their index range when the range is dense
// or small, else one copy per entry.  Everything the engine does runs on
// this one stream, so a range copy overlaps no kernel.  The other entries it
// covers are either those of live slots (the same bytes: descriptors do not
// change after admission, and a finished slot's state no longer changes),
// or of free slots, or of slots whose own copy comes later on the stream.
int Engine::copy_slots(void *dst, const void *src, size_t elem, const std::vector<int> &ids, hipMemcpyKind kind)
{
    if (ids.empty()) return TT_OK;
    int lo = ids[0], hi = ids[0];
    for (int i : ids) { lo = std::min(lo, i); hi = std::max(hi, i); }
    const size_t span = (size_t)(hi - lo + 1);
    // one copy when the range is dense or small; a wide sparse range copied
    // whole measured slower than its entries one by one
    if (span <= 4 * ids.size() || span * elem <= ((size_t)64 << 10)) {
        HIPCHK(hipMemcpyAsync((char *)dst + lo * elem, (const char *)src + lo * elem, span * elem, kind, stream));
    } else {
        for (int i : ids)
            HIPCHK(hipMemcpyAsync((char *)dst + (size_t)i * elem, (const char *)src + (size_t)i * elem, elem, kind, stream));
    }
    return TT_OK;
}

// Launch setup for every slot admitted since the last call.
template <typename V> int Engine::launch_setup(std::vector<int> &ids)
{
    // only descriptors that differ from what the device array already holds
    // are copied: a batch of the same problems run again copies none
    std::vector<int> changed;
    for (int i : ids)
        if (!shadow_ok[i] || std::memcmp(&shadow[i], &hPa[i], sizeof(ProbDev)) != 0) changed.push_back(i);
    int cst = copy_slots(dPa, hPa, sizeof(ProbDev), changed, hipMemcpyHostToDevice);
    if (cst) return cst;
    for (int i : changed) {
        shadow[i] = hPa[i];
        shadow_ok[i] = 1;
    }
    for (size_t c0 = 0; c0 < ids.size(); c0 += MAXB) {
        const int na = (int)std::min<size_t>(MAXB, ids.size() - c0);
        BatchMap bm;
        bm.na = na;
        int xs = 1, maxnk = 1, xi = 1;
        for (int a = 0; a < na; ++a) {
            const Slot &s = slots[ids[c0 + a]];
            const Problem &Q = *s.Q;
            bm.p[a] = (uint16_t)s.idx;
            bm.boff[a] = a;
            xs = std::max(xs, sample_blocks(Q.opt.n_samples));
            maxnk = std::max(maxnk, Q.d - 1);
            for (int u = 0; u < Q.d - 1; ++u) xi = std::max(xi, (Q.n[u] * Q.n[u + 1] + NT - 1) / NT);
        }
        bm.boff[na] = na;
        xi = std::min(xi, 1024);
        k_samples_b<<<dim3(xs, na), NT, 0, stream>>>(dPa, bm);
        k_setup_b<V><<<na, NT, 0, stream>>>(dPa, bm);
        k_init_eval_b<V><<<dim3(xi, maxnk, na), NT, 0, stream>>>(dPa, bm);
        HIPCHK(hipGetLastError());
    }
    return TT_OK;
}

// One search + commit round over the given sweeping slots.
template <typename V> int Engine::launch_sweep(std::vector<int> &ids)
{
    for (size_t c0 = 0; c0 < ids.size(); c0 += MAXB) {
        const int na = (int)std::min<size_t>(MAXB, ids.size() - c0);
        BatchMap bm;
        bm.na = na;
        int off = 0;
        size_t lds = 0;
        for (int a = 0; a < na; ++a) {
            Slot &s = slots[ids[c0 + a]];
            const Problem &Q = *s.Q;
            const int d = Q.d;
            // work units as the single-problem launch counts them: new tiles
            // one per workgroup, stored tiles four (the kernel strides over
            // the exact count, so a wrong estimate costs time only)
            int tot = 0;
            for (int u = 0; u < d - 1; ++u) {
                const int k = u + 1;
                const KDev &K = Q.hP.kd[u];
                const int all = s.rub[k - 1] * K.RTp * s.rub[k + 1] * K.CTq;
                const int st = std::min(all, s.rst[k - 1] * K.RTp * s.rst[k + 1] * K.CTq);
                tot += (all - st) + (st + NT / 64 - 1) / (NT / 64);
                lds = std::max(lds, sweep_lds_bytes(s.rub[k], K.TR, K.TC, sizeof(V)));
            }
            bm.p[a] = (uint16_t)s.idx;
            bm.boff[a] = off;
            off += std::max(1, std::min(tot, Q.sweep_grid_cap));
            ++s.launched;
            for (int k = 0; k <= d; ++k) s.rst[k] = s.rub[k];
            for (int k = 1; k <= d - 1; ++k) s.rub[k] = std::min(s.rub[k] + 1, Q.rc[k]);
        }
        bm.boff[na] = off;
        k_sweep_b<V><<<off, NT, lds, stream>>>(dPa, bm);
        k_commit_b<V><<<na, NTC, 0, stream>>>(dPa, bm);
        HIPCHK(hipGetLastError());
    }
    return TT_OK;
}

// Cores for the given slots, then their final device state to the host and
// one event that marks them complete.
int Engine::launch_cores(std::vector<int> &ids)
{
    for (size_t c0 = 0; c0 < ids.size(); c0 += MAXB) {
        const int na = (int)std::min<size_t>(MAXB, ids.size() - c0);
        BatchMap bm;
        int m = 0, off = 0, maxr = 1;
        for (int a = 0; a < na; ++a) {
            Slot &s = slots[ids[c0 + a]];
            const Problem &Q = *s.Q;
            int r[TT_MAX_D + 1];
            for (int k = 0; k <= Q.d; ++k) r[k] = hm[s.idx].r[k];
            r[0] = r[Q.d] = 1;
            for (int k = 1; k <= Q.d - 1; ++k) maxr = std::max(maxr, r[k]);
            CoreArgs ca;
            int64_t len;
            const int blocks = make_core_args(Q.d, Q.n, r, ca, len);
            bm.p[m] = (uint16_t)s.idx;
            bm.boff[m] = off;
            off += blocks;
            ++m;
        }
        bm.na = m;
        bm.boff[m] = off;
        const size_t lc = sizeof(double) * ((size_t)2 * maxr * (maxr + 1) + (size_t)2 * maxr * A4W);
        if (m > 0 && off > 0) k_cores_b<<<off, A4W, lc, stream>>>(dPa, bm);
        HIPCHK(hipGetLastError());
        // sampled-error checks of the slots that want one
        BatchMap bv;
        int nv = 0;
        for (int a = 0; a < na; ++a) {
            const Slot &s = slots[ids[c0 + a]];
            if (s.verify_R > 0) {
                bv.p[nv] = (uint16_t)s.idx;
                bv.boff[nv] = nv;
                ++nv;
            }
        }
        bv.na = nv;
        bv.boff[nv] = nv;
        if (nv > 0) {
            k_verify_b<<<dim3(NBV, nv), NT, 0, stream>>>(dPa, bv, dPart);   // partials land on the host
            HIPCHK(hipGetLastError());
        }
        // the finished states, to host memory
        BatchMap bo;
        bo.na = na;
        for (int a = 0; a < na; ++a) {
            bo.p[a] = (uint16_t)ids[c0 + a];
            bo.boff[a] = a;
        }
        bo.boff[na] = na;
        k_state_out_b<<<na, 64, 0, stream>>>(dS, dhS, bo);
        HIPCHK(hipGetLastError());
    }
    hipEvent_t ev = nullptr;
    if (!ev_free.empty()) { ev = ev_free.back(); ev_free.pop_back(); }
    else HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, stream));
    // the event is shared by the slots of this call; the last one to see it
    // complete returns it to the pool
    for (int i : ids) {
        slots[i].ev = ev;
        slots[i].phase = Slot::CORES;
    }
    ev_users.emplace_back(ev, (int)ids.size());
    return TT_OK;
}

int Engine::tick(std::vector<int> *completed)
{
    busy_tick = false;
    // 1. read the mirrors: progress and stop flags of sweeping slots
    std::vector<int> to_cores;
    bool any_sweeping = false;
    for (Slot &s : slots) {
        if (s.phase != Slot::SWEEP) continue;
        const HostMirror &h = hm[s.idx];
        const int sd = __atomic_load_n(&h.sweeps_done, __ATOMIC_ACQUIRE);
        if (sd > s.done) s.done = sd;
        if (__atomic_load_n(&h.stop, __ATOMIC_ACQUIRE)) s.stop_seen = true;
        const bool exhausted = s.launched >= s.Q->max_sweeps && s.done >= s.launched;
        if (s.stop_seen || exhausted || s.idle_done) {
            // without the stop flag's release the mirror's ranks are read only
            // after the stream has drained
            if (!s.stop_seen) HIPCHK(hipStreamSynchronize(stream));
            if (h.err) {
                s.Q->status = h.err;
                s.Q->ran = false;
                s.phase = Slot::FAILED;
                if (completed) completed->push_back(s.idx);
                continue;
            }
            to_cores.push_back(s.idx);
        } else {
            any_sweeping = true;
            // the next round's shapes have at most the committed ranks plus one
            // per queued round; its stored tiles, one round fewer
            for (int k = 1; k <= s.Q->d - 1; ++k) {
                const int rc = __atomic_load_n(&h.r[k], __ATOMIC_RELAXED), q = s.launched - s.done;
                s.rub[k] = std::min(s.Q->rc[k], rc + q);
                s.rst[k] = std::min(s.Q->rc[k], rc + std::max(0, q - 1));
            }
        }
    }
    if (!to_cores.empty()) {
        busy_tick = true;
        int st = launch_cores(to_cores);
        if (st) return st;
    }
    // 2. setup for new admissions
    std::vector<int> new32, new64;
    for (Slot &s : slots)
        if (s.phase == Slot::SETUP) {
            (s.Q->fp32 ? new32 : new64).push_back(s.idx);
            s.phase = Slot::SWEEP;
            any_sweeping = true;
        }
    if (!new32.empty()) { int st = launch_setup<float>(new32); if (st) return st; }
    if (!new64.empty()) { int st = launch_setup<double>(new64); if (st) return st; }
    // 3. queue sweep rounds up to the lookahead (and extra_ahead more)
    bool launched_any = false;
    for (;;) {
        std::vector<int> r32, r64;
        for (Slot &s : slots) {
            if (s.phase != Slot::SWEEP || s.stop_seen) continue;
            const int L = std::max(1, s.Q->opt.lookahead) + extra_ahead;
            if (s.launched < s.done + L && s.launched < s.Q->max_sweeps) (s.Q->fp32 ? r32 : r64).push_back(s.idx);
        }
        if (r32.empty() && r64.empty()) break;
        if (!r32.empty()) { int st = launch_sweep<float>(r32); if (st) return st; }
        if (!r64.empty()) { int st = launch_sweep<double>(r64); if (st) return st; }
        launched_any = true;
    }
    if (launched_any) busy_tick = true;
    // 4. completions (each cores launch's event queried once per tick)
    std::vector<std::pair<hipEvent_t, hipError_t>> evq;
    for (Slot &s : slots) {
        if (s.phase != Slot::CORES) continue;
        hipError_t q = hipErrorNotReady;
        bool known = false;
        for (const auto &e : evq)
            if (e.first == s.ev) { q = e.second; known = true; break; }
        if (!known) {
            q = hipEventQuery(s.ev);
            evq.emplace_back(s.ev, q);
        }
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return set_err(TT_EDEVICE, "batch: %s", hipGetErrorString(q));
        finish_slot(s);
        busy_tick = true;
        if (completed) completed->push_back(s.idx);
    }
    // 5. nothing queued that could still report progress: the stream is idle
    //    once every queued round has run, and the mirrors are final
    if (any_sweeping && !launched_any) {
        hipError_t q = hipStreamQuery(stream);
        if (q != hipErrorNotReady && q != hipSuccess) return set_err(TT_EDEVICE, "batch: %s", hipGetErrorString(q));
        if (q == hipSuccess) {
            for (Slot &s : slots) {
                if (s.phase != Slot::SWEEP) continue;
                const HostMirror &h = hm[s.idx];
                const int sd = __atomic_load_n(&h.sweeps_done, __ATOMIC_ACQUIRE);
                if (sd > s.done) s.done = sd;
                else if (s.done >= s.launched || s.launched >= s.Q->max_sweeps) s.idle_done = true;
            }
        }
    }
    return TT_OK;
}

void Engine::finish_slot(Slot &s)
{
    Problem &Q = *s.Q;
    const ProbState &S = hS[s.idx];
    int r[TT_MAX_D + 1];
    for (int k = 0; k <= Q.d; ++k) r[k] = hm[s.idx].r[k];
    r[0] = r[Q.d] = 1;
    if (S.err) {
        Q.status = S.err;
        Q.ran = false;
    } else {
        Q.finalize(S, r);
        if (s.verify_R > 0) {
            // the same in-order sum of the same partials as a single solve
            const double *hp = hPart + (size_t)2 * NBV * s.idx;
            double num = 0.0, den = 0.0;
            for (int b = 0; b < NBV; ++b) { num += hp[2 * b]; den += hp[2 * b + 1]; }
            const double err = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
            Q.sampled_err = err;
            if (err > Q.eps) {
                if (s.can_escalate) s.escalate = true;
                else if (Q.status == TT_OK) Q.status = TT_WARN_SAMPLED_ERR;
            }
        }
    }
    s.t_done = now_s();
    Q.time_to_eps = s.t_done - s.t_admit;
    Q.sweep_launches = 0;
    Q.sweep_kernel_s = Q.sweep_phase_s = 0;
    // return the event once no other slot still waits on it
    hipEvent_t ev = s.ev;
    s.ev = nullptr;
    for (size_t i = 0; i < ev_users.size(); ++i)
        if (ev_users[i].first == ev) {
            if (--ev_users[i].second == 0) {
                ev_free.push_back(ev);
                ev_users[i] = ev_users.back();
                ev_users.pop_back();
            }
            break;
        }
    s.phase = Slot::DONE;
}

void Engine::retire(int idx)
{
    if (idx < 0 || idx >= cap) return;
    Slot &s = slots[idx];
    if (s.phase == Slot::DONE || s.phase == Slot::FAILED) {
        s = Slot();
        s.idx = idx;
    }
}

bool Engine::idle() const
{
    for (const Slot &s : slots)
        if (s.phase == Slot::SETUP || s.phase == Slot::SWEEP || s.phase == Slot::CORES) return false;
    return true;
}

}  // namespace ttc

using namespace ttc;

extern "C" int tt_batch_run(tt_cross_h *hs, int count, void *hip_stream)
{
    if (count < 0 || (count > 0 && !hs)) return set_err(TT_EINVAL, "bad batch arguments");
    if (count == 0) return TT_OK;
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) return set_err(TT_EINVAL, "handle %d is NULL", i);
        if (hs[i]->p.opt.pivot_mode != TT_PIVOT_GREEDY)
            return set_err(TT_EINVAL, "handle %d: rook pivoting runs through tt_cross_run only", i);
        if (hs[i]->p.busy()) return set_err(TT_ESTATE, "handle %d has a run in flight", i);
    }
    {
        // distinct handles: sorted, no two neighbours equal
        std::vector<tt_cross_h> sorted(hs, hs + count);
        std::sort(sorted.begin(), sorted.end());
        for (int i = 1; i < count; ++i)
            if (sorted[i] == sorted[i - 1]) {
                int first = -1, second = -1;
                for (int j = 0; j < count && second < 0; ++j)
                    if (hs[j] == sorted[i]) (first < 0 ? first : second) = j;
                return set_err(TT_EINVAL, "handle %d appears twice", second);
            }
    }
    static const int zero = 0;
    for (int i = 0; i < count; ++i) {
        Problem &Q = hs[i]->p;
        const int st = Q.prepare();
        if (st) return st;
        // a batch runs every problem from its first pivot alone (restarts
        // after false convergence are tt_cross_run's)
        Q.h_plan.npts = 0;
        Q.restarts_used = 0;
        Q.restart_cause = 0;
        if (Q.dev_plan_npts != 0) {
            HIPCHK(hipMemcpyAsync(&Q.d_plan->npts, &zero, sizeof(int), hipMemcpyHostToDevice, Q.stream));
            Q.dev_plan_npts = 0;
        }
    }
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : hs[0]->p.stream;
    // the handles' own streams must not still be working on these buffers
    for (int i = 0; i < count; ++i) HIPCHK(hipStreamSynchronize(hs[i]->p.stream));
    // one engine per thread, kept for later batches (never torn down, so that
    // nothing is freed after the runtime has shut down at process exit)
    static thread_local Engine *engp = nullptr;
    if (!engp) engp = new Engine();
    Engine &eng = *engp;
    eng.extra_ahead = 1;
    if (eng.cap < count || eng.stream != stream) {
        const int st = eng.init(std::max(count, eng.cap), stream);
        if (st) return st;
    }
    struct EvPair {
        hipEvent_t a = nullptr, b = nullptr;
        ~EvPair()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    // after a failure with slots admitted: let the stream drain and reset the
    // engine, so that no slot stays taken for the thread's next batch
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(stream);
        (void)eng.init(eng.cap, stream);
        return code;
    };
    // pass 1: every problem; pass 2: those whose FP32 sweeps missed eps, in FP64
    std::vector<int> todo(count);
    for (int i = 0; i < count; ++i) todo[i] = i;
    double total = 0.0;
    int st = TT_OK;
    for (int pass = 0; pass < 2 && !todo.empty(); ++pass) {
        hipError_t he = hipEventRecord(ev.a, stream);
        if (he != hipSuccess) return fail(set_err(TT_EDEVICE, "batch: %s", hipGetErrorString(he)));
        std::vector<int> ids(todo.size());
        for (size_t i = 0; i < todo.size(); ++i) {
            const int id = eng.admit(&hs[todo[i]]->p, nullptr);
            if (id < 0) return fail(id);
            ids[i] = id;
        }
        while (!eng.idle()) {
            st = eng.tick(nullptr);
            if (st) return fail(st);
            if (!eng.busy_tick) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        he = hipEventRecord(ev.b, stream);
        if (he == hipSuccess) he = hipStreamSynchronize(stream);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, ev.a, ev.b);
        if (he != hipSuccess) return fail(set_err(TT_EDEVICE, "batch: %s", hipGetErrorString(he)));
        total += ms * 1e-3;
        std::vector<int> next;
        for (size_t i = 0; i < todo.size(); ++i) {
            if (eng.slot(ids[i]).escalate) next.push_back(todo[i]);
            eng.retire(ids[i]);
        }
        for (int i : next) {
            Problem &Q = hs[i]->p;
            Q.force_fp64 = true;
            const int ps = Q.prepare();
            if (ps) return ps;                  // every slot is retired here
        }
        todo.swap(next);
    }
    for (int i = 0; i < count; ++i) hs[i]->p.time_to_eps = total;
    return st;
}

extern "C" int tt_batch_statuses(tt_cross_h *hs, int count, int32_t *status)
{
    if (count < 0 || (count > 0 && (!hs || !status))) return set_err(TT_EINVAL, "bad arguments");
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) return set_err(TT_EINVAL, "handle %d is NULL", i);
        if (hs[i]->p.busy()) return set_err(TT_ESTATE, "handle %d has a run in flight", i);
        status[i] = hs[i]->p.status;
    }
    return TT_OK;
}
