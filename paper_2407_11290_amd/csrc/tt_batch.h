// tt_batch.h -- engine that keeps many independent solves resident on one GPU
// and advances all of them with shared launches (batched and served solves).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "tt_device.h"
#include "tt_internal.h"

namespace ttc {

struct Slot {
    enum Phase { FREE, SETUP, SWEEP, CORES, DONE, FAILED };
    int idx = 0;                  // entry in the engine's descriptor array
    Phase phase = FREE;
    Problem *Q = nullptr;
    void *user = nullptr;
    int launched = 0;             // sweep rounds queued for this slot
    int done = 0;                 // sweep rounds it has committed (host mirror)
    bool stop_seen = false;       // its stop flag reached the host
    bool idle_done = false;       // stream idle with nothing left to run for it
    int rub[TT_MAX_D + 1] = {0};  // rank bounds for the next round it gets
    int rst[TT_MAX_D + 1] = {0};  // bounds on the ranks its stored tiles were made with
    hipEvent_t ev = nullptr;      // completes when its cores and state are on the host
    double t_admit = 0, t_done = 0;
    int64_t verify_R = 0;         // samples of its sampled-error check (0: none)
    bool can_escalate = false;    // FP32 sweeps chosen by the precision policy
    bool escalate = false;        // finished above eps: the owner solves it again in FP64
};

class Engine {
public:
    int cap = 0;
    hipStream_t stream = nullptr;
    // sweep rounds queued beyond each problem's own lookahead: tt_batch_run
    // queues one more (its rounds cover many slots, and the host's pass over
    // their mirrors comes later after a round than a single solve's check;
    // surplus rounds find the stop flag set and return); the server none
    // (at a light load one more round only delays the next request's setup)
    int extra_ahead = 0;
    // whether the last tick launched work or finished a slot.  A caller that
    // finds it false waits a little before the next tick: back-to-back ticks
    // make runtime calls (event and stream queries) that compete with the
    // launches they are waiting for
    bool busy_tick = false;

    ~Engine();
    void release();
    int init(int capacity, hipStream_t s);
    // Takes a prepared problem into a free slot; returns the slot or an error.
    int admit(Problem *Q, void *user);
    // Reads progress, launches whatever can run, and appends the slots that
    // finished (cores on the host side, or failed) to *completed.
    int tick(std::vector<int> *completed);
    void retire(int idx);         // frees a finished slot
    bool idle() const;            // no slot is waiting for the device
    int free_slots() const;
    int busy() const;
    const Slot &slot(int i) const { return slots[i]; }

private:
    template <typename V> int launch_setup(std::vector<int> &ids);
    template <typename V> int launch_sweep(std::vector<int> &ids);
    int launch_cores(std::vector<int> &ids);
    void finish_slot(Slot &s);
    int copy_slots(void *dst, const void *src, size_t elem, const std::vector<int> &ids, hipMemcpyKind kind);

    std::vector<Slot> slots;
    std::vector<hipEvent_t> ev_free;
    // slots still holding each event of a cores launch (one event per launch,
    // shared by its slots; back to ev_free when the count reaches zero)
    std::vector<std::pair<hipEvent_t, int>> ev_users;
    ProbDev *dPa = nullptr, *hPa = nullptr;   // descriptors: device array, pinned staging
    std::vector<ProbDev> shadow;              // what dPa holds per slot (valid where shadow_ok)
    std::vector<char> shadow_ok;
    ProbState *dS = nullptr, *hS = nullptr;   // per-slot device state and its host copy (mapped)
    ProbState *dhS = nullptr;                 // device view of hS
    HostMirror *hm = nullptr, *dhm = nullptr; // mapped host mirrors (host / device view)
    double *dPart = nullptr, *hPart = nullptr;// sampled-error partial sums, 2 * NBV per slot (mapped
                                              // host memory; dPart is its device view)
};

}  // namespace ttc
