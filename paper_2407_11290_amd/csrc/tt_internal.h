// tt_internal.h -- host-side problem object behind the C ABI handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <vector>

#include "tt_cross.h"
#include "tt_device.h"

namespace ttc {

int set_err(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_err(TT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct FnHost {
    FnDev dev;
    std::vector<double> table;     // per-mode value table (host copy; see FnDev)
    std::vector<float> table32;    // its FP32 rounding, made at upload
    double *d_table = nullptr;     // device copies owned by the holder
    float *d_table32 = nullptr;
    size_t d_cap = 0;              // entries the device copies can hold
    void free_device();
};

int build_fn(int fn_id, int d, const int32_t *n, const double *params, int nparams, FnHost &out);
// Copies the table to the device (reusing the holder's buffers when it fits)
// and points dev.tab / dev.tab32 at it; with a stream the copies are queued on
// it, else they complete before the return.
int upload_fn(FnHost &fh, hipStream_t stream = nullptr);

struct Problem {
    // problem definition
    int d = 0;
    int n[TT_MAX_D] = {0};
    double eps = 0.0;
    FnHost fn;
    tt_options opt;
    // resolved geometry
    int rc[TT_MAX_D + 1] = {0};    // rank capacity per unfolding (rc[0] = rc[d] = 1)
    int grid[TT_MAX_D] = {0};      // subtensor blocks per mode
    int fp32 = 0;
    int tileTR[TT_MAX_D] = {0}, tileTC[TT_MAX_D] = {0};
    int req_tr = 0, req_tc = 0;    // tile request in force: the options', else the tuned table's
    bool use_table = true;         // false while the tuner times its own candidates
    int rook_g = 1;                // rook search: workgroups per subtensor block
    int kcap[TT_MAX_D + 1] = {0};  // prescribed rank per unfolding (0: none)
    int alloc_kcap[TT_MAX_D + 1] = {0};
    int hist_cap = 0, max_sweeps = 0;
    int lds_limit = 65536;         // LDS bytes one workgroup may allocate on this device
    int lds_static = 0;            // static LDS of the search kernel
    int sweep_grid_cap = 2048;     // workgroups of a search launch (8 per CU on 256 CUs)
    // device state
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool allocated = false;
    int alloc_fp32 = -1, alloc_rmax = -1, alloc_tr = -1, alloc_tc = -1, alloc_ns = -1, alloc_pivot = -1,
        alloc_split = -1;
    int alloc_grid[TT_MAX_D] = {0};
    std::vector<void *> allocs;
    ProbDev hP;
    ProbDev *dP = nullptr;
    HostMirror *hm = nullptr;
    double *d_cores = nullptr, *d_vals = nullptr;
    double *d_ctab = nullptr;          // the cores' pivot-row recursion, per unfolding
    SamplePart *d_spart = nullptr;
    // results
    bool ran = false;
    int status = TT_ESTATE;
    int ranks[TT_MAX_D + 1] = {0};
    int64_t cores_len = 0, evaluated = 0, pivoted = 0;
    int sweeps = 0;
    double rms = 0, tau = 0, time_to_eps = 0;
    double last_best[TT_MAX_D] = {0};
    int sweep_launches = 0;
    int rook_rounds = 0, rook_long = 0;      // rook walk statistics of the last run
    size_t stamp_words = 0;                  // phase stamps (library built with TT_STAMPS)
    double sweep_kernel_s = 0, sweep_alg_bytes = 0, new_entries = 0, sweep_phase_s = 0;
    std::vector<hipEvent_t> prof_events;     // 3 per sweep when profiling
    hipEvent_t run_ev[3] = {nullptr, nullptr, nullptr};  // start / end of a run's device time;
                                             // end of its last queued copy
    ProbState *hS_pinned = nullptr;          // pinned host copy of the final device state
    double *h_part = nullptr;                // pinned host copy of the check's partial sums
    int i0[TT_MAX_D] = {0};
    // sampled-error check and FP32 -> FP64 escalation
    double sampled_err = -1.0;
    int escalated = 0;
    bool force_fp64 = false;       // sweep in FP64 whatever the precision policy says
    double *d_part = nullptr;      // partial sums of the check (2 * NBV doubles)
    // restarts after false convergence (tt_options.restarts)
    SeedPlan h_plan;               // the point list of the current run and its index sets
    SeedPlan *d_plan = nullptr;    // its device copy (npts = 0: a plain run)
    int dev_plan_npts = 0;         // npts of the device copy
    PointCheck *d_pc = nullptr;    // candidates of a restart
    double *d_pres = nullptr;      // their residuals, TT_RESTART_TRIES x TT_MAX_D
    double *d_serr = nullptr;      // |X - X~| per check sample
    int64_t serr_cap = 0;
    int restarts_used = 0, restart_cause = 0;

    // a run in steps (tt_cross_run_async / tt_cross_query / tt_cross_wait)
    enum { PH_IDLE = 0, PH_SWEEPS, PH_TAIL, PH_VERIFY, PH_DONE };
    int phase = PH_IDLE;
    bool cur_fp32 = false;         // precision of the sweeps in flight
    int launched = 0, done_known = 0;                    // sweeps queued / reported done
    int rub[TT_MAX_D + 1] = {0}, rst[TT_MAX_D + 1] = {0}; // rank bounds of the next sweep / its stored region
    int ranks_now[TT_MAX_D + 1] = {0};                   // ranks of the final sweep
    double t_first = 0.0;          // device time of an FP32 run that was escalated
    bool busy() const { return phase == PH_SWEEPS || phase == PH_TAIL || phase == PH_VERIFY; }

    int64_t verify_samples() const;
    bool auto_fp32() const { return opt.precision == TT_PREC_AUTO && fp32 && !force_fp64; }
    bool restarts_on() const { return opt.restarts > 0 && opt.pivot_mode != TT_PIVOT_ROOK && !cur_fp32; }

    ~Problem();
    void release();
    int dalloc(void **p, size_t bytes);
    size_t device_bytes() const;
    void resolve_geometry();
    int allocate();
    int prepare();
    void finalize(const ProbState &S, const int *ranks_now);
    int start();
    int advance(bool wait);
    int run();
    template <typename V> int begin_sweeps();
    template <typename V> int launch_ahead();
    template <typename V> int poll_sweeps(bool wait);
    template <typename V> int launch_tail();
    int tail_event(bool wait);
    int poll_tail(bool wait);
    int poll_verify(bool wait);
    int plan_from_points();
    int point_levels(const int *pt) const;
    int restart_check(int nc, const int (*cand)[TT_MAX_D], const int *cin, double (*res)[TT_MAX_D]);
    int try_restart(bool &restarted);
};

// Process-wide table of tuned tile shapes by problem class (tt_tune.hip).
// Looked up when a problem's tile options are both 0.
bool tuned_tiles(const Problem &P, int &tr, int &tc);

}  // namespace ttc

// The object behind a tt_cross_h.
struct tt_cross_s {
    ttc::Problem p;
};
