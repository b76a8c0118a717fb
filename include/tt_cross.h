/*
 * tt_cross.h -- C ABI of the MI355X (gfx950) greedy adaptive TT-cross library.
 *
 * The library computes a tensor-train (TT) approximation of a tensor that is
 * known only through a generating function evaluated entry by entry, following
 * Shi, Hayes and Qiu, "Distributed memory parallel adaptive tensor-train cross
 * approximation":
 *   problem statement       -- Sec. 1, eq. (FrobeniusNorm): find X~ in TT format
 *                              with ||X - X~||_F <= eps ||X||_F;
 *   TT format               -- Sec. 2.2: X(i_1..i_d) = G_1(:,i_1,:) ... G_d(:,i_d,:);
 *   pivot search            -- Alg. 1 (greedy largest |residual|) run on the
 *                              superblocks of Alg. 2 for every unfolding at once;
 *   residual update         -- eq. (aca_approx_E) / (submatrix_cross_iter), in
 *                              residual form R <- R - R(:,j) R(i,:) / R(i,j);
 *   core construction       -- Alg. 4 with eq. (aca_approx_T) on the sliced
 *                              fibers, reshaped by eq. (corereshape);
 *   subtensor blocks        -- Sec. 3: every mode n_j is split evenly into C_j
 *                              pieces; each workgroup of the search works inside
 *                              one subtensor block and the global pivot is the
 *                              best of the block-local pivots (Sec. 3.2.1).
 * All of the blocks of all of the unfoldings run on one GPU.
 *
 * Conventions
 *   - Indices are 0-based at this interface.  The generating functions apply
 *     the paper's 1-based formulas internally.
 *   - A handle owns all device memory it uses.  Getters copy into caller-owned
 *     buffers; a NULL output pointer asks for the required size.
 *   - `on_device` = 0: pointers are host memory; = 1: they are device memory
 *     on the handle's GPU (for instance from a torch tensor), used on the
 *     handle's stream.
 *   - Negative return codes are errors, positive ones are warnings.  After an
 *     error tt_last_error() returns a message for the calling thread.
 *   - One thread may use a handle at a time.
 */
#ifndef TT_CROSS_H
#define TT_CROSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_D 16     /* largest supported number of modes */
#define TT_MAX_RANK 64  /* largest supported TT rank per unfolding */

/* Generating functions (fn_id) and their params[] layouts. */
enum tt_fn {
    /* Hilbert tensor, eq. (HilbertTensor): 1/(i_1+..+i_d + shift), 1-based i.
     * params: [] -> shift = 1-d (the paper's tensor), or [shift]. */
    TT_FN_HILBERT = 1,
    /* Single 3d3v Maxwellian, d = 6, modes x1,x2,x3,v1,v2,v3:
     * rho(x) (2 pi T)^{-3/2} exp(-|v-u(x)|^2/(2T)), rho = 1 + a sin(2pi x1)cos(2pi x2),
     * u = (b sin(2pi x3),0,0), x_l = i/n on [0,1), v cell-centred on [-vmax,vmax].
     * params: [] -> (a,b,T,vmax) = (0.5,0.3,1,8), or [a,b,T,vmax]. */
    TT_FN_MAXWELL = 2,
    /* Sum of two spatially uniform 3v Maxwellians, d >= 3; the d-3 leading modes
     * are spatial (f does not depend on them), the last three are v1,v2,v3.
     * params: [rho1,u1x,u1y,u1z,T1, rho2,u2x,u2y,u2z,T2 (, vmax=8)]. */
    TT_FN_BIMAXWELL = 3,
    /* Sum of r separable products, f = sum_m prod_j g_{m,j}(i_j).
     * params: [r, g...], g_{m,j}(i) at 1 + m*sum(n) + n_0+..+n_{j-1} + i. */
    TT_FN_SEPSUM = 4,
    /* The paper's kinetic tensors of Sec. 5.2, eq. (2d2vFunction): modes
     * x,v_x,y,v_y (d = 4) or x,v_x,y,v_y,z,v_z (d = 6); x in [-1/2,1/2],
     * v in [-3,3], cell-centred grids.  params: []. */
    TT_FN_MAXWELL_2D2V = 5,
    TT_FN_MAXWELL_3D3V = 6,
    /* TT_FN_MAXWELL with its modes in the order x1,v1,x2,v2,x3,v3 (the
     * position-velocity interleaving of the paper's kinetic tensors): mode
     * 2w holds x_{w+1}, mode 2w+1 holds v_{w+1}.  The greedy cross started
     * from one pivot stops at rank 1 on it with a large sampled error (see
     * tt_options.restarts).  params: as TT_FN_MAXWELL. */
    TT_FN_MAXWELL_IL = 7
};

enum tt_status {
    TT_OK = 0,
    TT_NOT_CONVERGED = 1,     /* some unfolding hit r_max with |residual| > tau */
    TT_WARN_SAMPLED_ERR = 2,  /* sampled error above eps (tt_cross_sampled_error) */
    TT_EINVAL = -1,           /* bad argument */
    TT_ENOMEM = -2,           /* device or host allocation failed, or over budget */
    TT_EDEVICE = -3,          /* HIP runtime error */
    TT_ESINGULAR = -4,        /* zero pivot */
    TT_ESTATE = -5,           /* call not valid in the handle's state */
    TT_EFN = -6,              /* unknown generating function or bad params */
    TT_EBUSY = -7             /* server queue full */
};

enum tt_precision {
    TT_PREC_AUTO = 0,  /* FP32 entry evaluation and sweeps iff eps >= 1e-6, else FP64 */
    TT_PREC_FP64 = 1,  /* FP64 everywhere (bit-exact with a canonical FP64 reference) */
    TT_PREC_FP32 = 2   /* FP32 evaluation and sweeps; pivot check, stop test and cores in FP64 */
};

enum tt_pivot_mode {
    TT_PIVOT_GREEDY = 0, /* largest |residual| over the whole superblock (stored residuals) */
    TT_PIVOT_ROOK = 1    /* Alg. 1 inside every subtensor block, best of the local pivots
                            (Alg. 3), on residual factors instead of stored residuals;
                            FP64 sweeps; single solves only (tt_cross_run) */
};

typedef struct tt_options {
    uint64_t seed;              /* seeds the N_s sample entries (default 0) */
    int32_t r_max;              /* rank cap per unfolding, 1..TT_MAX_RANK (default 64) */
    int32_t precision;          /* enum tt_precision (default TT_PREC_AUTO) */
    int32_t pivot_mode;         /* enum tt_pivot_mode (default greedy) */
    int32_t n_samples;          /* N_s sample entries for rms and the first pivot (default 16384) */
    int32_t grid[TT_MAX_D];     /* subtensor blocks per mode C_j (default 1; 1 <= C_j <= n_j) */
    int32_t tile_rows;          /* rows per workgroup tile, 1..256; 0 (with tile_cols 0) = the
                                   tuned shape of the problem's class (tt_autotune), else the
                                   library's default */
    int32_t tile_cols;          /* columns per workgroup tile, 1..64 (rounded up to a power of
                                   two); 0 as for tile_rows */
    int32_t lookahead;          /* sweeps queued ahead of the host's stop check (default 2;
                                   tt_batch_run queues one round more) */
    int32_t profile;            /* 1: time every search launch with HIP events (stats below) */
    void *stream;               /* hipStream_t to run on; NULL = a stream owned by the handle */
    int32_t verify;             /* sampled-error check after the run (Sec. 5), on an independent
                                   SplitMix64(seed + 1) set: -1 (default) = 4096 samples when the
                                   precision policy chose FP32 sweeps, none otherwise; 0 = never;
                                   > 0 = always, with that many samples.  When the error exceeds
                                   eps after FP32 sweeps chosen by TT_PREC_AUTO, the problem is
                                   solved again with FP64 sweeps; if it still exceeds eps the
                                   status is TT_WARN_SAMPLED_ERR. */
    int32_t rook_split;         /* rook pivoting: workgroups per subtensor block in the search;
                                   0 (default) = chosen by the library from the block sizes,
                                   1 = one workgroup per block, 2..1024 = that many (results
                                   do not depend on it) */
    int32_t restarts;           /* restarts after false convergence, 0..8 (default 0 = none);
                                   greedy FP64 sweeps only (not in the paper, whose guards are
                                   the random start of Alg. 1 and the sampled error of Sec. 5).
                                   When the sampled-error check (verify; 4096 samples if verify
                                   is -1, which restarts need, not 0) exceeds eps after a run
                                   that stopped below tau, the run is repeated from more initial
                                   pivots.  The initial index sets come from a point list, i0
                                   first: a point enters the unfoldings where neither its prefix
                                   (i_1..i_k) nor its suffix (i_{k+1}..i_d) is present yet (one
                                   run of unfoldings, so the sets stay nested and every cross
                                   square), as their next pivot.  The check's samples are tried
                                   by decreasing |X - X~| (lowest sample first on ties, the 64
                                   worst at most): a sample whose residual exceeds tau in every
                                   unfolding it enters joins the list; one that fails is
                                   trimmed to its longest run of unfoldings that pass (the
                                   first on ties), with i0's indices outside it, and tested
                                   again.  With no point found, or the restarts used up, the
                                   status is TT_WARN_SAMPLED_ERR (tt_stats.restart_cause).  The
                                   first sweep of a restarted run evaluates every tile anew. */
} tt_options;

typedef struct tt_stats {
    int64_t evaluated;          /* entries of the final superblocks, summed over unfoldings: the
                                   distinct entries the greedy search evaluates; with rook
                                   pivoting the same measure (the search evaluates only the
                                   entries it looks at, counted in pivoted) */
    int64_t pivoted;            /* residual entries scanned by argmax passes, all sweeps */
    int64_t samples;            /* sample entries evaluated for rms and the first pivot */
    int32_t sweeps;             /* search sweeps run (the last one proposes nothing) */
    int32_t precision_used;     /* TT_PREC_FP64 or TT_PREC_FP32 */
    int32_t status;             /* last tt_cross_run status */
    int32_t d;
    int32_t ranks[TT_MAX_D + 1];
    double rms;                 /* rms of the sample entries */
    double tau;                 /* stop threshold eps * rms */
    double time_to_eps_s;       /* device time of the last tt_cross_run */
    double last_best[TT_MAX_D]; /* largest unmasked |residual| per unfolding in the final sweep */
    /* filled when options.profile = 1 (device times from HIP events on the run's stream) */
    int32_t sweep_launches;     /* search-tile launches that did work (one per sweep); rook
                                   pivoting: sweeps, each timed over its search launches */
    int32_t rook_max_rounds;    /* rook pivoting: most rounds of Alg. 1's loop (a column step and
                                   a row step) that any block search of the run took; the loop
                                   runs until neither step moves.  0 for greedy search */
    double sweep_kernel_s;      /* summed duration of those launches */
    double sweep_alg_bytes;     /* algorithmic residual traffic of the tile launches: 2w per
                                   updated stored entry, w per scanned-only stored entry,
                                   w per newly evaluated entry (w = 8 FP64, 4 FP32); rook
                                   pivoting: 8 r_k per residual the search looked at (one
                                   factor vector streamed) */
    double new_entries;         /* superblock entries evaluated by the tile launches */
    double sweep_phase_s;       /* device time from the first search launch to the end of the last one */
    double sampled_err;         /* the verify check's sampled relative error, -1 if not run */
    int32_t escalated;          /* 1: the FP32 solve missed eps and was redone in FP64 */
    int32_t rook_long_walks;    /* rook pivoting: block searches whose walk took more than 8
                                   rounds (with several workgroups per block these finish in
                                   the search's last launch, one workgroup per block) */
    int32_t restarts_used;      /* restarts after false convergence (tt_options.restarts) */
    int32_t restart_cause;      /* why restarts stopped with the error above eps: 0 none, 1 the
                                   restarts were used up, 2 no check sample gave a point */
} tt_stats;

typedef struct tt_cross_s *tt_cross_h;

/* Fill *opt with the defaults listed in tt_options. */
void tt_options_default(tt_options *opt);

/* Create a problem: d modes of sizes n[0..d-1] (each in [1, 2^20]), tolerance eps >= 0
 * (eq. FrobeniusNorm), generating function fn_id with nparams doubles of
 * params (may be NULL when nparams == 0).  params are copied.  Returns NULL on
 * bad arguments (reason in tt_last_error). */
tt_cross_h tt_cross_create(int d, const int32_t *n, double eps, int fn_id, const double *params,
                           int nparams);

/* Replace the options (before tt_cross_run; a later run reuses them). */
int tt_cross_set_options(tt_cross_h h, const tt_options *opt);

/* Prescribed ranks (the paper's experiments run at fixed core ranks, Sec. 5):
 * unfolding k stops growing at min(r_max, caps[k-1]) pivots; caps holds d-1
 * values, 0 meaning r_max alone (caps NULL: all 0).  Together with eps = 0 a
 * run adds pivots until every unfolding has its prescribed rank (status
 * TT_NOT_CONVERGED, the rank cap being what stopped it) or its residual on
 * the superblock is exactly zero.  Takes effect at the next run; kept until
 * changed.  Errors: TT_EINVAL (NULL handle, a cap outside [0, TT_MAX_RANK]). */
int tt_cross_set_rank_caps(tt_cross_h h, const int32_t *caps);

/* Run the approximation to completion on the handle's stream and wait for it.
 * Returns TT_OK, TT_NOT_CONVERGED, TT_WARN_SAMPLED_ERR (after a sampled-error
 * check, see tt_options.verify), or an error code.  The same as
 * tt_cross_run_async followed by tt_cross_wait. */
int tt_cross_run(tt_cross_h h);

/* The same run as tt_cross_run (the problem of Sec. 1), started without
 * waiting: the call queues the samples, the setup and the first sweeps on
 * hip_stream and returns.  The rest of the run (further sweeps, queued as
 * the device reports its progress through mapped host memory; the cores;
 * the sampled-error check and an FP64 escalation when the precision policy
 * asks for them) is queued by later tt_cross_query / tt_cross_wait calls on
 * the same handle, so a caller that polls keeps the device busy while its
 * host thread does other work.  hip_stream: a hipStream_t, which the handle
 * then keeps for its later calls (as tt_options.stream); NULL = the handle's
 * stream.  While the run is in flight every other call on the handle
 * returns TT_ESTATE, except tt_cross_query, tt_cross_wait and
 * tt_cross_destroy (which finishes the run first).  Results are bit for bit
 * those of tt_cross_run.  Returns TT_OK when the run is started, else an
 * error code (the run is then over). */
int tt_cross_run_async(tt_cross_h h, void *hip_stream);

/* Advances a run started by tt_cross_run_async as far as the device allows,
 * without blocking.  Returns 0 while the run is in flight, 1 when no run is
 * in flight (the last one has finished: its status comes from tt_cross_wait
 * or tt_cross_get_stats), or a negative error code when a step failed (the
 * run is then over with that status). */
int tt_cross_query(tt_cross_h h);

/* Blocks until the run in flight has finished and returns its status, as
 * tt_cross_run would (at once for a finished run).  Errors: TT_ESTATE when no
 * run was ever started on the handle. */
int tt_cross_wait(tt_cross_h h);

/* ranks[0..d] = (1, r_1, .., r_{d-1}, 1) after a run. */
int tt_cross_get_ranks(tt_cross_h h, int32_t *ranks);

/* Tile shapes of the last run's search launches, one per unfolding:
 * rows[k-1] x cols[k-1] for k = 1..d-1 (see tt_autotune below). */
int tt_cross_get_tiles(tt_cross_h h, int32_t *rows, int32_t *cols);

/* Copy the cores G_1..G_d, concatenated, each r_{k-1} x n_k x r_k in row-major
 * order, into out (cap doubles).  Returns the number of doubles needed; with
 * out == NULL only the size is returned. */
int64_t tt_cross_get_cores(tt_cross_h h, double *out, int64_t cap, int on_device);

/* Evaluate the TT at m multi-indices idx (m x d, 0-based, row-major) into
 * out[m]; each matrix product is accumulated in ascending index order. */
int tt_eval(tt_cross_h h, int64_t m, const int32_t *idx, double *out, int on_device);

/* Pivots of unfolding k (1 <= k <= d-1) in insertion order: rows (r_k x k)
 * hold the index tuples of I_{<=k}, cols (r_k x (d-k)) those of J_{>k}; either
 * may be NULL.  Returns r_k. */
int tt_cross_get_pivots(tt_cross_h h, int k, int32_t *rows, int32_t *cols);

/* Per-sweep history of the largest unmasked |residual| of unfolding k (1-based):
 * copies up to cap values, returns the number of sweeps. */
int tt_cross_get_history(tt_cross_h h, int k, double *out, int cap);

int tt_cross_get_stats(tt_cross_h h, tt_stats *st);

/* Phase stamps of the last run, for the instrumented build of the library
 * (libttcross_stamps.so, compiled with TT_STAMPS; the normal build returns
 * TT_ESTATE).  The device's 100 MHz clock at phase boundaries: layout[0]
 * words per record, layout[1] records per sweep (search workgroups, by
 * workgroup index), layout[2] sweeps with records, layout[3] sweeps run; the
 * search records of all sweeps come first, then one record per commit.
 * Search record: 0 entry, 1 state loaded, 2-6 the first new-entry tile
 * (start, staging, raw factors, factor solves, entries done), 7-8 wavefront
 * 0's first stored tile (geometry known, done), 9 end, 10 new tiles, 11
 * stored tiles of wavefront 0, 12 the first new-entry tile's entries
 * computed (before its reduction), 13 that tile's kind (1 + 1 if its rows
 * were stored + 2 if its columns were).  Commit record: 0 entry, 1 state
 * (and first candidates) loaded, 2 wavefront 0's candidates reduced, 3
 * pivots committed, 4 end.  Zero = not reached.
 * Returns the number of values (out NULL: the size). */
int64_t tt_cross_get_stamps(tt_cross_h h, uint64_t *out, int64_t cap, int32_t *layout);

/* Sampled relative error (Sec. 5): sqrt(sum (X - X~)^2 / sum X^2) over R
 * multi-indices drawn from SplitMix64(seed), coordinate j of sample s being
 * draw(s*d + j) mod n_j. */
int tt_cross_sampled_error(tt_cross_h h, int64_t R, uint64_t seed, double *err);

/* The sampled relative error of tt_cross_sampled_error, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result, bit for bit, but the indices, values and partial sums live in one
 * static device array of the library (about 5 MiB per GPU that calls it,
 * held until the process ends) instead of buffers allocated per call.
 * R must be in [1, TT_NOALLOC_MAX_SAMPLES] (else TT_EINVAL).  Calls that
 * overlap on one GPU (several host threads, or a caller's own graph
 * replays) share the array and race; run them one at a time.  Runs on the
 * handle's stream and returns when done; nothing is allocated on the device
 * or pinned on the host.  Returns as tt_cross_sampled_error. */
#define TT_NOALLOC_MAX_SAMPLES 65536
int tt_cross_sampled_error_noalloc(tt_cross_h h, int64_t R, uint64_t seed, double *err);

/* Evaluate a generating function (the tensor's entries, Sec. 1: element
 * access only) at m multi-indices, no handle needed.  tt_fn_eval computes in
 * FP64; tt_fn_eval_f32 uses the FP32 arithmetic that FP32 sweeps use for
 * superblock entries.  idx: m x d int32, row-major, 0-based; out: m values.
 * on_device = 0: host buffers, every index checked (TT_EINVAL if outside
 * [0, n_j)); = 1: device buffers, indices not checked and must lie in range.
 * Runs on the null stream and returns when done.  The Maxwellians' per-mode
 * value tables (built on the host, copied to the device) of the last four
 * functions evaluated stay on the device for later calls; concurrent calls
 * run one after the other.
 * Errors: TT_EFN (unknown function or bad params), TT_EINVAL, TT_EDEVICE. */
int tt_fn_eval(int fn_id, int d, const int32_t *n, const double *params, int nparams, int64_t m,
               const int32_t *idx, double *out, int on_device);
int tt_fn_eval_f32(int fn_id, int d, const int32_t *n, const double *params, int nparams, int64_t m,
                   const int32_t *idx, float *out, int on_device);

/* Device time in milliseconds of the kernel of the last bulk evaluation
 * (tt_fn_eval or tt_fn_eval_f32) that completed in this process, from events
 * attached to its dispatch: host work before the launch is not included.
 * Errors: TT_EINVAL (ms NULL), TT_ESTATE (no evaluation has completed). */
int tt_fn_eval_last_kernel_ms(double *ms);

void tt_cross_destroy(tt_cross_h h);

/* Solve count independent problems together on one GPU.
 *
 * Every handle is solved exactly as tt_cross_run would solve it (same
 * samples, pivots, ranks and cores, bit for bit), but all of them are
 * resident at once.  Each launch covers every problem at the same phase:
 *   - setup covers all problems;
 *   - each search launch covers all problems still sweeping, every one over
 *     its own superblocks and subtensor blocks (Alg. 2, Sec. 3);
 *   - each commit launch covers the same problems.
 * A problem that stops leaves the rounds, and its cores (Alg. 4) are built
 * with those of the others that stopped at the same time.
 *
 * hip_stream: the stream all launches go to (NULL: the first handle's).
 * The handles keep their buffers; results are read with the usual getters,
 * and time_to_eps in the stats is the whole batch's.  Handles must be
 * distinct.  Returns TT_OK when every launch succeeded; each problem's own
 * status (TT_OK, TT_NOT_CONVERGED, or a device-reported error) is in its
 * stats.  Errors: TT_EINVAL (bad arguments), TT_EDEVICE, TT_ENOMEM. */
int tt_batch_run(tt_cross_h *hs, int count, void *hip_stream);

/* Each problem's own status after its last run (tt_batch_run or
 * tt_cross_run), all in one call: status[i] receives handle i's, the same
 * value tt_cross_get_stats reports in tt_stats.status.  hs: count handles
 * (host array); status: count int32 (host array, caller-owned).  Reads host
 * state only (no device work, no synchronisation).  Errors: TT_EINVAL (NULL
 * arrays or a NULL handle, count < 0), TT_ESTATE (a handle with a run in
 * flight); entries before the failing handle are filled. */
int tt_batch_statuses(tt_cross_h *hs, int count, int32_t *status);

/* ---------------------------------------------------------------------------
 * Tile-shape autotuning (batching: tiles chosen by measurement).
 *
 * A search tile covers tile_rows superblock rows by tile_cols columns inside
 * one subtensor block (Sec. 3) and one prefix (suffix) of the nested index
 * sets.  The result of a solve does not depend on the tile shape -- entries
 * are computed one by one in a fixed order, and the tiles' local pivots are
 * combined with the lowest-(row, column) tie-break (Alg. 3) -- only its time
 * does.  The library keeps one process-wide table of tuned shapes by problem
 * class: mode sizes, subtensor grid, sweep precision, rank cap, and whether
 * the tensor is the Hilbert tensor (which has kernels of its own).  A handle
 * whose tile_rows and tile_cols are both 0 uses its class's entry, if any,
 * when it is next prepared; otherwise the library's default shape.
 *
 * Candidates: the default shape, then every power-of-two tile_rows in
 * [8, 256] and tile_cols in [8, 64] up to the longest run of a mode inside
 * one subtensor block; shapes that do not fit in LDS at the rank cap are
 * skipped.  A candidate replaces the default only if it is at least 2%
 * (batches: 5%) faster.  The tuners allocate (each shape has its own tile tables) and
 * leave the handles' options, precision state and results as a solve with
 * the last candidate left them.
 * ------------------------------------------------------------------------- */

/* Times complete solves of h (reps timed runs after one untimed run, median
 * of the device time-to-eps) under every candidate shape and records the
 * fastest for h's class.  Outputs (each may be NULL): the recorded shape,
 * 0/0 meaning the default, and its median time in ms.
 * Errors: TT_EINVAL (NULL handle, reps outside [1,64]), or a solve's error. */
int tt_autotune(tt_cross_h h, int reps, int32_t *tile_rows, int32_t *tile_cols, double *best_ms);

/* The same for batched solves: the handles are grouped by class, and for
 * every class up to per_class of its handles are solved together with
 * tt_batch_run (on hip_stream, as there) under every candidate shape; the
 * median device time of reps timed batches decides.  Returns the number
 * of classes tuned, or an error as tt_batch_run. */
int tt_batch_autotune(tt_cross_h *hs, int count, int reps, int per_class, void *hip_stream);

/* Copies the tuned-shape table: row i of out (TT_TILE_ROW_WORDS int32 each)
 * is d, fp32 sweeps (0/1), Hilbert kernels (0/1), r_max, n[TT_MAX_D],
 * grid[TT_MAX_D] (zero past d), tile_rows, tile_cols.  At most cap rows are
 * written; returns the number of entries (out NULL: only the count). */
#define TT_TILE_ROW_WORDS (6 + 2 * TT_MAX_D)
int tt_tile_table(int32_t *out, int cap);

/* Empties the tuned-shape table. */
void tt_tile_table_clear(void);

/* ---------------------------------------------------------------------------
 * Served solves: continuous batching on one GPU.
 *
 * A server owns a stream, a batch engine (as in tt_batch_run) and a pool of
 * problem objects with their device buffers.  Requests are submitted at any
 * time from any thread.  A server thread admits them in arrival order when an
 * engine slot is free and a problem object of the request's shape (modes,
 * subtensor grid, sweep precision, rank cap) is idle or fits within
 * hbm_budget bytes.  To make room it evicts idle objects of other shapes.
 * Admitted requests join the search rounds of those already running.  Each
 * request is solved exactly as tt_cross_run would solve it with the server's
 * options and the request's seed.  When it ends, its stats and cores are
 * copied to the request and its problem object returns to the pool.
 * ------------------------------------------------------------------------- */
typedef struct tt_server_s *tt_server_h;

typedef struct {
    int64_t submitted, completed, queued, running;
    int64_t pool_bytes;     /* device bytes held by pooled problem objects */
    int64_t pool_objects;
    int64_t allocations;    /* problem objects created so far */
} tt_server_stats;

/* opt: options applied to every request (r_max, grid, precision, n_samples,
 * lookahead; seed and stream are ignored).  NULL gives the defaults with
 * r_max = 32 and two subtensor blocks per mode.  max_slots bounds the solves
 * in flight.  Returns NULL on bad arguments or when no GPU can be used. */
tt_server_h tt_server_create(size_t hbm_budget, int max_slots, const tt_options *opt);

/* Queue one request (arguments as in tt_cross_create, plus its sample seed).
 * Separable sums (TT_FN_SEPSUM, whose factor tables come from the caller) are
 * not served.  Returns
 * TT_OK and the ticket, or an error for a request that can never run. */
int tt_server_submit(tt_server_h s, int d, const int32_t *n, double eps, int fn_id, const double *params,
                     int nparams, uint64_t seed, uint64_t *ticket);

/* 1 when the request has finished, 0 while queued or running, < 0 on error. */
int tt_server_poll(tt_server_h s, uint64_t ticket);

/* Block until the request finishes.  latency_s (may be NULL) receives
 * completion minus submission time, queueing included.  Returns the request's
 * status (TT_OK, TT_NOT_CONVERGED, or an error such as TT_ENOMEM when it needs
 * more than the whole budget). */
int tt_server_wait(tt_server_h s, uint64_t ticket, double *latency_s);

/* Stats and cores (layout as tt_cross_get_cores) of a finished request;
 * either pointer may be NULL.  Returns the number of doubles of the cores. */
int64_t tt_server_result(tt_server_h s, uint64_t ticket, tt_stats *st, double *cores, int64_t cap);

/* Forget a finished request. */
int tt_server_release(tt_server_h s, uint64_t ticket);

int tt_server_get_stats(tt_server_h s, tt_server_stats *st);

/* Stops the server thread after the solves in flight and frees everything. */
void tt_server_destroy(tt_server_h s);

/* Message for the last error on the calling thread (empty if none). */
const char *tt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TT_CROSS_H */
