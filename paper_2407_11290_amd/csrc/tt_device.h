// tt_device.h -- device-side data layout and generating functions of the
// gfx950 greedy adaptive TT-cross library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tt_cross.h"

namespace ttc {

constexpr int NT = 256;                    // threads per workgroup (4 wave64)
constexpr int TT_TILE_ROWS_MAX = 256;      // largest tile extent along the rows
constexpr double PI = 3.14159265358979323846;
constexpr uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ULL;
constexpr int TT_ROOK_ITERS = 8;           // rounds of Alg. 1's loop in the split search's fixed
                                           // launch sequence; longer walks finish in its last launch

// ---------------------------------------------------------------------------
// Generating function descriptor (copied to the device with the problem).
// ---------------------------------------------------------------------------
// Table-driven functions keep per-mode values in one device table of rows of
// tab_ld entries: row t holds, for every mode j, the values of indices
// 0..n_j-1 from column off[j] on.  The separable sum stores its factor
// vectors there (row m = term m).  The Maxwellians store their per-mode
// factors there ("atoms": the sines, cosines and velocities that depend on one
// index alone), computed once on the host in FP64 by the same operations the
// formulas prescribe; an entry then combines table values and needs no
// trigonometric call.  tab32 holds the same table rounded to FP32.
struct FnDev {
    int id, d;
    int n[TT_MAX_D];
    double prm[12];
    int nprm;
    double shift;               // Hilbert denominator shift
    double cst[2];              // Maxwellians: per-Maxwellian constant factors
    const double *tab;          // per-mode value table (device), else null
    const float *tab32;         // the same table in FP32 (device), else null
    int sep_r, tab_ld;          // separable-sum terms; entries per table row
    int tab_rows;               // rows of the table (0: no table)
    int off[TT_MAX_D];          // first column of mode j in a table row
};

// SplitMix64 (Steele, Lea, Flood 2014) is counter based: draw t of the stream
// seeded with s is the finaliser applied to s + (t+1) * gamma.
__host__ __device__ inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t sm64_at(uint64_t seed, uint64_t t)
{
    return sm64_mix(seed + (t + 1) * SM64_GAMMA);
}

template <typename V> struct M;
template <> struct M<double> {
    __device__ static double sin(double x) { return ::sin(x); }
    __device__ static double cos(double x) { return ::cos(x); }
    __device__ static double exp(double x) { return ::exp(x); }
    __device__ static double pow(double x, double y) { return ::pow(x, y); }
    __device__ static double sqrt(double x) { return ::sqrt(x); }
};
template <> struct M<float> {
    __device__ static float sin(float x) { return ::sinf(x); }
    __device__ static float cos(float x) { return ::cosf(x); }
    __device__ static float exp(float x) { return ::expf(x); }
    __device__ static float pow(float x, float y) { return ::powf(x, y); }
    __device__ static float sqrt(float x) { return ::sqrtf(x); }
};

template <typename V> __host__ __device__ inline V cell(int i, int n, V lo, V hi)
{
    return lo + ((V)i + (V)0.5) * ((hi - lo) / (V)n);
}

// Velocity grid: cell centres of [-vmax, vmax] in n cells.
template <typename V> __host__ __device__ inline V vel(int i, int n, V vmax)
{
    return -vmax + ((V)i + (V)0.5) * ((V)2 * vmax / (V)n);
}

// Buffers reached through a descriptor are generic pointers to the compiler;
// naming their address space lets it emit global instead of flat loads and
// stores, which wait on the vector-memory counter alone.
template <typename T> using gptr_t = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline gptr_t<T> as_global(T *p) { return (gptr_t<T>)p; }

// Rook factors: a row of W and a column of U are contiguous vectors whose
// starts lie 64 bytes apart at least, the rank cap rounded up to 8 values, so
// a residual reads each vector as whole aligned 64-byte chunks.
__host__ __device__ inline int factor_pitch(int rank_cap) { return (rank_cap + 7) & ~7; }

// The per-mode table in the arithmetic's precision.
template <typename V> __host__ __device__ inline const V *fn_table(const FnDev &F);
template <> __host__ __device__ inline const double *fn_table<double>(const FnDev &F) { return F.tab; }
template <> __host__ __device__ inline const float *fn_table<float>(const FnDev &F) { return F.tab32; }

// Value of the generating function at a full 0-based multi-index, read
// through ix(j) (an accessor, so callers can assemble the index from LDS-staged
// prefixes and suffixes without a private array).  The operation order follows
// the written formulas term by term, so that FP64 values of the Hilbert and
// separable functions are bitwise reproducible; the Maxwellians' per-index
// factors come from the host-built table, and only their exponentials are
// evaluated here.
// FNS = 0 reads the function from F.id; a nonzero FNS fixes it at compile
// time, so a kernel built for one function carries no code of the others.
// fn_value_tx reads the per-mode table through tb (a copy of it in LDS, or the
// table itself); fn_value_ix reads the table in device memory.
template <typename V, int FNS = 0, typename IX, typename TP>
__device__ inline V fn_value_tx(const FnDev &F, IX ix, TP tb)
{
    // value t of index i of mode j
    auto atom = [&](int t, int j, int i) -> V { return tb[(int64_t)t * F.tab_ld + F.off[j] + i]; };
    switch (FNS ? FNS : F.id) {
    case TT_FN_HILBERT: {
        long long s = 0;
        for (int j = 0; j < F.d; ++j) s += (long long)ix(j) + 1;
        return (V)1 / ((V)s + (V)F.shift);
    }
    case TT_FN_MAXWELL: {
        // table row 0: sin(2 pi x1), cos(2 pi x2), sin(2 pi x3), v1, v2, v3
        const V a = (V)F.prm[0], b = (V)F.prm[1], T = (V)F.prm[2];
        const V s1 = atom(0, 0, ix(0)), c2 = atom(0, 1, ix(1)), s3 = atom(0, 2, ix(2));
        const V v1 = atom(0, 3, ix(3)), v2 = atom(0, 4, ix(4)), v3 = atom(0, 5, ix(5));
        V rho = (V)1 + a * s1 * c2;
        V ux = b * s3;
        V q = (v1 - ux) * (v1 - ux) + v2 * v2 + v3 * v3;
        return rho * (V)F.cst[0] * M<V>::exp(-q / ((V)2 * T));
    }
    case TT_FN_MAXWELL_IL: {
        // modes x1, v1, x2, v2, x3, v3; the same atoms and formula
        const V a = (V)F.prm[0], b = (V)F.prm[1], T = (V)F.prm[2];
        const V s1 = atom(0, 0, ix(0)), c2 = atom(0, 2, ix(2)), s3 = atom(0, 4, ix(4));
        const V v1 = atom(0, 1, ix(1)), v2 = atom(0, 3, ix(3)), v3 = atom(0, 5, ix(5));
        V rho = (V)1 + a * s1 * c2;
        V ux = b * s3;
        V q = (v1 - ux) * (v1 - ux) + v2 * v2 + v3 * v3;
        return rho * (V)F.cst[0] * M<V>::exp(-q / ((V)2 * T));
    }
    case TT_FN_BIMAXWELL: {
        // table row m: (v_c - u_{m,c})^2 on the velocity modes; cst[m] = rho_m (2 pi T_m)^{-3/2}
        const int d = F.d;
        V f = 0;
        for (int m = 0; m < 2; ++m) {
            const V T = (V)F.prm[5 * m + 4];
            V q = 0;
            for (int c = 0; c < 3; ++c) q += atom(m, d - 3 + c, ix(d - 3 + c));
            f += (V)F.cst[m] * M<V>::exp(-q / ((V)2 * T));
        }
        return f;
    }
    case TT_FN_SEPSUM: {
        V f = 0;
        for (int m = 0; m < F.sep_r; ++m) {
            V prod = 1;
            for (int j = 0; j < F.d; ++j) prod *= atom(m, j, ix(j));
            f += prod;
        }
        return f;
    }
    case TT_FN_MAXWELL_2D2V:
    case TT_FN_MAXWELL_3D3V: {
        // x modes: rows rho/(2 sqrt(2 pi T)) and 2T; v modes: (v - 3/4)^2 and (v + 3/4)^2
        const int ndim = (F.id == TT_FN_MAXWELL_2D2V) ? 2 : 3;
        V pre = 0, em = 0, ep = 0;
        for (int w = 0; w < ndim; ++w) {
            const int ix_x = ix(2 * w), ix_v = ix(2 * w + 1);
            const V t2 = atom(1, 2 * w, ix_x);
            pre += atom(0, 2 * w, ix_x);
            em += atom(0, 2 * w + 1, ix_v) / t2;
            ep += atom(1, 2 * w + 1, ix_v) / t2;
        }
        return pre * (M<V>::exp(-em) + M<V>::exp(-ep));
    }
    }
    return (V)0;
}

template <typename V, int FNS = 0, typename IX> __device__ inline V fn_value_ix(const FnDev &F, IX ix)
{
    return fn_value_tx<V, FNS>(F, ix, as_global(fn_table<V>(F)));
}

template <typename V, int FNS = 0> __device__ inline V fn_value(const FnDev &F, const int *idx)
{
    return fn_value_ix<V, FNS>(F, [&](int j) { return idx[j]; });
}


// ---------------------------------------------------------------------------
// Problem layout in device memory.
// Unfolding u = k-1 (k = 1..d-1 in the paper's numbering) owns superblock
// X_k(I_{<=k-1} x [n_k], [n_{k+1}] x J_{>k+1}).  Row position of (p, i_k) is
// p*n_k + i_k, column position of (i_{k+1}, q) is q*n_{k+1} + i_{k+1}, with p,
// q the insertion indices in I_{<=k-1} and J_{>k+1}; index sets only grow, so
// positions never move and the superblock grows by appending row and column
// blocks.
// ---------------------------------------------------------------------------
struct Cand {
    double v;        // |residual| (-1 = none)
    uint64_t key;    // (row << 32) | col
    double sv;       // signed residual
};

struct KDev {
    int k;                        // paper index of the unfolding
    int nk, nk1;                  // n_k, n_{k+1}
    int rowcap, colcap;           // capacity of the stored superblock
    int ld;                       // row pitch of E in entries (colcap padded off powers of two)
    int rk_cap;                   // pivot capacity of this unfolding
    int RTp, CTq;                 // row tiles per prefix, column tiles per suffix
    int TR, TC;                   // largest tile extent (LDS/thread layout)
    const int *rt_start, *rt_len, *rt_blk;    // per row tile within a prefix
    const int *ct_start, *ct_len, *ct_blk;    // per column tile within a suffix
    void *E;                      // residual / frozen factors, rowcap x colcap, row-major, pitch ld
    uint8_t *rpiv, *cpiv;         // z+1 on the row / column of pivot z, else 0 (padded to whole words)
    int *Ifull;                   // I_{<=k}: rcap tuples of k indices
    int *Jfull;                   // J_{>k}: rcap tuples of d-k indices
    int *rho, *gam;               // pivot positions in the superblock
    double *piv;                  // pivot residual in sweep precision (widened)
    double *piv64;                // FP64 pivot residual (FP32 sweeps: from the FP64 check)
    double *Wp64;                 // FP64 pivot-block factors: Wp64[z*rcap+z'] (z' < z)
    double *Up64;                 // Up64[z'*rcap+z] (z' < z)
    Cand *cand;                   // per-tile (rook: per-block) candidates of the current sweep
    int cand_cap;
    double *hist;                 // per-sweep largest |residual|
    // rook mode: factors instead of a stored residual, and the block grid
    double *Wf;                   // W(i, z) = Wf[i * factor_pitch(rk_cap) + z], rowcap rows
    double *Uf;                   // U(z, j) = Uf[j * factor_pitch(rk_cap) + z], colcap columns
    int nrb, ncb;                 // row blocks (modes 1..k), column blocks (modes k+1..d)
    unsigned long long *bcnt;     // residuals looked at per block in the current sweep
    // rook search split over G workgroups per block
    Cand *rpart;                  // partial bests: 2 buffers x blocks x G
    struct RookState *rst;        // block states: 2 buffers x blocks
    unsigned long long *rcnt;     // counts per (block, workgroup) in the current sweep
};

// The fields of an unfolding's descriptor that the search tiles read, with
// its neighbours' index-tuple arrays; kept apart and small, so that a search
// workgroup loads every unfolding's copy in its first round of loads.
struct KTile {
    int nk, nk1, ld, RTp, CTq, TR, TC, pad;
    const int *rt_start, *rt_len, *ct_start, *ct_len;
    void *E;
    const uint8_t *rpiv, *cpiv;
    const int *rho, *gam;
    const double *piv;
    const int *Ifull, *Jfull;
    const int *Ipre;              // I_{<=k-1} (unfolding k-1), null for k = 1
    const int *Jsuf;              // J_{>k+1} (unfolding k+1), null for k = d-1
    Cand *cand;
};
constexpr int KTILE_WORDS = (int)(sizeof(KTile) / 4);

// A block's rook search between the launches of the split search.
struct RookState {
    double v, sv;                 // |residual| and residual at (ci, cj)
    int ci, cj;                   // current row and column positions
    int valid;                    // the block has a start
    int active;                   // still searching
    int moved;                    // moved in the current round
    int rounds;                   // rounds of Alg. 1's loop completed
};

// What one search sweep does to one unfolding, prepared by the previous commit.
struct KSweep {
    int rk;                       // committed pivots (all eliminated from new entries)
    int apply;                    // 1: pivot rk-1 still has to be applied to stored residuals
    int nr_st, nc_st;             // stored region (the previous sweep's superblock)
    int nr, nc;                   // this sweep's superblock
    int arho, agam;               // position of pivot rk-1
    double apiv;                  // its value in sweep precision
};

// Tiles per unfolding of one sweep, split into new-entry tiles and stored
// tiles, with the running offsets of both kinds over the unfoldings.
struct SweepShape {
    int RT[TT_MAX_D], CT[TT_MAX_D], RTs[TT_MAX_D], CTs[TT_MAX_D];
    int noff[TT_MAX_D + 1], soff[TT_MAX_D + 1];
};
constexpr int SHAPE_WORDS = (int)(sizeof(SweepShape) / sizeof(int));

struct ProbState {
    int r[2][TT_MAX_D + 1];       // committed ranks, double-buffered by sweep parity
    KSweep ks[TT_MAX_D];
    SweepShape sh;                // tile counts of the sweep ks describes
    int stop, capped, err, sweeps;
    unsigned long long pivoted;
    unsigned long long alg_bytes;   // algorithmic residual traffic of the tile launches
    unsigned long long new_entries; // entries evaluated by the tile launches
    double rms, tau;
    int i0[TT_MAX_D];
    double last_best[TT_MAX_D];
    int rook_rounds;              // rook mode: most rounds any block walk of the run took
    int rook_long;                // rook mode: block walks longer than TT_ROOK_ITERS rounds
};

struct HostMirror {                // fine-grained host memory, written by the device
    int sweeps_done;
    int stop;
    int err;
    int r[TT_MAX_D + 1];
};

// Partial result of one workgroup of the sample pass (see samples_body).
struct SamplePart {
    double sumsq;
    double bv, bs;                // largest |value|, its signed value
    uint64_t bk;                  // its sample index
    int bad;                      // a non-finite value was seen
    int pad;
};

// Workgroups of the sample pass: one sample per thread, at least 64 (the
// pass also clears the pivot masks).
__host__ __device__ inline int sample_blocks(int ns)
{
    const int b = (ns + NT - 1) / NT;
    return b > 64 ? b : 64;
}

// Per-run inputs of a problem solved inside a batch (a single solve passes
// them as kernel arguments instead).
struct RunDev {
    uint64_t seed;
    double eps;
    int ns;                       // samples
    double *vals;                 // ns sample values
    SamplePart *spart;            // sample_blocks(ns) partial results
    double *cores;                // output cores
    int64_t verify_R;             // samples of the sampled-error check (0: none)
};

// Restarts after false convergence (tt_options.restarts): the initial pivots
// of a restarted run.  pts holds the point list, i0 first; unfolding u holds
// m[u] of them (point mem[u][z] as pivot z, at superblock positions rho, gam).
// npts = 0: a plain run (one pivot, i0, from the samples).
constexpr int TT_MAX_SEEDS = 8;              // points after i0
constexpr int TT_RESTART_TRIES = 64;         // check samples tried per restart
struct SeedPlan {
    int npts;
    int pts[TT_MAX_SEEDS + 1][TT_MAX_D];
    int m[TT_MAX_D];
    int mem[TT_MAX_D][TT_MAX_SEEDS + 1];
    int rho[TT_MAX_D][TT_MAX_SEEDS + 1];
    int gam[TT_MAX_D][TT_MAX_SEEDS + 1];
};

// Candidate points for the next restart: cand[c] enters the unfoldings whose
// bit is set in cin[c].
struct PointCheck {
    int nc;
    int cand[TT_RESTART_TRIES][TT_MAX_D];
    int cin[TT_RESTART_TRIES];
};

struct ProbDev {
    int d, nk;                    // modes, unfoldings (= d-1)
    int r_max, rcap;
    int hist_cap;
    int fp32;                     // sweeps in FP32 with FP64 pivot check
    int rook;                     // rook search (Alg. 1 per block) on factors, FP64
    int rook_g;                   // workgroups per block of the split rook search (1: not split)
    int grid[TT_MAX_D];           // subtensor blocks per mode
    FnDev F;
    KDev kd[TT_MAX_D];
    KTile kt[TT_MAX_D];           // the search tiles' copy of kd
    ProbState *S;
    HostMirror *hm;               // device alias of the host mirror
    RunDev run;
    SweepShape sh0;               // tile counts of the first sweep (every tile stored)
    const SeedPlan *plan;         // initial pivots of a restarted run (device)
    // phase stamps (only in the library built with TT_STAMPS; null otherwise):
    // STAMP_WORDS clock values per search workgroup (stamp_wgs per sweep),
    // then STAMP_WORDS per commit launch
    unsigned long long *stamps;
    int stamp_wgs, stamp_sweeps;
};

constexpr int STAMP_WORDS = 16;

struct SweepArgs {
    int sweep;
    int nk;
    ProbState *S;                 // the problem's state (saves a dependent load)
    // for the commit: each unfolding's candidate array and a bound on the
    // tiles (rook: blocks) the sweep searched, known on the host
    const Cand *cand[TT_MAX_D];
    int ntl_max[TT_MAX_D];
};

}  // namespace ttc
