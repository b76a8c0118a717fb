/*
 * tt_oracle.c -- plain, slow FP64 CPU oracle for greedy adaptive TT cross.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two are compared against
 * each other on the same seeded inputs.
 *
 * What it computes (Shi, Hayes, Qiu, "Distributed memory parallel adaptive
 * tensor-train cross approximation"):
 *   - the tensor is a black box evaluated entry by entry (Sec. 5 intro);
 *   - pivots for every unfolding k = 1..d-1 are found on the superblock
 *     X_k(I_{<=k-1} x [n_k], [n_{k+1}] x J_{>k+1}) (Alg. 2) by the greedy
 *     largest-|residual| rule (Alg. 1, full search);
 *   - the residual on a superblock is obtained from the raw entries by the
 *     rank-1 recursion of eq. (aca_approx_E) in residual form
 *       R_{z+1} = R_z - R_z(:,j) R_z(i,:) / R_z(i,j)
 *     (the paper's last line writes E = A~ - A with a "+": with that sign
 *     convention the update must be subtracted; the derivation line before it
 *     fixes the sign);
 *   - all unfoldings search on the same snapshot of the index sets and commit
 *     together ("dimension parallel", Sec. 2.3 and Sec. 3.2.3);
 *   - cores are built from the final pivots by Alg. 4 (eq. aca_approx_T) on the
 *     sliced fibers X(I_{<=k-1}, :, J_{>k}) and reshaped per eq. (corereshape);
 *   - accuracy is measured by the sampled relative error of Sec. 5 (reported
 *     as the square root of the printed ratio) or, on tiny tensors, by brute
 *     force over every entry (eq. FrobeniusNorm).
 *
 * Readings where the paper is silent (stated once here, used below):
 *   - stop: a sweep in which no unfolding finds |residual| > tau proposes
 *     nothing and ends the run; tau = eps * rms, with rms taken over N_s seeded
 *     sample entries (squares summed pairwise, see orc_pairwise_sumsq);  a k at
 *     the rank cap proposes nothing;
 *   - initial pivot: the sample with the largest |value| (first one on ties),
 *     replicated as pivot 1 of every unfolding (Alg. 1 starts from samples);
 *   - tie-break: lowest (row position, column position), where row position =
 *     p * n_k + i_k with p the insertion index of the prefix in I_{<=k-1} and
 *     column position = q * n_{k+1} + i_{k+1} with q the insertion index of
 *     the suffix in J_{>k+1};
 *   - rows and columns that already hold a pivot are excluded from the search;
 *   - arithmetic: IEEE double, explicit fma for every multiply-subtract of the
 *     recursion, plain division, sums in ascending index order; the file is
 *     compiled with -ffp-contract=off.
 *
 * Rook mode (orc_set_rook): the search on each superblock is Alg. 1 run
 * inside every subtensor block (Alg. 3's local pivot), and the pivot of the
 * unfolding is the best of the local ones.  Readings:
 *   - blocks: mode j is split into C_j pieces, piece b holding indices
 *     [floor(b n_j / C_j), floor((b+1) n_j / C_j)); a superblock row (prefix
 *     tuple, i_k) lies in the block of its k indices, a column (i_{k+1},
 *     suffix tuple) in the block of its d-k indices; row-block and
 *     column-block ids are mixed-radix numbers with the first mode fastest,
 *     and the block id is rowblock + (row blocks) * colblock;
 *   - the random set of Alg. 1: L = max(64, |rows| + |cols|) pairs drawn from
 *     SplitMix64 started at seed XOR mix(k | sweep << 8 | block << 32), where
 *     mix is SplitMix64's output function; each pair is (row draw mod |rows|,
 *     column draw mod |cols|) over the block's rows and columns in ascending
 *     position; pairs on a pivot row or column are skipped; if none is left,
 *     the start is the block's first row and first column without a pivot;
 *   - the loop of Alg. 1: a column step (largest |residual| in the current
 *     column) then a row step (in the current row), each taken only if it is
 *     strictly larger, until neither step moves.  Every move strictly raises
 *     |residual| over a finite set, so the loop ends by itself (a row once
 *     left by a row step is never entered again, so there are at most
 *     |rows| + 1 rounds); a cap on the rounds is a test option only.  Among
 *     equal values the lowest position wins, as in the greedy search;
 *   - the pivoted count adds one per residual the search looks at (each
 *     sample kept, each row or column entry scanned).
 *
 * Restarts after false convergence (orc_set_restarts; not in the paper,
 * which guards against it only by the random start of Alg. 1 and reports the
 * sampled error of Sec. 5).  A greedy run can stop with every superblock
 * residual at or below tau while the tensor has structure the superblocks
 * through its pivots never reach (their sampled error stays large).  The
 * remedy restarts the run from more initial pivots:
 *   - the initial index sets come from a list of points, i0 first: a point
 *     enters unfolding k when neither its prefix (i_1..i_k) is in I_{<=k} nor
 *     its suffix (i_{k+1}..i_d) in J_{>k} yet.  Those unfoldings form one
 *     run k_a..k_b (a prefix that is new at k is new at k+1, a suffix new at
 *     k is new at k-1), so every set stays nested: the point's prefix at
 *     k_a - 1 and its suffix at k_b + 1 are already present, and every
 *     unfolding's cross stays square.  Its pivot in unfolding k sits at the
 *     positions of its prefix and suffix; pivots keep the order of the list;
 *   - a point is usable only if, in every unfolding it enters, its residual
 *     after the earlier pivots of that unfolding is larger than tau in
 *     absolute value (a smaller one would be a near-singular pivot, and it
 *     cannot be left out of one unfolding alone without breaking nestedness).
 *     A sample that fails is trimmed to the longest run of consecutive
 *     unfoldings where its residual passes: its indices outside that run are
 *     replaced by i0's (orc_point_pick), and the trimmed point is tested
 *     again.  (The end unfoldings are the usual failures: an unfolding whose
 *     matrix has its exact rank already has zero residual everywhere.);
 *   - after a run, the sampled error (stream seed + 1, R samples) decides: at
 *     or below eps the run stands; else the samples are taken in order of
 *     decreasing |X - X~| (lowest sample first on ties), the point of the
 *     first one among the 64 worst that gives one joins the list, and the run
 *     is repeated from the samples on.  With no usable sample, or after max_restarts restarts, the
 *     status is ORC_WARN_SAMPLED_ERR (restart_cause says which).
 *
 * Indices are 0-based at this interface; the generating functions apply the
 * paper's 1-based formulas internally.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_D 16
#define ORC_MAX_SEEDS 8
#define ORC_RESTART_TRIES 64

enum { ORC_FN_HILBERT = 1, ORC_FN_MAXWELL = 2, ORC_FN_BIMAXWELL = 3, ORC_FN_SEPSUM = 4,
       ORC_FN_MAXWELL_2D2V = 5, ORC_FN_MAXWELL_3D3V = 6, ORC_FN_MAXWELL_IL = 7 };

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_WARN_SAMPLED_ERR = 2, ORC_EINVAL = -1, ORC_ENOMEM = -2,
       ORC_ESINGULAR = -4, ORC_EFN = -6 };

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state advances by the golden */
/* gamma, output is the variant-13 finaliser of the new state.               */
/* ------------------------------------------------------------------------ */
static uint64_t orc_sm64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_draw(uint64_t seed, int64_t count, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t t = 0; t < count; ++t) out[t] = orc_sm64(&s);
    return s;
}

/* Seeded multi-indices: coordinate j of sample s is draw mod n_j, draws taken */
/* in (s, j) order from one stream.                                            */
void orc_sample_indices(int d, const int *n, uint64_t seed, int64_t count, int *idx)
{
    uint64_t s = seed;
    for (int64_t t = 0; t < count; ++t)
        for (int j = 0; j < d; ++j) idx[t * d + j] = (int)(orc_sm64(&s) % (uint64_t)n[j]);
}

/* Sum of squares by pairwise summation: the squares, padded with zeros to a
 * power-of-two count, are added in adjacent pairs level by level until one
 * value remains.  (The paper does not fix a summation order for the sample
 * norm; a balanced tree is the order a parallel reduction can reproduce.) */
double orc_pairwise_sumsq(const double *v, int64_t n)
{
    int64_t m = 1;
    while (m < n) m <<= 1;
    double *a = (double *)calloc((size_t)m, sizeof(double));
    if (!a) return NAN;
    for (int64_t i = 0; i < n; ++i) a[i] = v[i] * v[i];
    for (int64_t w = m; w > 1; w >>= 1)
        for (int64_t i = 0; i < w / 2; ++i) a[i] = a[2 * i] + a[2 * i + 1];
    double s = a[0];
    free(a);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Generating functions.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int fn_id;
    int d;
    int n[ORC_MAX_D];
    const double *params;
    int nparams;
} orc_fn;

static const double ORC_PI = 3.14159265358979323846;

/* Hilbert tensor, eq. (HilbertTensor): 1 / (sum_j i_j + shift) with 1-based
 * i_j.  The paper's tensor has shift = 1 - d; params[0] overrides it. */
static double orc_hilbert(const orc_fn *F, const int *idx)
{
    double shift = (F->nparams >= 1) ? F->params[0] : (double)(1 - F->d);
    long long s = 0;
    for (int j = 0; j < F->d; ++j) s += (long long)idx[j] + 1;
    return 1.0 / ((double)s + shift);
}

/* Velocity grid: cell centres of [-vmax, vmax] split into n cells. */
static double orc_vel(int i, int n, double vmax)
{
    return -vmax + ((double)i + 0.5) * (2.0 * vmax / (double)n);
}

/* Single 3d3v Maxwellian, modes x1,x2,x3,v1,v2,v3; x on the periodic grid
 * i/n of [0,1), v cell-centred on [-vmax,vmax].
 *   f = rho(x) (2 pi T)^{-3/2} exp(-|v - u(x)|^2 / (2T)),
 *   rho = 1 + a sin(2 pi x1) cos(2 pi x2),  u = (b sin(2 pi x3), 0, 0).
 * params: [a=0.5, b=0.3, T=1, vmax=8]. */
static double orc_maxwell(const orc_fn *F, const int *idx)
{
    double a = 0.5, b = 0.3, T = 1.0, vmax = 8.0;
    if (F->nparams >= 4) { a = F->params[0]; b = F->params[1]; T = F->params[2]; vmax = F->params[3]; }
    double x1 = (double)idx[0] / F->n[0];
    double x2 = (double)idx[1] / F->n[1];
    double x3 = (double)idx[2] / F->n[2];
    double v1 = orc_vel(idx[3], F->n[3], vmax);
    double v2 = orc_vel(idx[4], F->n[4], vmax);
    double v3 = orc_vel(idx[5], F->n[5], vmax);
    double rho = 1.0 + a * sin(2.0 * ORC_PI * x1) * cos(2.0 * ORC_PI * x2);
    double ux = b * sin(2.0 * ORC_PI * x3);
    double q = (v1 - ux) * (v1 - ux) + v2 * v2 + v3 * v3;
    return rho * pow(2.0 * ORC_PI * T, -1.5) * exp(-q / (2.0 * T));
}

/* Sum of two spatially uniform 3v Maxwellians; the d-3 leading modes are
 * spatial and f does not depend on them; the last three are v1,v2,v3.
 * params: [rho1,u1x,u1y,u1z,T1, rho2,u2x,u2y,u2z,T2, vmax=8]. */
static double orc_bimaxwell(const orc_fn *F, const int *idx)
{
    const double *P = F->params;
    double vmax = (F->nparams >= 11) ? P[10] : 8.0;
    int d = F->d;
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = orc_vel(idx[d - 3 + c], F->n[d - 3 + c], vmax);
    double f = 0.0;
    for (int m = 0; m < 2; ++m) {
        const double *Q = P + 5 * m;
        double T = Q[4];
        double q = 0.0;
        for (int c = 0; c < 3; ++c) q += (v[c] - Q[1 + c]) * (v[c] - Q[1 + c]);
        f += Q[0] * pow(2.0 * ORC_PI * T, -1.5) * exp(-q / (2.0 * T));
    }
    return f;
}

/* Sum of r separable products: f = sum_m prod_j g_{m,j}(i_j).
 * params: [r, g...] with g_{m,j}(i) at 1 + m * sum(n) + (n_0 + .. + n_{j-1}) + i. */
static double orc_sepsum(const orc_fn *F, const int *idx)
{
    int r = (int)F->params[0];
    int total = 0;
    for (int j = 0; j < F->d; ++j) total += F->n[j];
    double f = 0.0;
    for (int m = 0; m < r; ++m) {
        double prod = 1.0;
        int off = 1 + m * total;
        for (int j = 0; j < F->d; ++j) { prod *= F->params[off + idx[j]]; off += F->n[j]; }
        f += prod;
    }
    return f;
}

/* The paper's kinetic examples (Sec. 5.2, eq. 2d2vFunction): modes x, v_x, y,
 * v_y (and z, v_z), x in [-1/2,1/2] and v in [-3,3]; grid points are the cell
 * centres of those intervals (the paper does not state the grid).
 *   rho(w) = 1 + 0.875 sin(2 pi w),  T(w) = 0.5 + 0.4 sin(2 pi w),
 *   f = sum_w rho(w)/(2 sqrt(2 pi T(w))) * [exp(-sum_w b_w^-) + exp(-sum_w b_w^+)],
 *   b_w^{+-} = |v_w +- 0.75|^2 / (2 T(w)).
 * For 3d3v the z and v_z terms are added to the spatial sum and to both
 * exponents (the paper only says "with the addition of z and v_z terms"). */
static double orc_cell(int i, int n, double lo, double hi)
{
    return lo + ((double)i + 0.5) * ((hi - lo) / (double)n);
}

static double orc_kinetic(const orc_fn *F, const int *idx, int ndim)
{
    double pre = 0.0, em = 0.0, ep = 0.0;
    for (int w = 0; w < ndim; ++w) {
        double x = orc_cell(idx[2 * w], F->n[2 * w], -0.5, 0.5);
        double v = orc_cell(idx[2 * w + 1], F->n[2 * w + 1], -3.0, 3.0);
        double rho = 1.0 + 0.875 * sin(2.0 * ORC_PI * x);
        double T = 0.5 + 0.4 * sin(2.0 * ORC_PI * x);
        pre += rho / (2.0 * sqrt(2.0 * ORC_PI * T));
        em += (v - 0.75) * (v - 0.75) / (2.0 * T);
        ep += (v + 0.75) * (v + 0.75) / (2.0 * T);
    }
    return pre * (exp(-em) + exp(-ep));
}

/* The same Maxwellian with its modes in the order x1, v1, x2, v2, x3, v3
 * (the position-velocity interleaving the paper uses for its kinetic
 * tensors): mode 2w holds x_{w+1}, mode 2w+1 holds v_{w+1}. */
static double orc_maxwell_il(const orc_fn *F, const int *idx)
{
    orc_fn G = *F;
    int p[6];
    for (int w = 0; w < 3; ++w) {
        p[w] = idx[2 * w];
        p[3 + w] = idx[2 * w + 1];
        G.n[w] = F->n[2 * w];
        G.n[3 + w] = F->n[2 * w + 1];
    }
    return orc_maxwell(&G, p);
}

static double orc_eval(const orc_fn *F, const int *idx)
{
    switch (F->fn_id) {
    case ORC_FN_HILBERT: return orc_hilbert(F, idx);
    case ORC_FN_MAXWELL: return orc_maxwell(F, idx);
    case ORC_FN_MAXWELL_IL: return orc_maxwell_il(F, idx);
    case ORC_FN_BIMAXWELL: return orc_bimaxwell(F, idx);
    case ORC_FN_SEPSUM: return orc_sepsum(F, idx);
    case ORC_FN_MAXWELL_2D2V: return orc_kinetic(F, idx, 2);
    case ORC_FN_MAXWELL_3D3V: return orc_kinetic(F, idx, 3);
    }
    return NAN;
}

static int orc_fn_check(int fn_id, int d, const int *n, const double *params, int nparams)
{
    if (d < 2 || d > ORC_MAX_D) return ORC_EINVAL;
    for (int j = 0; j < d; ++j) if (n[j] < 1) return ORC_EINVAL;
    switch (fn_id) {
    case ORC_FN_HILBERT: {
        double shift = (nparams >= 1) ? params[0] : (double)(1 - d);
        if ((double)d + shift <= 0.0) return ORC_EFN;    /* smallest denominator */
        return ORC_OK;
    }
    case ORC_FN_MAXWELL:
    case ORC_FN_MAXWELL_IL: return (d == 6 && (nparams == 0 || nparams >= 4)) ? ORC_OK : ORC_EFN;
    case ORC_FN_BIMAXWELL: return (d >= 3 && nparams >= 10) ? ORC_OK : ORC_EFN;
    case ORC_FN_SEPSUM: {
        if (nparams < 1) return ORC_EFN;
        int r = (int)params[0], total = 0;
        for (int j = 0; j < d; ++j) total += n[j];
        return (r >= 1 && nparams >= 1 + r * total) ? ORC_OK : ORC_EFN;
    }
    case ORC_FN_MAXWELL_2D2V: return d == 4 ? ORC_OK : ORC_EFN;
    case ORC_FN_MAXWELL_3D3V: return d == 6 ? ORC_OK : ORC_EFN;
    }
    return ORC_EFN;
}

/* Evaluate m entries (idx is m x d). */
int orc_fn_eval(int fn_id, int d, const int *n, const double *params, int nparams,
                int64_t m, const int *idx, double *out)
{
    int st = orc_fn_check(fn_id, d, n, params, nparams);
    if (st) return st;
    orc_fn F = { fn_id, d, {0}, params, nparams };
    for (int j = 0; j < d; ++j) F.n[j] = n[j];
    for (int64_t t = 0; t < m; ++t) out[t] = orc_eval(&F, idx + t * d);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Solver state.                                                              */
/* Unfoldings are numbered k = 1..d-1 as in the paper.  I[k] holds the       */
/* pivot row tuples (i_1..i_k) of X_k, J[k] the column tuples (i_{k+1}..i_d); */
/* I[0] and J[d] are the single empty tuple.                                  */
/* ------------------------------------------------------------------------ */
typedef struct orc_state {
    orc_fn F;
    double *params_copy;
    double eps;
    uint64_t seed;
    int r_max, n_samples;
    int d;
    int n[ORC_MAX_D];
    int r[ORC_MAX_D + 1];            /* r[0] = r[d] = 1 */
    int *I[ORC_MAX_D + 1];           /* I[k]: r_max x k */
    int *J[ORC_MAX_D + 1];           /* J[k]: r_max x (d-k) */
    int64_t *rho[ORC_MAX_D + 1];     /* pivot row positions in superblock k */
    int64_t *gam[ORC_MAX_D + 1];     /* pivot column positions */
    double *piv[ORC_MAX_D + 1];      /* pivot residuals p_z */
    double *best_hist[ORC_MAX_D + 1];/* per sweep: largest unmasked |residual| */
    double *gap_hist[ORC_MAX_D + 1]; /* per sweep: (best - runner-up) / best, 1 if none */
    int sweeps, hist_cap;
    double rms, tau;
    int i0[ORC_MAX_D];
    int64_t evaluated, pivoted;
    double min_rel_gap;              /* smallest (best - runner up)/best seen */
    int status;
    int ran;
    double *cores;                   /* G_1..G_d concatenated */
    int64_t cores_len;
    int rook, rook_iters;            /* rook mode: Alg. 1 inside every block; rook_iters = 0: no cap */
    int rook_max_rounds;             /* most rounds any block's walk took */
    int kcap[ORC_MAX_D + 1];         /* rank cap per unfolding (prescribed ranks), <= r_max */
    int grid[ORC_MAX_D];             /* subtensor blocks per mode (rook mode) */
    /* restarts after false convergence */
    int max_restarts;                /* 0: off */
    int64_t restart_R;               /* samples of the check that decides a restart */
    int nseed;                       /* points after i0 in the initial list */
    int seeds[ORC_MAX_SEEDS][ORC_MAX_D];
    int restarts_used, restart_cause;/* cause: 0 none, 1 restarts used up, 2 no usable sample */
    double sampled_err;              /* the last check's error (restarts on) */
} orc_state;

static void orc_free_state(orc_state *S)
{
    if (!S) return;
    for (int k = 0; k <= ORC_MAX_D; ++k) {
        free(S->I[k]); free(S->J[k]); free(S->rho[k]); free(S->gam[k]); free(S->piv[k]);
        free(S->best_hist[k]); free(S->gap_hist[k]);
    }
    free(S->params_copy);
    free(S->cores);
    free(S);
}

void orc_destroy(orc_state *S) { orc_free_state(S); }

orc_state *orc_create(int d, const int *n, double eps, int fn_id, const double *params, int nparams,
                      uint64_t seed, int r_max, int n_samples)
{
    if (orc_fn_check(fn_id, d, n, params, nparams) != ORC_OK) return NULL;
    if (!(eps >= 0.0) || r_max < 1 || n_samples < 1) return NULL;
    orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
    if (!S) return NULL;
    S->d = d;
    for (int j = 0; j < d; ++j) S->n[j] = n[j];
    S->eps = eps; S->seed = seed; S->r_max = r_max; S->n_samples = n_samples;
    if (nparams > 0) {
        S->params_copy = (double *)malloc(sizeof(double) * nparams);
        memcpy(S->params_copy, params, sizeof(double) * nparams);
    }
    S->F.fn_id = fn_id; S->F.d = d; S->F.params = S->params_copy; S->F.nparams = nparams;
    for (int j = 0; j < d; ++j) S->F.n[j] = n[j];
    S->hist_cap = (d - 1) * r_max + 2;
    S->rook = 0;
    S->rook_iters = 0;
    for (int k = 0; k <= ORC_MAX_D; ++k) S->kcap[k] = r_max;
    for (int j = 0; j < ORC_MAX_D; ++j) S->grid[j] = 1;
    for (int k = 1; k <= d - 1; ++k) {
        S->I[k] = (int *)calloc((size_t)r_max * k, sizeof(int));
        S->J[k] = (int *)calloc((size_t)r_max * (d - k), sizeof(int));
        S->rho[k] = (int64_t *)calloc(r_max, sizeof(int64_t));
        S->gam[k] = (int64_t *)calloc(r_max, sizeof(int64_t));
        S->piv[k] = (double *)calloc(r_max, sizeof(double));
        S->best_hist[k] = (double *)calloc(S->hist_cap, sizeof(double));
        S->gap_hist[k] = (double *)calloc(S->hist_cap, sizeof(double));
        if (!S->I[k] || !S->J[k] || !S->rho[k] || !S->gam[k] || !S->piv[k] || !S->best_hist[k] || !S->gap_hist[k]) {
            orc_free_state(S);
            return NULL;
        }
    }
    return S;
}

/* Multi-index of superblock entry (row, col) of unfolding k (1-based k):
 * row = p * n_k + i_k with prefix I[k-1][p]; col = q * n_{k+1} + i_{k+1} with
 * suffix J[k+1][q]. */
static void orc_entry_index(const orc_state *S, int k, int64_t row, int64_t col, int *idx)
{
    int d = S->d;
    int nk = S->n[k - 1], nk1 = S->n[k];
    int64_t p = row / nk, q = col / nk1;
    for (int j = 0; j < k - 1; ++j) idx[j] = S->I[k - 1][p * (k - 1) + j];
    idx[k - 1] = (int)(row % nk);
    idx[k] = (int)(col % nk1);
    int sl = d - k - 1;                                  /* length of J_{>k+1} tuples */
    for (int j = 0; j < sl; ++j) idx[k + 1 + j] = S->J[k + 1][q * sl + j];
}

/* Rook mode on: grid[j] blocks per mode (clamped to [1, n_j]; NULL = 1).
 * max_iters = 0 runs Alg. 1's loop until neither step moves (the method);
 * max_iters > 0 stops a walk after that many rounds (a test option). */
int orc_set_rook(orc_state *S, const int *grid, int max_iters)
{
    if (!S || max_iters < 0) return ORC_EINVAL;
    S->rook = 1;
    S->rook_iters = max_iters;
    for (int j = 0; j < S->d; ++j) {
        int c = grid ? grid[j] : 1;
        if (c < 1) c = 1;
        if (c > S->n[j]) c = S->n[j];
        S->grid[j] = c;
    }
    return ORC_OK;
}

/* Prescribed ranks (Sec. 5 runs at fixed core ranks): unfolding k stops
 * growing at min(r_max, caps[k-1]); caps holds d-1 values >= 1. */
int orc_set_rank_caps(orc_state *S, const int *caps)
{
    if (!S || !caps) return ORC_EINVAL;
    for (int k = 1; k <= S->d - 1; ++k) {
        if (caps[k - 1] < 1) return ORC_EINVAL;
        S->kcap[k] = caps[k - 1] < S->r_max ? caps[k - 1] : S->r_max;
    }
    return ORC_OK;
}

/* Piece of index i when n indices are split evenly into C pieces (Sec. 3):
 * piece b holds [floor(b n / C), floor((b+1) n / C)). */
static int orc_piece(int i, int n, int C)
{
    int b = 0;
    while (b + 1 < C && (int64_t)(b + 1) * n / C <= i) ++b;
    return b;
}

/* SplitMix64's output function (the finaliser without the state step). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* (a, ia, ja) beats (b, ib, jb): larger value, else lower position. */
static int orc_beats(double a, int64_t ia, int64_t ja, double b, int64_t ib, int64_t jb)
{
    if (a != b) return a > b;
    return ia < ib || (ia == ib && ja < jb);
}

/* Alg. 1 inside every subtensor block of superblock k (residual E, nrow x
 * ncol, masks of the pivot rows and columns), then the best of the local
 * pivots (Alg. 3).  Returns 1 and the pivot if some block has an entry
 * outside the pivot rows and columns. */
static int orc_rook_search(orc_state *S, int k, const int *rs, const double *E, int64_t nrow, int64_t ncol,
                           const unsigned char *rmask, const unsigned char *cmask, int64_t *row_out,
                           int64_t *col_out, double *val_out, int64_t *count_out)
{
    int d = S->d, nk = S->n[k - 1], nk1 = S->n[k];
    int sl = d - k - 1;
    int64_t *rblk = (int64_t *)malloc(sizeof(int64_t) * nrow);
    int64_t *cblk = (int64_t *)malloc(sizeof(int64_t) * ncol);
    int64_t *brow = (int64_t *)malloc(sizeof(int64_t) * nrow);
    int64_t *bcol = (int64_t *)malloc(sizeof(int64_t) * ncol);
    if (!rblk || !cblk || !brow || !bcol) {
        free(rblk); free(cblk); free(brow); free(bcol);
        return -1;
    }
    (void)rs;
    int64_t nrb = 1, ncb = 1;
    for (int j = 0; j < k; ++j) nrb *= S->grid[j];
    for (int j = k; j < d; ++j) ncb *= S->grid[j];
    for (int64_t i = 0; i < nrow; ++i) {
        int64_t p = i / nk, id = 0, mul = 1;
        for (int j = 0; j < k - 1; ++j) {
            id += orc_piece(S->I[k - 1][p * (k - 1) + j], S->n[j], S->grid[j]) * mul;
            mul *= S->grid[j];
        }
        id += orc_piece((int)(i % nk), nk, S->grid[k - 1]) * mul;
        rblk[i] = id;
    }
    for (int64_t c = 0; c < ncol; ++c) {
        int64_t q = c / nk1, id = orc_piece((int)(c % nk1), nk1, S->grid[k]), mul = S->grid[k];
        for (int j = 0; j < sl; ++j) {
            id += orc_piece(S->J[k + 1][q * sl + j], S->n[k + 1 + j], S->grid[k + 1 + j]) * mul;
            mul *= S->grid[k + 1 + j];
        }
        cblk[c] = id;
    }
    int found = 0;
    double best = -1.0, bestv = 0.0;
    int64_t br = -1, bc = -1, count = 0;
    for (int64_t cb = 0; cb < ncb; ++cb) {
        for (int64_t rb = 0; rb < nrb; ++rb) {
            int64_t nR = 0, nC = 0;
            for (int64_t i = 0; i < nrow; ++i) if (rblk[i] == rb) brow[nR++] = i;
            for (int64_t c = 0; c < ncol; ++c) if (cblk[c] == cb) bcol[nC++] = c;
            if (nR == 0 || nC == 0) continue;
            /* the random start of Alg. 1 */
            uint64_t tag = (uint64_t)k | ((uint64_t)S->sweeps << 8) | ((uint64_t)(rb + nrb * cb) << 32);
            uint64_t st = S->seed ^ orc_mix64(tag);
            int64_t L = nR + nC > 64 ? nR + nC : 64;
            int have = 0;
            double v = -1.0;
            int64_t bi = -1, bj = -1;
            for (int64_t t = 0; t < L; ++t) {
                uint64_t a = orc_sm64(&st), b = orc_sm64(&st);
                int64_t i = brow[a % (uint64_t)nR], j = bcol[b % (uint64_t)nC];
                if (rmask[i] || cmask[j]) continue;
                ++count;
                double x = fabs(E[i * ncol + j]);
                if (!have || orc_beats(x, i, j, v, bi, bj)) { v = x; bi = i; bj = j; have = 1; }
            }
            if (!have) {
                for (int64_t t = 0; t < nR && bi < 0; ++t) if (!rmask[brow[t]]) bi = brow[t];
                for (int64_t t = 0; t < nC && bj < 0; ++t) if (!cmask[bcol[t]]) bj = bcol[t];
                if (bi < 0 || bj < 0) continue;
                v = fabs(E[bi * ncol + bj]);
                ++count;
            }
            /* column step, row step, while either finds a strictly larger entry */
            for (int it = 0; S->rook_iters == 0 || it < S->rook_iters; ++it) {
                int moved = 0;
                if (it + 1 > S->rook_max_rounds) S->rook_max_rounds = it + 1;
                int64_t ti = -1;
                double tv = -1.0;
                for (int64_t t = 0; t < nR; ++t) {
                    int64_t i = brow[t];
                    if (rmask[i]) continue;
                    ++count;
                    double x = fabs(E[i * ncol + bj]);
                    if (x > tv) { tv = x; ti = i; }
                }
                if (tv > v) { v = tv; bi = ti; moved = 1; }
                int64_t tj = -1;
                tv = -1.0;
                for (int64_t t = 0; t < nC; ++t) {
                    int64_t j = bcol[t];
                    if (cmask[j]) continue;
                    ++count;
                    double x = fabs(E[bi * ncol + j]);
                    if (x > tv) { tv = x; tj = j; }
                }
                if (tv > v) { v = tv; bj = tj; moved = 1; }
                if (!moved) break;
            }
            if (!found || orc_beats(v, bi, bj, best, br, bc)) {
                best = v; br = bi; bc = bj; bestv = E[bi * ncol + bj]; found = 1;
            }
        }
    }
    free(rblk); free(cblk); free(brow); free(bcol);
    *row_out = br;
    *col_out = bc;
    *val_out = bestv;
    *count_out = count;
    return found;
}

/* One greedy search on superblock k from the raw entries, with the current
 * pivots eliminated in insertion order.  Returns 1 and the position of the
 * largest unmasked |residual| if one exists. */
static int orc_search(orc_state *S, int k, const int *rs, int64_t *row_out, int64_t *col_out,
                      double *val_out, double *runner_out)
{
    int d = S->d;
    int64_t nrow = (int64_t)rs[k - 1] * S->n[k - 1];
    int64_t ncol = (int64_t)S->n[k] * rs[k + 1];
    int nz = rs[k];
    double *E = (double *)malloc(sizeof(double) * nrow * ncol);
    double *u = (double *)malloc(sizeof(double) * ncol);
    double *w = (double *)malloc(sizeof(double) * nrow);
    unsigned char *rmask = (unsigned char *)calloc(nrow, 1);
    unsigned char *cmask = (unsigned char *)calloc(ncol, 1);
    int idx[ORC_MAX_D];
    if (!E || !u || !w || !rmask || !cmask) {
        free(E); free(u); free(w); free(rmask); free(cmask);
        S->status = ORC_ENOMEM;
        return -1;
    }
    /* raw entries X(R_k, C_k) */
    for (int64_t i = 0; i < nrow; ++i)
        for (int64_t j = 0; j < ncol; ++j) {
            orc_entry_index(S, k, i, j, idx);
            E[i * ncol + j] = orc_eval(&S->F, idx);
        }
    (void)d;
    /* residual: eliminate pivots z = 1..r_k in insertion order */
    for (int z = 0; z < nz; ++z) {
        int64_t pr = S->rho[k][z], pc = S->gam[k][z];
        double p = E[pr * ncol + pc];
        for (int64_t j = 0; j < ncol; ++j) u[j] = E[pr * ncol + j] / p;
        for (int64_t i = 0; i < nrow; ++i) w[i] = E[i * ncol + pc];
        for (int64_t i = 0; i < nrow; ++i)
            for (int64_t j = 0; j < ncol; ++j)
                E[i * ncol + j] = fma(-w[i], u[j], E[i * ncol + j]);
        rmask[pr] = 1;
        cmask[pc] = 1;
    }
    if (S->rook) {
        int64_t cnt = 0;
        double v = 0.0;
        int f = orc_rook_search(S, k, rs, E, nrow, ncol, rmask, cmask, row_out, col_out, &v, &cnt);
        free(E); free(u); free(w); free(rmask); free(cmask);
        if (f < 0) { S->status = ORC_ENOMEM; return -1; }
        if (f) *val_out = v;
        *runner_out = 0.0;               /* no gap log in rook mode */
        S->pivoted += cnt;
        return f;
    }
    /* argmax |E| over unmasked entries; row-major scan with strict '>' keeps
     * the lowest (row, col) among equal values */
    int found = 0;
    double best = -1.0;
    int64_t br = -1, bc = -1;
    for (int64_t i = 0; i < nrow; ++i) {
        if (rmask[i]) continue;
        for (int64_t j = 0; j < ncol; ++j) {
            if (cmask[j]) continue;
            double a = fabs(E[i * ncol + j]);
            if (!found || a > best) { best = a; br = i; bc = j; found = 1; }
        }
    }
    double runner = 0.0;
    if (found) {
        for (int64_t i = 0; i < nrow; ++i) {
            if (rmask[i]) continue;
            for (int64_t j = 0; j < ncol; ++j) {
                if (cmask[j]) continue;
                double a = fabs(E[i * ncol + j]);
                if (a != best && a > runner) runner = a;
            }
        }
        *val_out = E[br * ncol + bc];
    }
    *row_out = br;
    *col_out = bc;
    *runner_out = runner;
    S->pivoted += nrow * ncol;
    free(E); free(u); free(w); free(rmask); free(cmask);
    return found;
}

/* Position of tuple t (len entries) among the first cnt tuples of L, or -1;
 * the empty tuple (len 0) is at position 0. */
static int orc_find_tuple(const int *L, int cnt, int len, const int *t)
{
    if (len == 0) return 0;
    for (int p = 0; p < cnt; ++p) {
        int j = 0;
        while (j < len && L[p * len + j] == t[j]) ++j;
        if (j == len) return p;
    }
    return -1;
}

/* The unfoldings point pt enters (in[k] = 1): those where neither its prefix
 * nor its suffix is in the sets yet.  Returns their number, or -1 if they do
 * not form one run (which nested sets rule out) or one is at its rank cap. */
static int orc_point_levels(const orc_state *S, const int *pt, int *in)
{
    int d = S->d, cnt = 0, first = -1, last = -1;
    for (int k = 1; k <= d - 1; ++k) {
        in[k] = orc_find_tuple(S->I[k], S->r[k], k, pt) < 0 && orc_find_tuple(S->J[k], S->r[k], d - k, pt + k) < 0;
        if (in[k]) {
            if (first < 0) first = k;
            last = k;
            ++cnt;
            if (S->r[k] >= S->kcap[k]) return -1;
        }
    }
    if (cnt > 0 && last - first + 1 != cnt) return -1;
    return cnt;
}

/* Appends point pt to the unfoldings marked in in[]: its tuples first, then
 * its pivot positions (its prefix at k - 1 and its suffix at k + 1 may be its
 * own, appended in the first pass). */
static void orc_append_point(orc_state *S, const int *pt, const int *in)
{
    int d = S->d;
    for (int k = 1; k <= d - 1; ++k) {
        if (!in[k]) continue;
        int z = S->r[k];
        for (int j = 0; j < k; ++j) S->I[k][z * k + j] = pt[j];
        for (int j = 0; j < d - k; ++j) S->J[k][z * (d - k) + j] = pt[k + j];
        S->r[k] = z + 1;
    }
    for (int k = 1; k <= d - 1; ++k) {
        if (!in[k]) continue;
        int z = S->r[k] - 1;
        int p = orc_find_tuple(S->I[k - 1], S->r[k - 1], k - 1, pt);
        int q = orc_find_tuple(S->J[k + 1], S->r[k + 1], d - k - 1, pt + k + 1);
        S->rho[k][z] = (int64_t)p * S->n[k - 1] + pt[k - 1];
        S->gam[k][z] = (int64_t)q * S->n[k] + pt[k];
    }
}

/* Residuals at the pivots of unfolding k: pv[z] is the residual at pivot z
 * after pivots 0..z-1, by the rank-1 recursion restricted to the pivot rows
 * and columns (an entry of those depends on nothing else).  The matrix entry
 * (a, b) is X at the a-th row tuple of I_{<=k} followed by the b-th column
 * tuple of J_{>k}. */
static int orc_pivot_residuals(orc_state *S, int k, double *pv)
{
    int d = S->d, m = S->r[k];
    int idx[ORC_MAX_D];
    double *P = (double *)malloc(sizeof(double) * m * m);
    double *u = (double *)malloc(sizeof(double) * m);
    if (!P || !u) { free(P); free(u); return ORC_ENOMEM; }
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            for (int j = 0; j < k; ++j) idx[j] = S->I[k][a * k + j];
            for (int j = 0; j < d - k; ++j) idx[k + j] = S->J[k][b * (d - k) + j];
            P[a * m + b] = orc_eval(&S->F, idx);
        }
    for (int z = 0; z < m; ++z) {
        double p = P[z * m + z];
        pv[z] = p;
        for (int b = 0; b < m; ++b) u[b] = P[z * m + b] / p;
        for (int a = 0; a < m; ++a) {
            double w = P[a * m + z];
            for (int b = 0; b < m; ++b) P[a * m + b] = fma(-w, u[b], P[a * m + b]);
        }
    }
    free(P); free(u);
    return ORC_OK;
}

/* Initial index sets from i0 and the seeds, in that order, with the pivot
 * residuals of every unfolding. */
static int orc_init_sets(orc_state *S)
{
    int d = S->d, in[ORC_MAX_D + 1];
    S->r[0] = 1; S->r[d] = 1;
    for (int k = 1; k <= d - 1; ++k) S->r[k] = 0;
    orc_point_levels(S, S->i0, in);              /* every unfolding: the sets are empty */
    orc_append_point(S, S->i0, in);
    for (int s = 0; s < S->nseed; ++s) {
        if (orc_point_levels(S, S->seeds[s], in) < 0) return ORC_EINVAL;
        orc_append_point(S, S->seeds[s], in);
    }
    for (int k = 1; k <= d - 1; ++k) {
        int st = orc_pivot_residuals(S, k, S->piv[k]);
        if (st) return st;
    }
    return ORC_OK;
}

/* Residual of point pt, as the next pivot, in each unfolding it enters
 * (res[k]; in[k] marks them).  Returns how many it enters (-1: see
 * orc_point_levels).  The sets are left as they were. */
static int orc_point_residuals(orc_state *S, const int *pt, int *in, double *res)
{
    int d = S->d, rsave[ORC_MAX_D + 1];
    int cnt = orc_point_levels(S, pt, in);
    if (cnt <= 0) return cnt;
    for (int k = 0; k <= d; ++k) rsave[k] = S->r[k];
    orc_append_point(S, pt, in);
    double *pv = (double *)malloc(sizeof(double) * S->r_max);
    for (int k = 1; k <= d - 1; ++k) {
        res[k] = 0.0;
        if (!in[k] || !pv) continue;
        if (orc_pivot_residuals(S, k, pv) == ORC_OK) res[k] = fabs(pv[S->r[k] - 1]);
    }
    free(pv);
    for (int k = 0; k <= d; ++k) S->r[k] = rsave[k];
    return cnt;
}

/* The point a sample contributes to the initial list, in q: the sample
 * itself if its residual is larger than tau in every unfolding it enters;
 * else, trimmed to the longest run of consecutive such unfoldings (the first
 * on ties) k_c..k_d, the point that takes i0's indices before position k_c
 * and after position k_d + 1 (1-based: modes 1..k_c-1 and k_d+2..d), whose
 * prefix at k_c - 1 and suffix at k_d + 1 are i0's and hence present, if
 * that point passes the same test.  Returns 1 if there is such a point. */
static int orc_point_pick(orc_state *S, const int *pt, int *q)
{
    int d = S->d, in[ORC_MAX_D + 1];
    double res[ORC_MAX_D + 1];
    int cnt = orc_point_residuals(S, pt, in, res);
    if (cnt <= 0) return 0;
    int all = 1, kc = -1, kd = -1, run0 = -1;
    for (int k = 1; k <= d - 1; ++k) {
        if (!in[k]) continue;
        if (res[k] > S->tau) {
            if (run0 < 0) run0 = k;
            if (kc < 0 || k - run0 > kd - kc) { kc = run0; kd = k; }
        } else {
            all = 0;
            run0 = -1;
        }
    }
    if (all) {
        for (int j = 0; j < d; ++j) q[j] = pt[j];
        return 1;
    }
    if (kc < 0) return 0;
    for (int j = 0; j < d; ++j) q[j] = (j < kc - 1 || j > kd) ? S->i0[j] : pt[j];
    cnt = orc_point_residuals(S, q, in, res);
    if (cnt <= 0) return 0;
    for (int k = 1; k <= d - 1; ++k)
        if (in[k] && !(res[k] > S->tau)) return 0;
    return 1;
}

static double orc_tt_value(int d, const int *n, const int *ranks, const double *cores, const int *idx,
                           double *v, double *vn);

/* The sampled-error check on the R multi-indices idx (R x d): out[t] =
 * |X - X~| at sample t and *err the relative error, sums in sample order. */
static int orc_sample_errors(const orc_state *S, int64_t R, const int *idx, double *out, double *err)
{
    int d = S->d, rmax = 1;
    for (int k = 0; k <= d; ++k) if (S->r[k] > rmax) rmax = S->r[k];
    double *v = (double *)malloc(sizeof(double) * rmax);
    double *vn = (double *)malloc(sizeof(double) * rmax);
    if (!v || !vn) { free(v); free(vn); return ORC_ENOMEM; }
    double num = 0.0, den = 0.0;
    for (int64_t t = 0; t < R; ++t) {
        double x = orc_eval(&S->F, idx + t * d);
        double y = orc_tt_value(d, S->n, S->r, S->cores, idx + t * d, v, vn);
        num += (x - y) * (x - y);
        den += x * x;
        out[t] = fabs(x - y);
    }
    free(v); free(vn);
    *err = den > 0.0 ? sqrt(num / den) : sqrt(num);
    return ORC_OK;
}

/* order = 0..R-1 sorted by decreasing key, lower index first among equal
 * keys (a stable merge sort). */
static void orc_order_by_error(const double *key, int64_t R, int64_t *order)
{
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    for (int64_t t = 0; t < R; ++t) order[t] = t;
    if (!tmp) {                                   /* insertion sort without scratch */
        for (int64_t i = 1; i < R; ++i) {
            int64_t x = order[i], j = i;
            while (j > 0 && key[order[j - 1]] < key[x]) { order[j] = order[j - 1]; --j; }
            order[j] = x;
        }
        return;
    }
    for (int64_t w = 1; w < R; w *= 2) {
        for (int64_t lo = 0; lo < R; lo += 2 * w) {
            int64_t mid = lo + w < R ? lo + w : R, hi = lo + 2 * w < R ? lo + 2 * w : R;
            int64_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi) tmp[o++] = (key[order[b]] > key[order[a]]) ? order[b++] : order[a++];
            while (a < mid) tmp[o++] = order[a++];
            while (b < hi) tmp[o++] = order[b++];
        }
        memcpy(order, tmp, sizeof(int64_t) * (size_t)R);
    }
    free(tmp);
}

/* Restarts after false convergence (see the header): at most max_restarts
 * (<= ORC_MAX_SEEDS) restarts decided by R check samples; 0 turns them off. */
int orc_set_restarts(orc_state *S, int max_restarts, int64_t R)
{
    if (!S || max_restarts < 0 || max_restarts > ORC_MAX_SEEDS || (max_restarts > 0 && R < 1)) return ORC_EINVAL;
    S->max_restarts = max_restarts;
    S->restart_R = R;
    return ORC_OK;
}

/* out: [restarts used, cause, seeds], err: the last check's error (-1 if
 * none), pts: the seeds (restarts used x d). */
int orc_get_restarts(const orc_state *S, int *out, double *err, int *pts)
{
    if (!S) return ORC_EINVAL;
    out[0] = S->restarts_used;
    out[1] = S->restart_cause;
    out[2] = S->nseed;
    *err = S->sampled_err;
    if (pts)
        for (int s = 0; s < S->nseed; ++s)
            for (int j = 0; j < S->d; ++j) pts[s * S->d + j] = S->seeds[s][j];
    return ORC_OK;
}

static int orc_solve(orc_state *S);

int orc_run(orc_state *S)
{
    if (!S) return ORC_EINVAL;
    if (S->ran) return S->status;
    int d = S->d;
    /* samples: rms for the stop threshold and the initial pivot */
    int *sidx = (int *)malloc(sizeof(int) * (size_t)S->n_samples * d);
    if (!sidx) return S->status = ORC_ENOMEM;
    orc_sample_indices(d, S->n, S->seed, S->n_samples, sidx);
    double *sval = (double *)malloc(sizeof(double) * (size_t)S->n_samples);
    if (!sval) { free(sidx); return S->status = ORC_ENOMEM; }
    double bestv = -1.0;
    int64_t bests = 0;
    for (int64_t s = 0; s < S->n_samples; ++s) {
        double v = orc_eval(&S->F, sidx + s * d);
        if (!isfinite(v)) { free(sidx); free(sval); return S->status = ORC_EFN; }
        sval[s] = v;
        if (fabs(v) > bestv) { bestv = fabs(v); bests = s; }
    }
    double sumsq = orc_pairwise_sumsq(sval, S->n_samples);
    free(sval);
    S->rms = sqrt(sumsq / (double)S->n_samples);
    S->tau = S->eps * S->rms;
    for (int j = 0; j < d; ++j) S->i0[j] = sidx[bests * d + j];
    free(sidx);
    double p0 = orc_eval(&S->F, S->i0);
    if (p0 == 0.0) return S->status = ORC_ESINGULAR;


    S->nseed = 0;
    S->restarts_used = 0;
    S->restart_cause = 0;
    S->sampled_err = -1.0;
    int st = orc_solve(S);
    if (st < 0 || S->max_restarts <= 0) return st;
    /* restarts after false convergence */
    int64_t R = S->restart_R;
    int *ridx = (int *)malloc(sizeof(int) * (size_t)R * d);
    double *rerr = (double *)malloc(sizeof(double) * (size_t)R);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    if (!ridx || !rerr || !order) { free(ridx); free(rerr); free(order); return S->status = ORC_ENOMEM; }
    orc_sample_indices(d, S->n, S->seed + 1, R, ridx);
    while (S->status == ORC_OK) {
        double err = 0.0;
        if (orc_sample_errors(S, R, ridx, rerr, &err) != ORC_OK) { S->status = ORC_ENOMEM; break; }
        S->sampled_err = err;
        if (err <= S->eps) break;
        if (S->restarts_used >= S->max_restarts || S->nseed >= ORC_MAX_SEEDS) {
            S->status = ORC_WARN_SAMPLED_ERR;
            S->restart_cause = 1;
            break;
        }
        orc_order_by_error(rerr, R, order);
        int picked = 0;
        for (int64_t t = 0; t < R && t < ORC_RESTART_TRIES && !picked; ++t)
            picked = orc_point_pick(S, ridx + order[t] * d, S->seeds[S->nseed]);
        if (!picked) {
            S->status = ORC_WARN_SAMPLED_ERR;
            S->restart_cause = 2;
            break;
        }
        S->nseed++;
        S->restarts_used++;
        st = orc_solve(S);
        if (st < 0) break;
    }
    free(ridx); free(rerr); free(order);
    return S->status;
}

/* One run from the initial list: sweeps until the stop test, then the cores. */
static int orc_solve(orc_state *S)
{
    int d = S->d;
    int st0 = orc_init_sets(S);
    if (st0) return S->status = st0;
    S->sweeps = 0;
    S->pivoted = 0;
    S->ran = 0;
    free(S->cores);
    S->cores = NULL;
    S->min_rel_gap = INFINITY;
    S->status = ORC_OK;

    int rs[ORC_MAX_D + 1];
    int64_t prow[ORC_MAX_D + 1], pcol[ORC_MAX_D + 1];
    double pval[ORC_MAX_D + 1];
    int prop[ORC_MAX_D + 1];
    for (;;) {
        for (int k = 0; k <= d; ++k) rs[k] = S->r[k];      /* sweep snapshot */
        int any = 0, capped = 0;
        S->evaluated = 0;
        for (int k = 1; k <= d - 1; ++k) {
            int64_t br, bc;
            double bv = 0.0, runner = 0.0;
            S->evaluated += (int64_t)rs[k - 1] * S->n[k - 1] * (int64_t)S->n[k] * rs[k + 1];
            int found = orc_search(S, k, rs, &br, &bc, &bv, &runner);
            if (found < 0) return S->status;
            prop[k] = 0;
            double a = found ? fabs(bv) : 0.0;
            if (S->sweeps < S->hist_cap) {
                S->best_hist[k][S->sweeps] = a;
                S->gap_hist[k][S->sweeps] = (found && a > 0.0 && !S->rook) ? (a - runner) / a : 1.0;
            }
            if (found && a > S->tau) {
                if (a > 0.0 && !S->rook) {
                    double g = (a - runner) / a;
                    if (g < S->min_rel_gap) S->min_rel_gap = g;
                }
                if (rs[k] < S->kcap[k]) {
                    prop[k] = 1; prow[k] = br; pcol[k] = bc; pval[k] = bv; any = 1;
                } else {
                    capped = 1;
                }
            }
        }
        S->sweeps++;
        if (capped) S->status = ORC_NOT_CONVERGED;
        if (!any) break;
        /* commit all proposals (append-only, so positions stay valid) */
        for (int k = 1; k <= d - 1; ++k) {
            if (!prop[k]) continue;
            int z = S->r[k];
            int nk = S->n[k - 1], nk1 = S->n[k];
            int64_t p = prow[k] / nk, q = pcol[k] / nk1;
            for (int j = 0; j < k - 1; ++j) S->I[k][z * k + j] = S->I[k - 1][p * (k - 1) + j];
            S->I[k][z * k + k - 1] = (int)(prow[k] % nk);
            int sl = d - k - 1;
            S->J[k][z * (d - k)] = (int)(pcol[k] % nk1);
            for (int j = 0; j < sl; ++j) S->J[k][z * (d - k) + 1 + j] = S->J[k + 1][q * sl + j];
            S->rho[k][z] = prow[k];
            S->gam[k][z] = pcol[k];
            S->piv[k][z] = pval[k];
            S->r[k] = z + 1;
        }
    }
    if (!isfinite(S->min_rel_gap)) S->min_rel_gap = 1.0;
    S->ran = 1;

    /* cores by Alg. 4 on the sliced fibers */
    int64_t total = 0;
    for (int k = 1; k <= d; ++k) total += (int64_t)S->r[k - 1] * S->n[k - 1] * S->r[k];
    S->cores = (double *)malloc(sizeof(double) * total);
    if (!S->cores) return S->status = ORC_ENOMEM;
    S->cores_len = total;
    int64_t off = 0;
    int idx[ORC_MAX_D];
    for (int k = 1; k <= d - 1; ++k) {
        int64_t nrow = (int64_t)S->r[k - 1] * S->n[k - 1];
        int rk = S->r[k];
        double *A = (double *)malloc(sizeof(double) * nrow * rk);
        double *Trho = (double *)malloc(sizeof(double) * rk);
        double *a = (double *)malloc(sizeof(double) * rk);
        double *s = (double *)malloc(sizeof(double) * nrow);
        double *T = S->cores + off;
        if (!A || !Trho || !a || !s) {
            free(A); free(Trho); free(a); free(s);
            return S->status = ORC_ENOMEM;
        }
        /* A = X(I_{<=k-1} x [n_k], J_{>k}); column z is the z-th column tuple */
        for (int64_t i = 0; i < nrow; ++i) {
            int64_t p = i / S->n[k - 1];
            for (int z = 0; z < rk; ++z) {
                for (int j = 0; j < k - 1; ++j) idx[j] = S->I[k - 1][p * (k - 1) + j];
                idx[k - 1] = (int)(i % S->n[k - 1]);
                for (int j = 0; j < d - k; ++j) idx[k + j] = S->J[k][z * (d - k) + j];
                A[i * rk + z] = orc_eval(&S->F, idx);
            }
        }
        /* T_1 = A(:, j_1) / A(i_1, j_1) */
        double a11 = A[S->rho[k][0] * rk + 0];
        for (int64_t i = 0; i < nrow; ++i) {
            for (int z = 0; z < rk; ++z) T[i * rk + z] = 0.0;
            T[i * rk + 0] = A[i * rk + 0] / a11;
        }
        for (int z = 1; z < rk; ++z) {
            int64_t iz = S->rho[k][z];
            for (int zz = 0; zz < z; ++zz) a[zz] = A[S->rho[k][zz] * rk + z];   /* A(I_z, j_z) */
            /* s = T A(I_z, j_z) - A(:, j_z), dot products in ascending order */
            for (int64_t i = 0; i < nrow; ++i) {
                double dot = 0.0;
                for (int zz = 0; zz < z; ++zz) dot = fma(T[i * rk + zz], a[zz], dot);
                s[i] = dot - A[i * rk + z];
            }
            /* delta^{-1} = A(i_z, j_z) - T(i_z,:) A(I_z, j_z) = -s(i_z) */
            double dinv = -s[iz];
            if (dinv == 0.0) {
                free(A); free(Trho); free(a); free(s);
                return S->status = ORC_ESINGULAR;
            }
            double delta = 1.0 / dinv;
            for (int zz = 0; zz < z; ++zz) Trho[zz] = T[iz * rk + zz];
            /* T = [T + delta s T(i_z,:), -delta s] */
            for (int64_t i = 0; i < nrow; ++i) {
                double c = delta * s[i];
                for (int zz = 0; zz < z; ++zz) T[i * rk + zz] = fma(c, Trho[zz], T[i * rk + zz]);
                T[i * rk + z] = -c;
            }
        }
        free(A); free(Trho); free(a); free(s);
        off += nrow * rk;
    }
    /* G_d = X(I_{<=d-1}, :) */
    {
        int rd = S->r[d - 1];
        for (int p = 0; p < rd; ++p)
            for (int i = 0; i < S->n[d - 1]; ++i) {
                for (int j = 0; j < d - 1; ++j) idx[j] = S->I[d - 1][p * (d - 1) + j];
                idx[d - 1] = i;
                S->cores[off + (int64_t)p * S->n[d - 1] + i] = orc_eval(&S->F, idx);
            }
    }
    return S->status;
}

/* ------------------------------------------------------------------------ */
/* Accessors.                                                                 */
/* ------------------------------------------------------------------------ */
int orc_get_ranks(const orc_state *S, int *ranks)
{
    if (!S || !S->ran) return ORC_EINVAL;
    for (int k = 0; k <= S->d; ++k) ranks[k] = S->r[k];
    return ORC_OK;
}

/* rows: r_k x k tuples, cols: r_k x (d-k) tuples, rho/gam: superblock
 * positions, piv: pivot residuals; any output may be NULL. */
int orc_get_pivots(const orc_state *S, int k, int *rows, int *cols, int64_t *rho, int64_t *gam,
                   double *piv)
{
    if (!S || !S->ran || k < 1 || k > S->d - 1) return ORC_EINVAL;
    int rk = S->r[k];
    if (rows) memcpy(rows, S->I[k], sizeof(int) * rk * k);
    if (cols) memcpy(cols, S->J[k], sizeof(int) * rk * (S->d - k));
    if (rho) memcpy(rho, S->rho[k], sizeof(int64_t) * rk);
    if (gam) memcpy(gam, S->gam[k], sizeof(int64_t) * rk);
    if (piv) memcpy(piv, S->piv[k], sizeof(double) * rk);
    return rk;
}

/* stats: [rms, tau, evaluated, pivoted, sweeps, min_rel_gap, status] */
int orc_get_stats(const orc_state *S, double *out, int *i0)
{
    if (!S || !S->ran) return ORC_EINVAL;
    out[0] = S->rms; out[1] = S->tau; out[2] = (double)S->evaluated; out[3] = (double)S->pivoted;
    out[4] = S->sweeps; out[5] = S->min_rel_gap; out[6] = S->status;
    if (i0) for (int j = 0; j < S->d; ++j) i0[j] = S->i0[j];
    return ORC_OK;
}

/* Per sweep of unfolding k: the relative gap (best - runner-up) / best
 * between the largest unmasked |residual| and the largest one not bitwise
 * equal to it (greedy search; 1 when there is none).  A pivot decided by a
 * gap at the level of rounding may legitimately differ in an arithmetic
 * whose last bits differ (another exp). */
int orc_get_gap_history(const orc_state *S, int k, double *out, int cap)
{
    if (!S || !S->ran || k < 1 || k > S->d - 1) return ORC_EINVAL;
    int m = S->sweeps < cap ? S->sweeps : cap;
    if (m > S->hist_cap) m = S->hist_cap;
    memcpy(out, S->gap_hist[k], sizeof(double) * m);
    return m;
}

/* Most rounds of Alg. 1's loop that any block search of the last run took
 * (rook mode; 0 otherwise). */
int orc_get_rook_rounds(const orc_state *S)
{
    if (!S || !S->ran) return ORC_EINVAL;
    return S->rook_max_rounds;
}

/* best |residual| of unfolding k in each sweep */
int orc_get_history(const orc_state *S, int k, double *out, int cap)
{
    if (!S || !S->ran || k < 1 || k > S->d - 1) return ORC_EINVAL;
    int m = S->sweeps < cap ? S->sweeps : cap;
    if (m > S->hist_cap) m = S->hist_cap;
    memcpy(out, S->best_hist[k], sizeof(double) * m);
    return m;
}

int64_t orc_get_cores(const orc_state *S, double *out, int64_t cap)
{
    if (!S || !S->ran || !S->cores) return ORC_EINVAL;
    if (out) {
        if (cap < S->cores_len) return ORC_EINVAL;
        memcpy(out, S->cores, sizeof(double) * S->cores_len);
    }
    return S->cores_len;
}

/* Value of the TT at a multi-index: G_1(i_1) G_2(i_2) ... G_d(i_d), each
 * product accumulated in ascending order of the contracted index. */
static double orc_tt_value(int d, const int *n, const int *ranks, const double *cores, const int *idx,
                           double *v, double *vn)
{
    int64_t off = 0;
    v[0] = 1.0;
    for (int k = 0; k < d; ++k) {
        int ra = ranks[k], rb = ranks[k + 1];
        const double *G = cores + off;                    /* ra x n_k x rb */
        for (int b = 0; b < rb; ++b) {
            double acc = 0.0;
            for (int a = 0; a < ra; ++a)
                acc = fma(v[a], G[((int64_t)a * n[k] + idx[k]) * rb + b], acc);
            vn[b] = acc;
        }
        for (int b = 0; b < rb; ++b) v[b] = vn[b];
        off += (int64_t)ra * n[k] * rb;
    }
    return v[0];
}

int orc_tt_eval(int d, const int *n, const int *ranks, const double *cores, int64_t m, const int *idx,
                double *out)
{
    int rmax = 1;
    for (int k = 0; k <= d; ++k) if (ranks[k] > rmax) rmax = ranks[k];
    double *v = (double *)malloc(sizeof(double) * rmax);
    double *vn = (double *)malloc(sizeof(double) * rmax);
    if (!v || !vn) { free(v); free(vn); return ORC_ENOMEM; }
    for (int64_t t = 0; t < m; ++t) out[t] = orc_tt_value(d, n, ranks, cores, idx + t * d, v, vn);
    free(v); free(vn);
    return ORC_OK;
}

int orc_state_tt_eval(const orc_state *S, int64_t m, const int *idx, double *out)
{
    if (!S || !S->ran) return ORC_EINVAL;
    return orc_tt_eval(S->d, S->n, S->r, S->cores, m, idx, out);
}

/* Sampled relative error of Sec. 5 on R seeded indices (stream seed): the
 * square root of sum (X - X~)^2 / sum X^2, sums in sample order. */
int orc_sampled_error(const orc_state *S, int64_t R, uint64_t seed, double *err)
{
    if (!S || !S->ran) return ORC_EINVAL;
    int d = S->d;
    int idx[ORC_MAX_D];
    int rmax = 1;
    for (int k = 0; k <= d; ++k) if (S->r[k] > rmax) rmax = S->r[k];
    double *v = (double *)malloc(sizeof(double) * rmax);
    double *vn = (double *)malloc(sizeof(double) * rmax);
    if (!v || !vn) { free(v); free(vn); return ORC_ENOMEM; }
    uint64_t st = seed;
    double num = 0.0, den = 0.0;
    for (int64_t t = 0; t < R; ++t) {
        for (int j = 0; j < d; ++j) idx[j] = (int)(orc_sm64(&st) % (uint64_t)S->n[j]);
        double x = orc_eval(&S->F, idx);
        double y = orc_tt_value(d, S->n, S->r, S->cores, idx, v, vn);
        num += (x - y) * (x - y);
        den += x * x;
    }
    free(v); free(vn);
    *err = den > 0.0 ? sqrt(num / den) : sqrt(num);
    return ORC_OK;
}

/* The final guard of a run: the sampled relative error (Sec. 5) over R
 * indices of the independent stream seed + 1.  A run that stopped with
 * every superblock residual at or below tau (status ORC_OK) but whose
 * sampled error exceeds eps has converged falsely; its status becomes
 * ORC_WARN_SAMPLED_ERR.  Returns the status; *err receives the error. */
int orc_verify(orc_state *S, int64_t R, double *err)
{
    if (!S || !S->ran || R < 1) return ORC_EINVAL;
    int st = orc_sampled_error(S, R, S->seed + 1, err);
    if (st) return st;
    if (*err > S->eps && S->status == ORC_OK) S->status = ORC_WARN_SAMPLED_ERR;
    return S->status;
}

/* Brute force over every entry (eq. FrobeniusNorm); tiny tensors only. */
int orc_full_error(const orc_state *S, double *err, double *max_abs_err)
{
    if (!S || !S->ran) return ORC_EINVAL;
    int d = S->d;
    int64_t N = 1;
    for (int j = 0; j < d; ++j) N *= S->n[j];
    if (N > (int64_t)200000000) return ORC_EINVAL;
    int idx[ORC_MAX_D] = {0};
    int rmax = 1;
    for (int k = 0; k <= d; ++k) if (S->r[k] > rmax) rmax = S->r[k];
    double *v = (double *)malloc(sizeof(double) * rmax);
    double *vn = (double *)malloc(sizeof(double) * rmax);
    if (!v || !vn) { free(v); free(vn); return ORC_ENOMEM; }
    double num = 0.0, den = 0.0, mx = 0.0;
    for (int64_t t = 0; t < N; ++t) {
        double x = orc_eval(&S->F, idx);
        double y = orc_tt_value(d, S->n, S->r, S->cores, idx, v, vn);
        num += (x - y) * (x - y);
        den += x * x;
        if (fabs(x - y) > mx) mx = fabs(x - y);
        for (int j = d - 1; j >= 0; --j) {                 /* odometer, last index fastest */
            if (++idx[j] < S->n[j]) break;
            idx[j] = 0;
        }
    }
    free(v); free(vn);
    *err = den > 0.0 ? sqrt(num / den) : sqrt(num);
    if (max_abs_err) *max_abs_err = mx;
    return ORC_OK;
}

/* Residual of superblock k after its current pivots, from the raw entries,
 * for inspection by tests (nrow x ncol, row-major).  Returns nrow*ncol. */
int64_t orc_superblock_residual(orc_state *S, int k, double *out, int64_t cap, int64_t *nrow_out,
                                int64_t *ncol_out)
{
    if (!S || !S->ran || k < 1 || k > S->d - 1) return ORC_EINVAL;
    int64_t nrow = (int64_t)S->r[k - 1] * S->n[k - 1];
    int64_t ncol = (int64_t)S->n[k] * S->r[k + 1];
    *nrow_out = nrow; *ncol_out = ncol;
    if (!out) return nrow * ncol;
    if (cap < nrow * ncol) return ORC_EINVAL;
    int idx[ORC_MAX_D];
    double *u = (double *)malloc(sizeof(double) * ncol);
    double *w = (double *)malloc(sizeof(double) * nrow);
    if (!u || !w) { free(u); free(w); return ORC_ENOMEM; }
    for (int64_t i = 0; i < nrow; ++i)
        for (int64_t j = 0; j < ncol; ++j) {
            orc_entry_index(S, k, i, j, idx);
            out[i * ncol + j] = orc_eval(&S->F, idx);
        }
    for (int z = 0; z < S->r[k]; ++z) {
        int64_t pr = S->rho[k][z], pc = S->gam[k][z];
        double p = out[pr * ncol + pc];
        for (int64_t j = 0; j < ncol; ++j) u[j] = out[pr * ncol + j] / p;
        for (int64_t i = 0; i < nrow; ++i) w[i] = out[i * ncol + pc];
        for (int64_t i = 0; i < nrow; ++i)
            for (int64_t j = 0; j < ncol; ++j) out[i * ncol + j] = fma(-w[i], u[j], out[i * ncol + j]);
    }
    free(u); free(w);
    return nrow * ncol;
}

/* Plain rank-1 recursion on a dense matrix with given pivots (d = 2 view,
 * eq. aca_approx_E in residual form): A is m x n row-major and is overwritten
 * by the residual after eliminating pivots (rows[z], cols[z]) in order. */
int orc_matrix_residual(int64_t m, int64_t n, double *A, int npiv, const int64_t *rows,
                        const int64_t *cols)
{
    double *u = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * m);
    if (!u || !w) { free(u); free(w); return ORC_ENOMEM; }
    for (int z = 0; z < npiv; ++z) {
        double p = A[rows[z] * n + cols[z]];
        if (p == 0.0) { free(u); free(w); return ORC_ESINGULAR; }
        for (int64_t j = 0; j < n; ++j) u[j] = A[rows[z] * n + j] / p;
        for (int64_t i = 0; i < m; ++i) w[i] = A[i * n + cols[z]];
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) A[i * n + j] = fma(-w[i], u[j], A[i * n + j]);
    }
    free(u); free(w);
    return ORC_OK;
}
