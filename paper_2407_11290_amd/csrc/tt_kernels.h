// tt_kernels.h -- gfx950 kernels of the greedy adaptive TT-cross hot path.
//
// One search sweep over all unfoldings is two launches:
//   k_sweep   one workgroup per tile of every superblock; a tile lies inside a
//             single subtensor block and a single prefix/suffix, and either
//             applies the newest pivot to stored residuals (rank-1 update,
//             eq. submatrix_cross_iter) or evaluates new superblock entries and
//             eliminates all pivots from them; both fuse the |residual| argmax
//             of the tile (the block-local pivot of Alg. 3);
//   k_commit  one workgroup per unfolding: best of the local pivots, stop test,
//             append to the nested index sets, extract the new pivot's row and
//             column factors.
#pragma once

#include "tt_device.h"

namespace ttc {

__device__ inline bool better(double a, uint64_t ka, double b, uint64_t kb)
{
    return a > b || (a == b && ka < kb);
}

// Workgroup-wide (max |value|, lowest key) reduction; result valid in all threads.
__device__ inline void block_best(double &v, uint64_t &key)
{
    __shared__ double sv[NT / 64];
    __shared__ uint64_t sk[NT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off, 64);
        unsigned long long ok = __shfl_xor((unsigned long long)key, off, 64);
        if (better(ov, ok, v, key)) { v = ov; key = ok; }
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) { sv[w] = v; sk[w] = key; }
    __syncthreads();
    v = sv[0]; key = sk[0];
    for (int i = 1; i < NT / 64; ++i)
        if (better(sv[i], sk[i], v, key)) { v = sv[i]; key = sk[i]; }
    __syncthreads();
}

template <typename V> __device__ inline V vfma(V a, V b, V c);
template <> __device__ inline double vfma<double>(double a, double b, double c) { return __fma_rn(a, b, c); }
template <> __device__ inline float vfma<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }

// ---------------------------------------------------------------------------
// Search tile.
// ---------------------------------------------------------------------------
template <typename V>
__device__ void sweep_tile(const ProbDev *__restrict__ P, const KDev &K, const ProbState *S, int u, int par,
                           int R, int C, int rk, double &bv, uint64_t &bk, V *sm)
{
    const int d = P->d, k = u + 1;
    const int tid = threadIdx.x;
    const int p = R / K.RTp, t = R - p * K.RTp;
    const int q = C / K.CTq, tc = C - q * K.CTq;
    const int ik0 = K.rt_start[t], nrows = K.rt_len[t];
    const int ik10 = K.ct_start[tc], ncols = K.ct_len[tc];
    const int row0 = p * K.nk + ik0, col0 = q * K.nk1 + ik10;
    const int nr_st = S->nr_st[u], nc_st = S->nc_st[u], ra = S->ra[u];
    const bool rows_old = row0 < nr_st, cols_old = col0 < nc_st;
    V *E = (V *)K.E;
    V *W = (V *)K.W;
    V *U = (V *)K.U;
    const int64_t ld = K.colcap;
    const int TCt = K.TC, rpp = NT / TCt;
    const int tr = tid / TCt, tcol = tid - tr * TCt;
    const bool colact = tcol < ncols;

    if (rows_old && cols_old) {
        // stored residuals: apply the newest pivot (if any) and search
        const bool apply = ra < rk;
        const int col = col0 + tcol;
        V ucol = 0;
        bool cm = true;
        if (colact) {
            if (apply) ucol = U[(int64_t)ra * K.colcap + col];
            cm = K.cmask[col] != 0;
        }
        const V *wz = W + (int64_t)ra * K.rowcap;
        for (int ii = tr; ii < nrows; ii += rpp) {
            if (!colact) break;
            const int row = row0 + ii;
            V *e = E + (int64_t)row * ld + col;
            V x = *e;
            if (apply) {
                x = vfma<V>(-wz[row], ucol, x);
                *e = x;
            }
            if (!cm && !K.rmask[row]) {
                double ax = (double)fabs(x);
                uint64_t key = ((uint64_t)row << 32) | (uint32_t)col;
                if (better(ax, key, bv, bk)) { bv = ax; bk = key; }
            }
        }
        return;
    }

    // new entries: X minus the interpolant, pivots eliminated in insertion order
    __shared__ int pre[TT_MAX_D], suf[TT_MAX_D];
    const int npre = k - 1, nsuf = d - k - 1;
    if (tid < npre) pre[tid] = P->kd[u - 1].Ifull[p * npre + tid];
    if (tid < nsuf) suf[tid] = P->kd[u + 1].Jfull[q * nsuf + tid];
    const int TRm = K.TR, TCm = K.TC;
    V *Wt = sm;                       // Wt[z*TRm + ii]: W of the tile rows
    V *Ut = sm + (int64_t)rk * TRm;   // Ut[z*TCm + jj]: U of the tile columns
    __syncthreads();

    // factors of the tile rows
    if (rows_old) {
        for (int e = tid; e < rk * nrows; e += NT) {
            const int z = e / nrows, ii = e - z * nrows;
            Wt[z * TRm + ii] = W[(int64_t)z * K.rowcap + row0 + ii];
        }
    } else {
        const int nj = d - k;
        for (int e = tid; e < rk * nrows; e += NT) {
            const int z = e / nrows, ii = e - z * nrows;
            int idx[TT_MAX_D];
            for (int j = 0; j < npre; ++j) idx[j] = pre[j];
            idx[k - 1] = ik0 + ii;
            for (int j = 0; j < nj; ++j) idx[k + j] = K.Jfull[z * nj + j];
            Wt[z * TRm + ii] = fn_value<V>(P->F, idx);       // X(row, gamma_z)
        }
        __syncthreads();
        for (int zp = 0; zp + 1 < rk; ++zp) {
            for (int e = tid; e < rk * nrows; e += NT) {
                const int z = e / nrows, ii = e - z * nrows;
                if (z > zp) {
                    const V g = U[(int64_t)zp * K.colcap + K.gam[z]];
                    Wt[z * TRm + ii] = vfma<V>(-Wt[zp * TRm + ii], g, Wt[z * TRm + ii]);
                }
            }
            __syncthreads();
        }
    }
    // factors of the tile columns
    if (cols_old) {
        for (int e = tid; e < rk * ncols; e += NT) {
            const int z = e / ncols, jj = e - z * ncols;
            Ut[z * TCm + jj] = U[(int64_t)z * K.colcap + col0 + jj];
        }
    } else {
        for (int e = tid; e < rk * ncols; e += NT) {
            const int z = e / ncols, jj = e - z * ncols;
            int idx[TT_MAX_D];
            for (int j = 0; j < k; ++j) idx[j] = K.Ifull[z * k + j];
            idx[k] = ik10 + jj;
            for (int j = 0; j < nsuf; ++j) idx[k + 1 + j] = suf[j];
            Ut[z * TCm + jj] = fn_value<V>(P->F, idx);       // X(rho_z, col)
        }
        __syncthreads();
        for (int zp = 0; zp < rk; ++zp) {
            const V pz = (V)K.piv[zp];
            for (int e = tid; e < rk * ncols; e += NT) {
                const int z = e / ncols, jj = e - z * ncols;
                if (z > zp) {
                    const V uu = Ut[zp * TCm + jj] / pz;
                    const V g = W[(int64_t)zp * K.rowcap + K.rho[z]];
                    Ut[z * TCm + jj] = vfma<V>(-g, uu, Ut[z * TCm + jj]);
                }
            }
            __syncthreads();
            for (int jj = tid; jj < ncols; jj += NT) Ut[zp * TCm + jj] = Ut[zp * TCm + jj] / pz;
            __syncthreads();
        }
    }
    __syncthreads();
    // publish the factors of new rows / columns (one writer per row / column)
    if (!rows_old && C == 0) {
        for (int e = tid; e < rk * nrows; e += NT) {
            const int z = e / nrows, ii = e - z * nrows;
            W[(int64_t)z * K.rowcap + row0 + ii] = Wt[z * TRm + ii];
        }
    }
    if (!cols_old && R == 0) {
        for (int e = tid; e < rk * ncols; e += NT) {
            const int z = e / ncols, jj = e - z * ncols;
            U[(int64_t)z * K.colcap + col0 + jj] = Ut[z * TCm + jj];
        }
    }
    if (!colact) return;
    const int col = col0 + tcol;
    const bool cm = K.cmask[col] != 0;
    int idx[TT_MAX_D];
    for (int j = 0; j < npre; ++j) idx[j] = pre[j];
    idx[k] = ik10 + tcol;
    for (int j = 0; j < nsuf; ++j) idx[k + 1 + j] = suf[j];
    for (int ii = tr; ii < nrows; ii += rpp) {
        const int row = row0 + ii;
        idx[k - 1] = ik0 + ii;
        V x = fn_value<V>(P->F, idx);
        for (int z = 0; z < rk; ++z) x = vfma<V>(-Wt[z * TRm + ii], Ut[z * TCm + tcol], x);
        E[(int64_t)row * ld + col] = x;
        if (!cm && !K.rmask[row]) {
            double ax = (double)fabs(x);
            uint64_t key = ((uint64_t)row << 32) | (uint32_t)col;
            if (better(ax, key, bv, bk)) { bv = ax; bk = key; }
        }
    }
}

template <typename V>
__global__ void __launch_bounds__(NT) k_sweep(const ProbDev *__restrict__ P, SweepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ProbState *S = P->S;
    if (S->stop) return;
    const int bid = blockIdx.x;
    int u = 0;
    while (u + 1 < a.nk && bid >= a.koff[u + 1]) ++u;
    const KDev &K = P->kd[u];
    const int tl = bid - a.koff[u];
    const int R = tl / a.ctub[u], C = tl - R * a.ctub[u];
    const int par = a.sweep & 1, k = u + 1;
    const int rkm1 = S->r[par][k - 1], rk = S->r[par][k], rkp1 = S->r[par][k + 1];
    double bv = -1.0;
    uint64_t bk = ~0ULL;
    if (R < rkm1 * K.RTp && C < rkp1 * K.CTq)
        sweep_tile<V>(P, K, S, u, par, R, C, rk, bv, bk, (V *)smem_raw);
    block_best(bv, bk);
    if (threadIdx.x == 0) {
        K.cand[tl].v = bv;
        K.cand[tl].key = bk;
    }
}

// ---------------------------------------------------------------------------
// FP64 value of the residual at (row, col) of superblock k, from FP64 entries
// and the FP64 pivot-block factors (used to check FP32 candidates).  Writes
// the FP64 row factors w[z] = R(row, gamma_z) before pivot z and column factors
// v[z] = R(rho_z, col) before pivot z divided by p64_z, into LDS.
// ---------------------------------------------------------------------------
__device__ inline double fp64_check(const ProbDev *P, const KDev &K, int u, int rk, int row, int col,
                                    double *w, double *v)
{
    const int d = P->d, k = u + 1, tid = threadIdx.x;
    const int nk = K.nk, nk1 = K.nk1;
    const int p = row / nk, q = col / nk1;
    const int npre = k - 1, nsuf = d - k - 1;
    const int *preI = (k >= 2) ? P->kd[u - 1].Ifull + p * npre : nullptr;
    const int *sufJ = (nsuf > 0) ? P->kd[u + 1].Jfull + q * nsuf : nullptr;
    __shared__ double xrc;
    // raw entries X(row, gamma_z), X(rho_z, col), X(row, col)
    for (int z = tid; z < rk; z += NT) {
        int idx[TT_MAX_D];
        for (int j = 0; j < npre; ++j) idx[j] = preI[j];
        idx[k - 1] = row % nk;
        for (int j = 0; j < d - k; ++j) idx[k + j] = K.Jfull[z * (d - k) + j];
        w[z] = fn_value<double>(P->F, idx);
        for (int j = 0; j < k; ++j) idx[j] = K.Ifull[z * k + j];
        idx[k] = col % nk1;
        for (int j = 0; j < nsuf; ++j) idx[k + 1 + j] = sufJ[j];
        v[z] = fn_value<double>(P->F, idx);
    }
    if (tid == 0) {
        int idx[TT_MAX_D];
        for (int j = 0; j < npre; ++j) idx[j] = preI[j];
        idx[k - 1] = row % nk;
        idx[k] = col % nk1;
        for (int j = 0; j < nsuf; ++j) idx[k + 1 + j] = sufJ[j];
        xrc = fn_value<double>(P->F, idx);
    }
    __syncthreads();
    const int rc = P->rcap;
    for (int zp = 0; zp + 1 < rk; ++zp) {
        for (int z = zp + 1 + tid; z < rk; z += NT) {
            w[z] = __fma_rn(-w[zp], K.Up64[zp * rc + z], w[z]);
            const double uu = v[zp] / K.piv64[zp];
            v[z] = __fma_rn(-K.Wp64[z * rc + zp], uu, v[z]);
        }
        __syncthreads();
    }
    for (int z = tid; z < rk; z += NT) v[z] = v[z] / K.piv64[z];
    __syncthreads();
    double x = xrc;
    for (int z = 0; z < rk; ++z) x = __fma_rn(-w[z], v[z], x);
    __syncthreads();
    return x;
}

template <typename V>
__global__ void __launch_bounds__(NT) k_commit(const ProbDev *__restrict__ P, SweepArgs a)
{
    ProbState *S = P->S;
    if (S->stop) return;
    const int u = blockIdx.x, k = u + 1, d = P->d, tid = threadIdx.x;
    const int par = a.sweep & 1;
    const KDev &K = P->kd[u];
    const int rkm1 = S->r[par][k - 1], rk = S->r[par][k], rkp1 = S->r[par][k + 1];
    const int nr = rkm1 * K.nk, nc = K.nk1 * rkp1;
    double bv = -1.0;
    uint64_t bk = ~0ULL;
    for (int i = tid; i < a.ntl[u]; i += NT) {
        const Cand c = K.cand[i];
        if (better(c.v, c.key, bv, bk)) { bv = c.v; bk = c.key; }
    }
    block_best(bv, bk);
    const bool found = bv >= 0.0;
    const int row = (int)(bk >> 32), col = (int)(bk & 0xffffffffULL);
    const V *E = (const V *)K.E;
    __shared__ double w64[TT_MAX_RANK], v64[TT_MAX_RANK];
    double e = found ? bv : 0.0;
    double p64 = 0.0;
    if (P->fp32 && found) {
        // FP64 check of the FP32 candidate (stop test and pivot block in FP64)
        p64 = fp64_check(P, K, u, rk, row, col, w64, v64);
        e = fabs(p64);
    }
    const bool over = found && e > S->tau;
    const bool propose = over && rk < P->r_max && rk < K.rk_cap;
    if (tid == 0) {
        if (a.sweep < P->hist_cap) K.hist[a.sweep] = e;
        S->last_best[u] = e;
        if (over && !propose) S->capped = 1;
    }
    if (propose) {
        const int z = rk;
        const V pv = E[(int64_t)row * K.colcap + col];
        const int p = row / K.nk, ik = row - p * K.nk;
        const int q = col / K.nk1, ik1 = col - q * K.nk1;
        if (tid == 0) {
            K.rho[z] = row;
            K.gam[z] = col;
            K.piv[z] = (double)pv;
            K.piv64[z] = P->fp32 ? p64 : (double)pv;
            K.rmask[row] = 1;
            K.cmask[col] = 1;
            K.Ifull[z * k + k - 1] = ik;
            K.Jfull[z * (d - k)] = ik1;
            if (pv == (V)0) S->err = TT_ESINGULAR;
        }
        if (tid < k - 1) K.Ifull[z * k + tid] = P->kd[u - 1].Ifull[p * (k - 1) + tid];
        if (tid < d - k - 1) K.Jfull[z * (d - k) + 1 + tid] = P->kd[u + 1].Jfull[q * (d - k - 1) + tid];
        if (P->fp32) {
            for (int zz = tid; zz < z; zz += NT) {
                K.Wp64[z * P->rcap + zz] = w64[zz];
                K.Up64[zz * P->rcap + z] = v64[zz];
            }
        }
        V *Uz = (V *)K.U + (int64_t)z * K.colcap;
        V *Wz = (V *)K.W + (int64_t)z * K.rowcap;
        const V *Er = E + (int64_t)row * K.colcap;
        for (int j = tid; j < nc; j += NT) Uz[j] = Er[j] / pv;
        for (int i = tid; i < nr; i += NT) Wz[i] = E[(int64_t)i * K.colcap + col];
    }
    if (tid == 0) {
        // traffic accounting of this sweep's tiles, before the stored region moves on
        const unsigned long long stored = (unsigned long long)S->nr_st[u] * (unsigned long long)S->nc_st[u];
        const unsigned long long all = (unsigned long long)nr * (unsigned long long)nc;
        const unsigned long long w = sizeof(V);
        atomicAdd(&S->alg_bytes, stored * w * (S->ra[u] < rk ? 2ull : 1ull) + (all - stored) * w);
        atomicAdd(&S->new_entries, all - stored);
        S->ra[u] = rk;
        S->nr_st[u] = nr;
        S->nc_st[u] = nc;
        S->r[par ^ 1][k] = rk + (propose ? 1 : 0);
        atomicAdd(&S->pivoted, (unsigned long long)nr * (unsigned long long)nc);
        if (propose) atomicOr(&S->any, 1);
        __threadfence();
        const unsigned int t = atomicAdd(&S->kdone, 1u);
        if (t == (unsigned)(a.nk - 1)) {
            __threadfence();
            const int any = atomicAdd(&S->any, 0);
            const int stop = (!any || S->err) ? 1 : 0;
            S->stop = stop;
            S->any = 0;
            S->kdone = 0;
            S->sweeps = a.sweep + 1;
            HostMirror *hm = P->hm;
            for (int j = 0; j <= d; ++j) hm->r[j] = S->r[par ^ 1][j];
            hm->err = S->err;
            hm->stop = stop;
            __threadfence_system();
            __hip_atomic_store(&hm->sweeps_done, a.sweep + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ---------------------------------------------------------------------------
// Setup: samples, rms, first pivot, initial superblocks.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_samples(const ProbDev *__restrict__ P, uint64_t seed, int ns,
                                                  double *vals)
{
    const int s = blockIdx.x * NT + threadIdx.x;
    if (s >= ns) return;
    const int d = P->d;
    int idx[TT_MAX_D];
    for (int j = 0; j < d; ++j)
        idx[j] = (int)(sm64_at(seed, (uint64_t)s * d + j) % (uint64_t)P->F.n[j]);
    vals[s] = fn_value<double>(P->F, idx);
}

template <typename V>
__global__ void __launch_bounds__(NT) k_setup(const ProbDev *__restrict__ P, uint64_t seed, int ns,
                                                const double *vals, double eps)
{
    ProbState *S = P->S;
    const int tid = threadIdx.x, d = P->d;
    double bv = -1.0;
    uint64_t bk = ~0ULL;
    int bad = 0;
    for (int s = tid; s < ns; s += NT) {
        const double a = fabs(vals[s]);
        if (!(a <= 1.7976931348623157e308)) bad = 1;          // not finite
        if (better(a, (uint64_t)s, bv, bk)) { bv = a; bk = (uint64_t)s; }
    }
    __shared__ int sbad;
    if (tid == 0) sbad = 0;
    __syncthreads();
    if (bad) atomicOr(&sbad, 1);
    block_best(bv, bk);
    __shared__ int i0[TT_MAX_D];
    __shared__ double p0s;
    if (tid == 0) {
        // sum of squares in sample order (the stop threshold must not depend
        // on a reduction tree)
        double ss = 0.0;
        for (int s = 0; s < ns; ++s) ss = __dadd_rn(ss, __dmul_rn(vals[s], vals[s]));
        const double rms = sqrt(ss / (double)ns);
        S->rms = rms;
        S->tau = eps * rms;
        for (int j = 0; j < d; ++j) {
            i0[j] = (int)(sm64_at(seed, bk * d + j) % (uint64_t)P->F.n[j]);
            S->i0[j] = i0[j];
        }
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j <= d; ++j) S->r[b][j] = 1;
        S->kdone = 0; S->any = 0; S->stop = 0; S->capped = 0; S->sweeps = 0; S->pivoted = 0;
        S->alg_bytes = 0; S->new_entries = 0;
        S->err = sbad ? TT_EFN : 0;
        p0s = (double)fn_value<V>(P->F, i0);
        if (p0s == 0.0) S->err = TT_ESINGULAR;
        if (S->err) S->stop = 1;
        HostMirror *hm = P->hm;
        for (int j = 0; j <= d; ++j) hm->r[j] = 1;
        hm->err = S->err;
        hm->stop = S->stop;
        __threadfence_system();
    }
    __syncthreads();
    for (int u = 0; u < P->nk; ++u) {
        const KDev &K = P->kd[u];
        const int k = u + 1;
        if (tid < k) K.Ifull[tid] = i0[tid];
        if (tid < d - k) K.Jfull[tid] = i0[k + tid];
        if (tid == 0) {
            K.rho[0] = i0[k - 1];
            K.gam[0] = i0[k];
            K.piv[0] = p0s;
            K.piv64[0] = (double)fn_value<double>(P->F, i0);
            K.rmask[i0[k - 1]] = 1;
            K.cmask[i0[k]] = 1;
            S->ra[u] = 0;
            S->nr_st[u] = K.nk;
            S->nc_st[u] = K.nk1;
        }
    }
}

// E = X on the initial superblocks (one prefix, one suffix: the first pivot's).
template <typename V>
__global__ void __launch_bounds__(NT) k_init_eval(const ProbDev *__restrict__ P)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int u = blockIdx.y, k = u + 1, d = P->d;
    const KDev &K = P->kd[u];
    const int64_t tot = (int64_t)K.nk * K.nk1;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
        const int i = (int)(e / K.nk1), j = (int)(e - (int64_t)i * K.nk1);
        int idx[TT_MAX_D];
        for (int jj = 0; jj < d; ++jj) idx[jj] = S->i0[jj];
        idx[k - 1] = i;
        idx[k] = j;
        ((V *)K.E)[(int64_t)i * K.colcap + j] = fn_value<V>(P->F, idx);
    }
}

// Row and column factors of the first pivot.
template <typename V>
__global__ void __launch_bounds__(NT) k_init_extract(const ProbDev *__restrict__ P)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int u = blockIdx.x;
    const KDev &K = P->kd[u];
    const V *E = (const V *)K.E;
    const int row = K.rho[0], col = K.gam[0];
    const V pv = E[(int64_t)row * K.colcap + col];
    for (int j = threadIdx.x; j < K.nk1; j += NT) ((V *)K.U)[j] = E[(int64_t)row * K.colcap + j] / pv;
    for (int i = threadIdx.x; i < K.nk; i += NT) ((V *)K.W)[i] = E[(int64_t)i * K.colcap + col];
}

// ---------------------------------------------------------------------------
// Cores by Alg. 4 (FP64).  A_k = X(I_{<=k-1} x [n_k], J_{>k}) is evaluated
// into a scratch buffer; the pivot rows' recursion runs once per unfolding and
// records delta_z and T(i_z, :) before step z; every other row then follows
// eq. (aca_approx_T_sub) independently.
// ---------------------------------------------------------------------------
struct CoreArgs {
    int nk;
    int ranks[TT_MAX_D + 1];
    int64_t aoff[TT_MAX_D];     // offset of A_k in the scratch
    int64_t goff[TT_MAX_D + 1]; // offset of G_k in the cores buffer
    int64_t doff[TT_MAX_D];     // offset of (delta, Trho) records per unfolding
    int rowblocks[TT_MAX_D + 1];// prefix sum of row blocks per unfolding (k_alg4_rows)
};

__global__ void __launch_bounds__(NT) k_fibers(const ProbDev *__restrict__ P, CoreArgs a, double *A,
                                                 double *G)
{
    const int u = blockIdx.y, d = P->d;
    if (u < a.nk) {
        const int k = u + 1;
        const KDev &K = P->kd[u];
        const int rk = a.ranks[k], nr = a.ranks[k - 1] * K.nk;
        const int64_t tot = (int64_t)nr * rk;
        for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
            const int i = (int)(e / rk), z = (int)(e - (int64_t)i * rk);
            const int p = i / K.nk;
            int idx[TT_MAX_D];
            for (int j = 0; j < k - 1; ++j) idx[j] = P->kd[u - 1].Ifull[p * (k - 1) + j];
            idx[k - 1] = i - p * K.nk;
            for (int j = 0; j < d - k; ++j) idx[k + j] = K.Jfull[z * (d - k) + j];
            A[a.aoff[u] + e] = fn_value<double>(P->F, idx);
        }
    } else {
        // G_d = X(I_{<=d-1}, :)
        const KDev &K = P->kd[d - 2];
        const int rd = a.ranks[d - 1], nd = P->F.n[d - 1];
        const int64_t tot = (int64_t)rd * nd;
        for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
            const int pp = (int)(e / nd), i = (int)(e - (int64_t)pp * nd);
            int idx[TT_MAX_D];
            for (int j = 0; j < d - 1; ++j) idx[j] = K.Ifull[pp * (d - 1) + j];
            idx[d - 1] = i;
            G[a.goff[d - 1] + e] = fn_value<double>(P->F, idx);
        }
    }
}

__global__ void __launch_bounds__(NT) k_alg4_pivots(const ProbDev *__restrict__ P, CoreArgs a,
                                                      const double *A, double *rec)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int u = blockIdx.x, k = u + 1, tid = threadIdx.x;
    const KDev &K = P->kd[u];
    const int rk = a.ranks[k];
    const double *Ak = A + a.aoff[u];
    double *Tp = (double *)smem_raw;            // rk x rk: T of the pivot rows
    double *s = Tp + rk * rk;                   // rk
    double *Tr = s + rk;                        // rk
    double *R = rec + a.doff[u];                // per z: delta_z then T(i_z, 0..z-1)
    const double a11 = Ak[(int64_t)K.rho[0] * rk];
    for (int e = tid; e < rk * rk; e += NT) {
        const int t = e / rk, z = e - t * rk;
        Tp[e] = (z == 0) ? Ak[(int64_t)K.rho[t] * rk] / a11 : 0.0;
    }
    __syncthreads();
    for (int z = 1; z < rk; ++z) {
        if (tid < rk) {
            const double *Arow = Ak + (int64_t)K.rho[tid] * rk;
            double dot = 0.0;
            for (int zz = 0; zz < z; ++zz) dot = __fma_rn(Tp[tid * rk + zz], Ak[(int64_t)K.rho[zz] * rk + z], dot);
            s[tid] = dot - Arow[z];
        }
        if (tid < z) Tr[tid] = Tp[z * rk + tid];
        __syncthreads();
        const double delta = 1.0 / (-s[z]);
        if (tid == 0) R[(int64_t)z * (rk + 1)] = delta;
        if (tid < z) R[(int64_t)z * (rk + 1) + 1 + tid] = Tr[tid];
        if (tid < rk) {
            const double c = delta * s[tid];
            for (int zz = 0; zz < z; ++zz) Tp[tid * rk + zz] = __fma_rn(c, Tr[zz], Tp[tid * rk + zz]);
            Tp[tid * rk + z] = -c;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT) k_alg4_rows(const ProbDev *__restrict__ P, CoreArgs a, const double *A,
                                                    const double *rec, double *G)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int bid = blockIdx.x;
    int u = 0;
    while (u + 1 < a.nk && bid >= a.rowblocks[u + 1]) ++u;
    const int k = u + 1, tid = threadIdx.x;
    const KDev &K = P->kd[u];
    const int rk = a.ranks[k], nr = a.ranks[k - 1] * K.nk;
    const double *Ak = A + a.aoff[u];
    const double *Rk = rec + a.doff[u];
    double *Ap = (double *)smem_raw;            // Ap[zz*rk + z] = A(rho_zz, z)
    for (int e = tid; e < rk * rk; e += NT) {
        const int zz = e / rk, z = e - zz * rk;
        Ap[e] = Ak[(int64_t)K.rho[zz] * rk + z];
    }
    __syncthreads();
    const int i = (bid - a.rowblocks[u]) * NT + tid;
    if (i >= nr) return;
    double *T = G + a.goff[u] + (int64_t)i * rk;
    const double *Ai = Ak + (int64_t)i * rk;
    const double a11 = Ap[0];
    T[0] = Ai[0] / a11;
    for (int z = 1; z < rk; ++z) T[z] = 0.0;
    for (int z = 1; z < rk; ++z) {
        double dot = 0.0;
        for (int zz = 0; zz < z; ++zz) dot = __fma_rn(T[zz], Ap[zz * rk + z], dot);
        const double s = dot - Ai[z];
        const double *Rz = Rk + (int64_t)z * (rk + 1);
        const double c = Rz[0] * s;
        for (int zz = 0; zz < z; ++zz) T[zz] = __fma_rn(c, Rz[1 + zz], T[zz]);
        T[z] = -c;
    }
}

// ---------------------------------------------------------------------------
// Evaluation helpers.
// ---------------------------------------------------------------------------
struct TTArgs {
    int d;
    int n[TT_MAX_D];
    int ranks[TT_MAX_D + 1];
    int64_t goff[TT_MAX_D + 1];
};

// One wavefront per multi-index; lane b accumulates entry b of the row vector.
__global__ void __launch_bounds__(NT) k_tt_eval(TTArgs a, const double *__restrict__ G, int64_t m,
                                                  const int *__restrict__ idx, double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t t = wave; t < m; t += nw) {
        const int *ix = idx + t * a.d;
        double v = (lane == 0) ? 1.0 : 0.0;
        for (int kk = 0; kk < a.d; ++kk) {
            const int ra = a.ranks[kk], rb = a.ranks[kk + 1], i = ix[kk], nn = a.n[kk];
            const double *Gk = G + a.goff[kk];
            double acc = 0.0;
            for (int aa = 0; aa < ra; ++aa) {
                const double va = __shfl(v, aa, 64);
                if (lane < rb) acc = __fma_rn(va, Gk[((int64_t)aa * nn + i) * rb + lane], acc);
            }
            v = (lane < rb) ? acc : 0.0;
        }
        if (lane == 0) out[t] = v;
    }
}

template <typename V>
__global__ void __launch_bounds__(NT) k_fn_eval(FnDev F, int64_t m, const int *__restrict__ idx,
                                                  double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (t >= m) return;
    int ix[TT_MAX_D];
    for (int j = 0; j < F.d; ++j) ix[j] = idx[t * F.d + j];
    out[t] = (double)fn_value<V>(F, ix);
}

__global__ void __launch_bounds__(NT) k_gen_idx(int d, TTArgs a, uint64_t seed, int64_t m, int *idx)
{
    const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (t >= m) return;
    for (int j = 0; j < d; ++j) idx[t * d + j] = (int)(sm64_at(seed, (uint64_t)t * d + j) % (uint64_t)a.n[j]);
}

__global__ void __launch_bounds__(NT) k_err_partial(int64_t m, const double *__restrict__ x,
                                                      const double *__restrict__ y, double *part)
{
    double num = 0.0, den = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < m; t += (int64_t)gridDim.x * NT) {
        const double dx = x[t] - y[t];
        num += dx * dx;
        den += x[t] * x[t];
    }
    for (int off = 32; off > 0; off >>= 1) {
        num += __shfl_xor(num, off, 64);
        den += __shfl_xor(den, off, 64);
    }
    __shared__ double sn[NT / 64], sd[NT / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sn[w] = num; sd[w] = den; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int i = 0; i < NT / 64; ++i) { a += sn[i]; b += sd[i]; }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

}  // namespace ttc
