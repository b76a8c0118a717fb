// tt_kernels.h -- gfx950 kernels of the greedy adaptive TT-cross hot path.
//
// Residual storage is an in-place elimination: once a row (column) of a
// superblock holds a pivot it is never updated again, so it keeps the residual
// it had just before that pivot was eliminated.  Those frozen rows and
// columns are exactly the factors of the rank-1 updates of eq.
// (submatrix_cross_iter): for pivot z at (rho_z, gamma_z) with value p_z,
//   column factor  W(i, z) = E(i, gamma_z)        (frozen column)
//   row factor     U(z, j) = E(rho_z, j) / p_z     (frozen row)
// and every other entry holds the current residual.  Entries on pivot rows or
// columns are never searched, so nothing else is needed.
//
// One search sweep over all unfoldings is two launches:
//   k_sweep   one workgroup per tile of every superblock; a tile lies inside a
//             single subtensor block and a single prefix/suffix.  A stored tile
//             applies the newest pivot (rank-1 update); a new tile evaluates
//             the generating function on its entries and eliminates every
//             pivot from them in insertion order.  Both fuse the |residual|
//             argmax of the tile (the block-local pivot of Alg. 3).
//   k_commit  one workgroup for all unfoldings: best of the local pivots
//             (Sec. 3.2.1), stop test, append to the nested index sets.
#pragma once

#include <hip/hip_ext.h>

#include <algorithm>
#include <utility>

#include "tt_device.h"

namespace ttc {

// Phase stamps of the instrumented build (TT_STAMPS): the device's constant
// 100 MHz clock at the boundaries of the search and commit phases, one
// record of STAMP_WORDS values per workgroup.  The normal build compiles
// none of it.
#ifdef TT_STAMPS
__device__ inline unsigned long long *stamp_rec(const ProbDev *P, int sweep, int blk)
{
    if (!P->stamps || sweep >= P->stamp_sweeps || blk >= P->stamp_wgs) return nullptr;
    return P->stamps + ((size_t)sweep * P->stamp_wgs + blk) * STAMP_WORDS;
}
__device__ inline unsigned long long *stamp_commit_rec(const ProbDev *P, int sweep)
{
    if (!P->stamps || sweep >= P->stamp_sweeps) return nullptr;
    return P->stamps + ((size_t)P->stamp_sweeps * P->stamp_wgs + sweep) * STAMP_WORDS;
}
#define TT_STAMP(rec, slot)                                                              \
    do {                                                                                 \
        if ((rec) && threadIdx.x == 0) (rec)[slot] = __builtin_amdgcn_s_memrealtime();   \
    } while (0)
#define TT_STAMP_ADD(rec, slot, v)                                                       \
    do {                                                                                 \
        if ((rec) && threadIdx.x == 0) (rec)[slot] += (v);                               \
    } while (0)
#else
#define TT_STAMP(rec, slot) do {} while (0)
#define TT_STAMP_ADD(rec, slot, v) do {} while (0)
#endif

__device__ inline bool better(double a, uint64_t ka, double b, uint64_t kb)
{
    return a > b || (a == b && ka < kb);
}

// A workgroup barrier that orders LDS accesses only.  __syncthreads also
// waits for every global load and store the wavefront has in flight; where
// what follows reads nothing another thread wrote to device memory, the
// stores then drain while the workgroup goes on.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A 64-bit value moved by a DPP control across the rows ROWS selects; a lane
// whose source lies outside its row (or in a row not written) keeps its own.
template <int CTRL, int ROWS> __device__ inline uint64_t dpp64(uint64_t x)
{
    const int lo = __builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(x >> 32), (int)(x >> 32), CTRL, ROWS, 0xf, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int CTRL, int ROWS> __device__ inline void best_step(double &v, uint64_t &key, double &sv)
{
    const double ov = __longlong_as_double((long long)dpp64<CTRL, ROWS>((uint64_t)__double_as_longlong(v)));
    const uint64_t ok = dpp64<CTRL, ROWS>(key);
    const double osv = __longlong_as_double((long long)dpp64<CTRL, ROWS>((uint64_t)__double_as_longlong(sv)));
    if (better(ov, ok, v, key)) { v = ov; key = ok; sv = osv; }
}

__device__ inline uint64_t read_lane64(uint64_t x, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Wavefront-wide best (max |value|, lowest key), in every lane.  The order
// is total (keys are distinct), so any reduction order gives the same
// winner: DPP row shifts by 1, 2, 4, 8 leave each 16-lane row's best in its
// lane 15, the row broadcasts of lanes 15 and 31 carry it to lane 63, and
// lane 63's value goes to every lane (register moves instead of the LDS
// round trips of a shuffle butterfly).  Every lane must be active.
__device__ inline void wave_best(double &v, uint64_t &key, double &sv)
{
    best_step<0x111, 0xf>(v, key, sv);      // row_shr:1
    best_step<0x112, 0xf>(v, key, sv);      // row_shr:2
    best_step<0x114, 0xf>(v, key, sv);      // row_shr:4
    best_step<0x118, 0xf>(v, key, sv);      // row_shr:8
    best_step<0x142, 0xa>(v, key, sv);      // row_bcast:15 into rows 1 and 3
    best_step<0x143, 0xc>(v, key, sv);      // row_bcast:31 into rows 2 and 3
    v = __longlong_as_double((long long)read_lane64((uint64_t)__double_as_longlong(v), 63));
    key = read_lane64(key, 63);
    sv = __longlong_as_double((long long)read_lane64((uint64_t)__double_as_longlong(sv), 63));
}

// Workgroup-wide (max |value|, lowest key) reduction carrying the signed
// value; the result is valid in every thread.
__device__ inline void block_best(double &v, uint64_t &key, double &sv)
{
    __shared__ double s_v[NT / 64], s_sv[NT / 64];
    __shared__ uint64_t s_k[NT / 64];
    wave_best(v, key, sv);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) { s_v[w] = v; s_k[w] = key; s_sv[w] = sv; }
    __syncthreads();
    v = s_v[0]; key = s_k[0]; sv = s_sv[0];
    for (int i = 1; i < NT / 64; ++i)
        if (better(s_v[i], s_k[i], v, key)) { v = s_v[i]; key = s_k[i]; sv = s_sv[i]; }
    __syncthreads();
}

template <typename V> __device__ inline V vfma(V a, V b, V c);
template <> __device__ inline double vfma<double>(double a, double b, double c) { return __fma_rn(a, b, c); }
template <> __device__ inline float vfma<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }

// strictly upper triangular index (zp < z)
__device__ inline int tri(int zp, int z) { return z * (z - 1) / 2 + zp; }

// Copy of a small struct of 32-bit words read through the global address space.
template <typename T> __device__ inline void load_words(T &dst, const T *src)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized struct");
    const gptr_t<const int> w = as_global((const int *)src);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) ((int *)&dst)[i] = w[i];
}

// LDS bytes of a new-entry tile: factors of the tile rows and columns and the
// two pivot-block triangles.
__host__ __device__ inline size_t sweep_lds_bytes(int rk, int TR, int TC, size_t w)
{
    return ((size_t)rk * (TR + TC) + (size_t)rk * (rk > 0 ? rk - 1 : 0)) * w;
}

// ---------------------------------------------------------------------------
// Search tiles.
// ---------------------------------------------------------------------------
struct TileGeom {
    int u, R, C;                  // unfolding, row tile, column tile
    int ik0, nrows, ik10, ncols;  // i_k / i_{k+1} ranges of the tile
    int row0, col0, p, q;         // first row / column position, prefix / suffix
};

__device__ inline TileGeom tile_geom(const KTile &K, int u, int R, int C)
{
    TileGeom g;
    g.u = u; g.R = R; g.C = C;
    g.p = R / K.RTp;
    const int t = R - g.p * K.RTp;
    g.q = C / K.CTq;
    const int tc = C - g.q * K.CTq;
    g.ik0 = K.rt_start[t]; g.nrows = K.rt_len[t];
    g.ik10 = K.ct_start[tc]; g.ncols = K.ct_len[tc];
    g.row0 = g.p * K.nk + g.ik0;
    g.col0 = g.q * K.nk1 + g.ik10;
    return g;
}

// Workgroup-wide (max |value|, lowest key) reduction whose result is valid
// in thread 0 only (one barrier).  The caller's next barrier must come
// before the shared slots are written again.
__device__ inline void block_best_t0(double &v, uint64_t &key, double &sv)
{
    __shared__ double s_v[NT / 64], s_sv[NT / 64];
    __shared__ uint64_t s_k[NT / 64];
    wave_best(v, key, sv);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0 && w > 0) { s_v[w] = v; s_k[w] = key; s_sv[w] = sv; }
    lds_barrier();
    if (threadIdx.x == 0)
        for (int i = 1; i < NT / 64; ++i)
            if (better(s_v[i], s_k[i], v, key)) { v = s_v[i]; key = s_k[i]; sv = s_sv[i]; }
}

// Stored residuals, one wavefront per tile: apply the newest pivot (if any)
// and search, in batches of B * (64 / TC) rows.  A 64-row chunk's first
// batch goes out in one round of loads with the chunk's row masks and W
// factors (and, for the first chunk, the column's mask and pivot-row entry),
// from addresses that are always valid, and nothing loaded is used before
// the round is issued: each batch costs one round trip.  A lane fetches its
// row's mask as the aligned 32-bit word holding it (the mask arrays are
// padded to whole words) and the byte is taken out after the shuffle, so
// no conversion of a loaded value stands between the loads.
template <typename V, int B>
__device__ void stored_tile_wave(const KTile &K, const KSweep &ks, const TileGeom &gv, double &bv, uint64_t &bk,
                                 double &bs)
{
    // the tile's extents are the wavefront's: scalar loop counts
    TileGeom g = gv;
    g.nrows = __builtin_amdgcn_readfirstlane(gv.nrows);
    g.ncols = __builtin_amdgcn_readfirstlane(gv.ncols);
    g.row0 = __builtin_amdgcn_readfirstlane(gv.row0);
    g.col0 = __builtin_amdgcn_readfirstlane(gv.col0);
    const int lane = threadIdx.x & 63;
    const int TC = K.TC, rpw = 64 / TC;
    const int tr = lane / TC, tcol = lane - tr * TC;
    const bool colok = tcol < g.ncols;
    const gptr_t<V> E = as_global((V *)K.E);
    const gptr_t<const uint32_t> rpiv_w = as_global((const uint32_t *)K.rpiv);
    const gptr_t<const uint8_t> cpiv = as_global((const uint8_t *)K.cpiv);
    const int64_t ld = K.ld;
    const int col = g.col0 + (colok ? tcol : 0);
    const bool apply = ks.apply != 0;
    const int64_t urow = apply ? ks.arho : g.row0;   // any valid row when nothing is applied
    const int wcol = apply ? ks.agam : col;
    const V apiv = apply ? (V)ks.apiv : (V)1;
    // chunk c0's row data: lane l holds row c0 + l's mask word and factor
    uint32_t rpl;
    V wl;
    auto chunk_loads = [&](int c0, int nch) {
        const int rrow = g.row0 + c0 + (lane < nch ? lane : 0);
        rpl = rpiv_w[rrow >> 2];
        wl = E[(int64_t)rrow * ld + wcol];
    };
    V xv[B];
    auto batch_loads = [&](int c0, int nch, int base) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int ii = base + tr + b * rpw;
            xv[b] = (ii < nch) ? E[(int64_t)(g.row0 + c0 + ii) * ld + col] : (V)0;
        }
    };
    // the column's mask and pivot-row factor, once per tile (reloading them,
    // and dividing by the pivot, in every batch cost the tall tiles of large
    // superblocks 7-10% of a solve)
    const int cp = cpiv[col];
    const V ue = E[urow * ld + col];
    int nch = min(64, g.nrows);
    chunk_loads(0, nch);
    batch_loads(0, nch, 0);
    const bool live = colok && !cp;
    const V u = apply ? ue / apiv : (V)0;
    // every lane runs the same iterations so that the shuffles see all lanes
    // (a value is used only for rows below nch, whose lanes loaded it)
    int c0 = 0, base = 0;
    while (true) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int ii = base + tr + b * rpw;
            const int row = g.row0 + c0 + ii;
            const uint32_t rw = (uint32_t)__shfl((int)rpl, ii & 63, 64);
            const int rp = (rw >> ((row & 3) * 8)) & 0xff;
            const V w = __shfl(wl, ii & 63, 64);
            if (ii < nch && live && !rp) {
                V x = xv[b];
                if (apply) {
                    x = vfma<V>(-w, u, x);
                    E[(int64_t)row * ld + col] = x;
                }
                const double ax = (double)fabs(x);
                const uint64_t key = ((uint64_t)row << 32) | (uint32_t)col;
                if (better(ax, key, bv, bk)) { bv = ax; bk = key; bs = (double)x; }
            }
        }
        base += B * rpw;
        if (base >= nch) {
            c0 += 64;
            if (c0 >= g.nrows) break;
            nch = min(64, g.nrows - c0);
            base = 0;
            chunk_loads(c0, nch);
        }
        batch_loads(c0, nch, base);
    }
}

// Value of lane n of each 16-lane row of the wavefront (DPP row broadcast:
// a register move, no LDS round trip).  Every lane of the row must be active.
template <int n> __device__ inline double row_bcast(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + n, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + n, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int n> __device__ inline float row_bcast(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + n, 0xf, 0xf, false));
}

// Inclusive prefix sum over each 16-lane row of the wavefront (DPP row
// shifts; lanes with no source add zero).  Every lane of the row must be
// active.
__device__ inline int row_scan_incl(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
    return x;
}

// Factor solves of a new-entry tile for ranks rk <= RK <= 16: a 16-lane
// group per row (column), lane z holding factor z; at step z' the finished
// factor z' reaches the lanes z > z' of its group by a row broadcast.
//   row i:    w_z = W_raw(i, z) - sum_{z'<z} w_z' U(z', gamma_z)
//   column j: e_z = X(rho_z, j) - sum_{z'<z} W(rho_z, z') e_z' / p_z'
// each sum in ascending z'.  Steps past rk - 1 change no lane below rk.
template <typename V, int... Z>
__device__ inline void row_steps(V &w, const V *Gr, int zl, bool ok, std::integer_sequence<int, Z...>)
{
    ((void)[&] {
        const V wz = row_bcast<Z>(w);
        if (ok && zl > Z) w = vfma<V>(-wz, Gr[tri(Z, zl)], w);
    }(), ...);
}
// The quotient e_z' / p_z' of a column step comes from the pivot's correctly
// rounded reciprocal r and one correction with the exact remainder:
// y = e r, q = y + r (e - p y) (two fmas).  With r = RN(1/p) this is RN(e/p),
// the same bits as the division (Markstein's construction; no inputs here
// come near the overflow or underflow range), but three dependent operations
// in the chain instead of a division's nine.
template <typename V> __device__ inline V div_by_recip(V e, V p, V r)
{
    const V y = e * r;
    return vfma<V>(vfma<V>(-p, y, e), r, y);
}
// RECIP: the quotient from the reciprocal (the kernels with registers to
// spare for the pivots and reciprocals the compiler reads ahead), else the
// division itself.
template <typename V, bool RECIP, int... Z>
__device__ inline void col_steps(V &u, const V *Gc, const V *s_piv, const V *s_rpiv, int zl, bool ok,
                                 std::integer_sequence<int, Z...>)
{
    ((void)[&] {
        const V uz = row_bcast<Z>(u);
        const V uu = RECIP ? div_by_recip<V>(uz, s_piv[Z], s_rpiv[Z]) : uz / s_piv[Z];
        if (ok && zl > Z) u = vfma<V>(-Gc[tri(Z, zl)], uu, u);
    }(), ...);
}

// The frozen values on the pivot rows and columns inside the tile get the
// finished factors: W(i, z) at (row i, gamma_z), p_z U(z, j) at (rho_z,
// column j), except on rows (columns) that hold a pivot themselves, whose
// entries there belong to the pivot block.
template <typename V, int RK, bool RECIP>
__device__ inline void solves_lg(gptr_t<V> E, int64_t ld, const TileGeom &g, V *Wt, V *Ut, const V *Gr,
                                 const V *Gc, const V *s_piv, const V *s_rpiv, const int *s_rho, const int *s_gam,
                                 int TRm, int TCm, int rk, int nrw, int ncw, const uint8_t *s_rp,
                                 const uint8_t *s_cp)
{
    const int tid = threadIdx.x, zl = tid & 15, gid = tid >> 4;
    constexpr int ngroups = NT / 16;
    using Steps = std::make_integer_sequence<int, RK - 1>;
    for (int base = 0; base < nrw; base += ngroups) {
        const int ii = base + gid;
        const bool ok = ii < nrw && zl < rk;
        V w = ok ? Wt[zl * TRm + ii] : (V)0;
        row_steps<V>(w, Gr, zl, ok, Steps{});
        if (ok) {
            Wt[zl * TRm + ii] = w;
            const int gz = s_gam[zl];
            if (!s_rp[ii] && gz >= g.col0 && gz < g.col0 + g.ncols) E[(int64_t)(g.row0 + ii) * ld + gz] = w;
        }
    }
    for (int base = 0; base < ncw; base += ngroups) {
        const int jj = base + gid;
        const bool ok = jj < ncw && zl < rk;
        V u = ok ? Ut[zl * TCm + jj] : (V)0;
        col_steps<V, RECIP>(u, Gc, s_piv, s_rpiv, zl, ok, Steps{});
        if (ok) {
            const int rz = s_rho[zl];
            if (!s_cp[jj] && rz >= g.row0 && rz < g.row0 + g.nrows) E[(int64_t)rz * ld + g.col0 + jj] = u;
            Ut[zl * TCm + jj] = u / s_piv[zl];
        }
    }
}

// New entries (rows of the newest prefix and/or columns of the newest suffix):
// the generating function minus the interpolant, every pivot eliminated in
// insertion order.  One workgroup per tile.  Factors of stored rows / columns
// come from the frozen pivot columns / rows; those of new rows / columns are
// recomputed here, one thread per row (column), in LDS:
//   row i:    e_z = X(i, gamma_z); for z' < z: e_z -= e_z' * U(z', gamma_z)   -> W(i, z)
//   column j: e_z = X(rho_z, j);   for z' < z: e_z -= W(rho_z, z') * e_z'/p_z' -> p_z U(z, j)
// and the frozen pivot columns / rows of the tile receive those values.
template <typename V, int FNS>
__device__ void new_tile(const ProbDev *__restrict__ P, const KTile &K, int u, int R, int C, const KSweep &ks,
                         double &bv, uint64_t &bk, double &bs, V *sm, unsigned long long *rec)
{
    // (values read from LDS are per-lane to the compiler; the tile's are the
    // same in every lane, and saying so keeps its branches and descriptor
    // reads scalar)
    const int d = P->d, k = u + 1, tid = threadIdx.x, rk = __builtin_amdgcn_readfirstlane(ks.rk);
    // The descriptor and the neighbours' tuple arrays are at hand; the tile's
    // place follows by arithmetic, and its extents (the tile tables) load
    // together with the staging below.
    const gptr_t<const int> Ipre = as_global(K.Ipre);
    const gptr_t<const int> Jsuf = as_global(K.Jsuf);
    const int RTp = K.RTp, CTq = K.CTq;
    const int tp = R / RTp, tt = R - tp * RTp, tq = C / CTq, ttc = C - tq * CTq;
    // row (column) blocks are whole prefixes (suffixes), so whether the tile's
    // rows (columns) were stored follows from the prefix (suffix) index alone
    const bool rows_old = __builtin_amdgcn_readfirstlane(tp * K.nk < ks.nr_st ? 1 : 0) != 0;
    const bool cols_old = __builtin_amdgcn_readfirstlane(tq * K.nk1 < ks.nc_st ? 1 : 0) != 0;
#ifdef TT_STAMPS
    if (rec && tid == 0) rec[13] = 1 + (rows_old ? 1 : 0) + (cols_old ? 2 : 0);
#endif
    TileGeom g;
    g.u = u; g.R = R; g.C = C; g.p = tp; g.q = tq;
    g.ik0 = K.rt_start[tt]; g.nrows = K.rt_len[tt];
    g.ik10 = K.ct_start[ttc]; g.ncols = K.ct_len[ttc];
    const gptr_t<V> E = as_global((V *)K.E);
    const gptr_t<const int> rho = as_global((const int *)K.rho), gam = as_global((const int *)K.gam);
    const gptr_t<const int> Ifull = as_global((const int *)K.Ifull), Jfull = as_global((const int *)K.Jfull);
    const gptr_t<const double> piv = as_global((const double *)K.piv);
    const int64_t ld = K.ld;
    __shared__ int pre[TT_MAX_D], suf[TT_MAX_D];
    __shared__ int s_rho[TT_MAX_RANK], s_gam[TT_MAX_RANK];
    __shared__ V s_piv[TT_MAX_RANK], s_rpiv[TT_MAX_RANK];   // pivots and their reciprocals
    __shared__ uint8_t s_rp[TT_TILE_ROWS_MAX], s_cp[TT_TILE_ROWS_MAX];
    const int npre = k - 1, nsuf = d - k - 1, nj = d - k;
    const int TRm = K.TR, TCm = K.TC, ntri = rk * (rk - 1) / 2;
    V *Wt = sm;                                // Wt[z*TRm+ii] = W(row, z)
    V *Ut = Wt + (int64_t)rk * TRm;            // Ut[z*TCm+jj] = U(z, col)
    V *Gr = Ut + (int64_t)rk * TCm;            // U(z', gamma_z), z' < z
    V *Gc = Gr + ntri;                         // W(rho_z, z'), z' < z
    const int TCt = K.TC, rpp = NT / TCt;
    const int tr = tid / TCt, tcol = tid - tr * TCt;
    // one round of loads: the neighbours' tuples, the pivots (rk <= NT: one
    // per thread) and, for Hilbert, the words of the pivots' tuples, every
    // value in flight before the first is stored (a store waits for its load,
    // and loads written after it would start only then)
    static_assert(TT_MAX_RANK <= NT && TT_MAX_D <= NT, "one pivot and one tuple word per thread");
    int prev = 0, sufv = 0;
    if (tid < npre) prev = Ipre[g.p * npre + tid];
    if (tid < nsuf) sufv = Jsuf[g.q * nsuf + tid];
    const bool zt = tid < rk;
    int rz = 0, gz = 0;
    double pz = 0.0;
    if (zt) {
        rz = rho[tid];
        gz = gam[tid];
        pz = piv[tid];
    }
    // Hilbert entries depend on the integer index sum only: the pivots' tuple
    // sums replace the tuples (J_{>k} for new rows, I_{<=k} for new columns)
    __shared__ long long s_is[TT_MAX_RANK], s_js[TT_MAX_RANK];
    [[maybe_unused]] long long is = 0, js = 0;
    if constexpr (FNS == TT_FN_HILBERT) {
        int wj[TT_MAX_D], wi[TT_MAX_D];
        if (zt && !rows_old) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j) wj[j] = Jfull[tid * nj + min(j, nj - 1)];
        }
        if (zt && !cols_old) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j) wi[j] = Ifull[tid * k + min(j, k - 1)];
        }
        if (zt && !rows_old) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j)
                if (j < nj) js += wj[j] + 1;
        }
        if (zt && !cols_old) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j)
                if (j < k) is += wi[j] + 1;
        }
    }
    if (tid < npre) pre[tid] = prev;
    if (tid < nsuf) suf[tid] = sufv;
    if (zt) {
        s_rho[tid] = rz;
        s_gam[tid] = gz;
        s_piv[tid] = (V)pz;
        s_rpiv[tid] = (V)1 / (V)pz;
        if constexpr (FNS == TT_FN_HILBERT) {
            s_is[tid] = is;
            s_js[tid] = js;
        }
    }
    __syncthreads();
    TT_STAMP(rec, 3);
    // the tile's positions
    g.row0 = g.p * K.nk + g.ik0;
    g.col0 = g.q * K.nk1 + g.ik10;
    // raw factors: frozen entries, or the generating function at the
    // skeleton.  One round of loads: the tile's pivot masks, the first pass
    // of the frozen factors of stored rows (columns) and of the pivot-block
    // triangle that new rows (columns) need, all in flight before the first
    // is stored; tiles with more frozen values take further passes of UL
    // loads per thread.
    static_assert(TT_TILE_ROWS_MAX <= NT, "one tile row and one tile column per thread");
    constexpr int UL = 4;
    const gptr_t<const uint8_t> rpiv = as_global((const uint8_t *)K.rpiv), cpiv = as_global((const uint8_t *)K.cpiv);
    const int nw = rk * g.nrows, nu = rk * g.ncols;
    const int tzp = tid / max(rk, 1), tz = tid - tzp * rk;  // the thread's triangle entry (zp, z) in the first pass
    const bool tri_ok = tid < rk * rk && tzp < tz;
    // The loads of the round do not depend on the tile's kind, so that no
    // branch separates them (a branch between loads can make the later ones
    // wait for the earlier): a value the kind does not need is read from the
    // first pivot's entry, which no search workgroup writes, and dropped.
    const int64_t spare = rk > 0 ? (int64_t)s_rho[0] * ld + s_gam[0] : 0;
    const bool use_w = rows_old && nw > 0, use_u = cols_old && nu > 0;
    const uint8_t rpb = rpiv[g.row0 + min(tid, g.nrows - 1)];
    const uint8_t cpb = cpiv[g.col0 + min(tid, g.ncols - 1)];
    V xw[UL], xu[UL];
#pragma unroll
    for (int j = 0; j < UL; ++j) {
        const int e = max(min(tid + j * NT, nw - 1), 0);
        const int z = e / g.nrows, ii = e - z * g.nrows;
        xw[j] = E[use_w ? (int64_t)(g.row0 + ii) * ld + s_gam[z] : spare];
    }
#pragma unroll
    for (int j = 0; j < UL; ++j) {
        const int e = max(min(tid + j * NT, nu - 1), 0);
        const int z = e / g.ncols, jj = e - z * g.ncols;
        xu[j] = E[use_u ? (int64_t)s_rho[z] * ld + g.col0 + jj : spare];
    }
    // pivot-block entries (rho_zp, gamma_z) and (rho_z, gamma_zp)
    const int ta = max(min(tzp, rk - 1), 0), tb = max(min(tz, rk - 1), 0);
    const V tgr = E[(int64_t)s_rho[ta] * ld + s_gam[tb]];
    const V tgc = E[(int64_t)s_rho[tb] * ld + s_gam[ta]];
    if (tid < g.nrows) s_rp[tid] = rpb;
    if (tid < g.ncols) s_cp[tid] = cpb;
    if (rows_old) {
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            const int e = tid + j * NT;
            const int z = e / g.nrows, ii = e - z * g.nrows;
            if (e < nw) Wt[z * TRm + ii] = xw[j];
        }
    } else if (tri_ok) {
        Gr[tri(tzp, tz)] = tgr / s_piv[tzp];
    }
    if (cols_old) {
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            const int e = tid + j * NT;
            const int z = e / g.ncols, jj = e - z * g.ncols;
            if (e < nu) Ut[z * TCm + jj] = xu[j] / s_piv[z];
        }
    } else if (tri_ok) {
        Gc[tri(tzp, tz)] = tgc;
    }
    if (rows_old) {
        for (int e0 = tid + UL * NT; e0 < nw; e0 += UL * NT) {
            V x[UL];
#pragma unroll
            for (int j = 0; j < UL; ++j) {
                const int e = min(e0 + j * NT, nw - 1);
                const int z = e / g.nrows, ii = e - z * g.nrows;
                x[j] = E[(int64_t)(g.row0 + ii) * ld + s_gam[z]];
            }
#pragma unroll
            for (int j = 0; j < UL; ++j) {
                const int e = e0 + j * NT;
                const int z = e / g.nrows, ii = e - z * g.nrows;
                if (e < nw) Wt[z * TRm + ii] = x[j];
            }
        }
    } else {
        for (int e = tid + NT; e < rk * rk; e += NT) {
            const int zp = e / rk, z = e - zp * rk;
            if (zp < z) Gr[tri(zp, z)] = E[(int64_t)s_rho[zp] * ld + s_gam[z]] / s_piv[zp];
        }
        if constexpr (FNS == TT_FN_HILBERT) {
            long long ps = 1;
            for (int j = 0; j < npre; ++j) ps += pre[j] + 1;
            const V sh = (V)P->F.shift;
            for (int e = tid; e < rk * g.nrows; e += NT) {
                const int z = e / g.nrows, ii = e - z * g.nrows;
                Wt[z * TRm + ii] = (V)1 / ((V)(ps + g.ik0 + ii + s_js[z]) + sh);
            }
        } else {
            for (int e = tid; e < rk * g.nrows; e += NT) {
                const int z = e / g.nrows, ii = e - z * g.nrows;
                const int ikv = g.ik0 + ii;
                const gptr_t<const int> Jz = Jfull + z * nj;
                Wt[z * TRm + ii] = fn_value_ix<V, FNS>(P->F, [&](int j) {
                    return j < npre ? pre[j] : (j == k - 1 ? ikv : Jz[j - k]);
                });
            }
        }
    }
    if (cols_old) {
        for (int e0 = tid + UL * NT; e0 < nu; e0 += UL * NT) {
            V x[UL];
#pragma unroll
            for (int j = 0; j < UL; ++j) {
                const int e = min(e0 + j * NT, nu - 1);
                const int z = e / g.ncols, jj = e - z * g.ncols;
                x[j] = E[(int64_t)s_rho[z] * ld + g.col0 + jj];
            }
#pragma unroll
            for (int j = 0; j < UL; ++j) {
                const int e = e0 + j * NT;
                const int z = e / g.ncols, jj = e - z * g.ncols;
                if (e < nu) Ut[z * TCm + jj] = x[j] / s_piv[z];
            }
        }
    } else {
        for (int e = tid + NT; e < rk * rk; e += NT) {
            const int zp = e / rk, z = e - zp * rk;
            if (zp < z) Gc[tri(zp, z)] = E[(int64_t)s_rho[z] * ld + s_gam[zp]];
        }
        if constexpr (FNS == TT_FN_HILBERT) {
            long long ss = 1;
            for (int j = 0; j < nsuf; ++j) ss += suf[j] + 1;
            const V sh = (V)P->F.shift;
            for (int e = tid; e < rk * g.ncols; e += NT) {
                const int z = e / g.ncols, jj = e - z * g.ncols;
                Ut[z * TCm + jj] = (V)1 / ((V)(s_is[z] + g.ik10 + jj + ss) + sh);
            }
        } else {
            for (int e = tid; e < rk * g.ncols; e += NT) {
                const int z = e / g.ncols, jj = e - z * g.ncols;
                const int ik1v = g.ik10 + jj;
                const gptr_t<const int> Iz = Ifull + z * k;
                Ut[z * TCm + jj] = fn_value_ix<V, FNS>(P->F, [&](int j) {
                    return j < k ? Iz[j] : (j == k ? ik1v : suf[j - k - 1]);
                });
            }
        }
    }
    __syncthreads();
    TT_STAMP(rec, 4);
    // the thread's entry column's pivot mask
    const int cpv = (tcol < g.ncols) ? s_cp[tcol] : 1;
    // chains as triangular solves; each factor sees the same operations in
    // the same order as the written recursion, so both forms give the same
    // bits.  Up to rank 16 a lane group per row (column) with row broadcasts;
    // above, one thread per row (column) runs the factors in ascending z and
    // reads the finished lower ones back from LDS (a lane group would need
    // too many passes over the tile).
    const int nrw = rows_old ? 0 : g.nrows, ncw = cols_old ? 0 : g.ncols;
    // the Hilbert kernels only: the generic FP64 kernel has no registers to
    // spare for the reciprocals, and the generic FP32 one (batches) measured
    // slower with them
    constexpr bool RECIP = FNS == TT_FN_HILBERT;
    if (rk <= 8) {
        solves_lg<V, 8, RECIP>(E, ld, g, Wt, Ut, Gr, Gc, s_piv, s_rpiv, s_rho, s_gam, TRm, TCm, rk, nrw, ncw, s_rp,
                               s_cp);
    } else if (rk <= 16) {
        solves_lg<V, 16, RECIP>(E, ld, g, Wt, Ut, Gr, Gc, s_piv, s_rpiv, s_rho, s_gam, TRm, TCm, rk, nrw, ncw, s_rp,
                                s_cp);
    } else {
        for (int e = tid; e < nrw + ncw; e += NT) {
            if (e < nrw) {
                const int ii = e;
                for (int z = 1; z < rk; ++z) {
                    V w = Wt[z * TRm + ii];
#pragma unroll 8
                    for (int zp = 0; zp < z; ++zp) w = vfma<V>(-Wt[zp * TRm + ii], Gr[tri(zp, z)], w);
                    Wt[z * TRm + ii] = w;
                }
                if (!s_rp[ii])
                    for (int z = 0; z < rk; ++z) {
                        const int gz = s_gam[z];
                        if (gz >= g.col0 && gz < g.col0 + g.ncols)
                            E[(int64_t)(g.row0 + ii) * ld + gz] = Wt[z * TRm + ii];
                    }
            } else {
                const int jj = e - nrw;
                for (int z = 0; z < rk; ++z) {
                    V u = Ut[z * TCm + jj];
                    // Ut of a lower z already holds its finished factor over its pivot
#pragma unroll 8
                    for (int zp = 0; zp < z; ++zp) u = vfma<V>(-Gc[tri(zp, z)], Ut[zp * TCm + jj], u);
                    const int rz = s_rho[z];
                    if (!s_cp[jj] && rz >= g.row0 && rz < g.row0 + g.nrows) E[(int64_t)rz * ld + g.col0 + jj] = u;
                    Ut[z * TCm + jj] = u / s_piv[z];
                }
            }
        }
    }
    lds_barrier();
    TT_STAMP(rec, 5);
    if (tcol < g.ncols && !cpv) {
        const int col = g.col0 + tcol;
        const int ik1v = g.ik10 + tcol;
        const bool hilbert = (FNS ? FNS : P->F.id) == TT_FN_HILBERT;
        long long hsum = ik1v + 1;                 // integer index sum, exact in any order
        for (int j = 0; j < npre; ++j) hsum += pre[j] + 1;
        for (int j = 0; j < nsuf; ++j) hsum += suf[j] + 1;
        // IL rows of the thread's column at once: each entry still takes
        // every pivot out in insertion order, but the IL chains interleave
        // and share each U(z, col) read
        constexpr int IL = 4;
        for (int ii0 = tr; ii0 < g.nrows; ii0 += IL * rpp) {
            V x[IL];
            int iv[IL];
            bool ok[IL];
#pragma unroll
            for (int j = 0; j < IL; ++j) {
                const int ii = ii0 + j * rpp;
                iv[j] = min(ii, g.nrows - 1);
                ok[j] = ii < g.nrows && !s_rp[iv[j]];
                const int ikv = g.ik0 + iv[j];
                if (hilbert) {
                    x[j] = (V)1 / ((V)(hsum + ikv + 1) + (V)P->F.shift);
                } else {
                    x[j] = fn_value_ix<V, FNS>(P->F, [&](int jj) {
                        return jj < npre ? pre[jj] : (jj == k - 1 ? ikv : (jj == k ? ik1v : suf[jj - k - 1]));
                    });
                }
            }
            for (int z = 0; z < rk; ++z) {
                const V uz = Ut[z * TCm + tcol];
#pragma unroll
                for (int j = 0; j < IL; ++j) x[j] = vfma<V>(-Wt[z * TRm + iv[j]], uz, x[j]);
            }
#pragma unroll
            for (int j = 0; j < IL; ++j) {
                if (!ok[j]) continue;
                const int row = g.row0 + iv[j];
                E[(int64_t)row * ld + col] = x[j];
                const double ax = (double)fabs(x[j]);
                const uint64_t key = ((uint64_t)row << 32) | (uint32_t)col;
                if (better(ax, key, bv, bk)) { bv = ax; bk = key; bs = (double)x[j]; }
            }
        }
    }
#ifdef TT_STAMPS
    if (rec && tid == 0) rec[12] = __builtin_amdgcn_s_memrealtime();
#endif
    block_best_t0(bv, bk, bs);
    TT_STAMP(rec, 6);
}




// Fixed grid striding over work units: first the new-entry tiles (one per
// workgroup), then the stored tiles four at a time (one per wavefront).
template <typename V, int FNS>
__device__ void sweep_body(const ProbDev *__restrict__ P, const ProbState *S, int nk, int blk, int nblk,
                           int sweep = -1)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
#ifdef TT_STAMPS
    const unsigned long long t_entry = __builtin_amdgcn_s_memrealtime();
    unsigned long long *rec = sweep >= 0 ? stamp_rec(P, sweep, blk) : nullptr;
    if (rec && tid == 0) rec[0] = t_entry;
#else
    unsigned long long *const rec = nullptr;
#endif
    __shared__ KSweep ks[TT_MAX_D];
    __shared__ SweepShape sh;
    // one round of loads: the stop flag, and the shapes and tile counts the
    // previous commit left (read before the flag is known, so that all of
    // them are in flight together)
    const int stop = as_global(&S->stop)[0];
    if (tid < nk) load_words(ks[tid], &S->ks[tid]);
    if (tid < SHAPE_WORDS) ((int *)&sh)[tid] = as_global((const int *)&S->sh)[tid];
    if (stop) return;                   // the same value in every thread
    __syncthreads();
    TT_STAMP(rec, 1);
    const int nnew = sh.noff[nk], nst = sh.soff[nk];
    const int units = nnew + (nst + NT / 64 - 1) / (NT / 64);
    for (int t = blk; t < units; t += nblk) {
        double bv = -1.0, bs = 0.0;
        uint64_t bk = ~0ULL;
        if (t < nnew) {
            int u = 0;
            while (u + 1 < nk && t >= sh.noff[u + 1]) ++u;
            const int idx = t - sh.noff[u], RT = sh.RT[u], CT = sh.CT[u], RTs = sh.RTs[u], CTs = sh.CTs[u];
            int R, C;
            if (idx < (RT - RTs) * CT) {
                R = RTs + idx / CT;
                C = idx % CT;
            } else {
                const int i2 = idx - (RT - RTs) * CT;
                R = i2 / (CT - CTs);
                C = CTs + i2 % (CT - CTs);
            }
            unsigned long long *nrec = nullptr;
#ifdef TT_STAMPS
            if (rec && rec[10] == 0) nrec = rec;          // the workgroup's first new tile
            TT_STAMP(nrec, 2);
#endif
            // the unit is the workgroup's: uniform
            u = __builtin_amdgcn_readfirstlane(u);
            R = __builtin_amdgcn_readfirstlane(R);
            C = __builtin_amdgcn_readfirstlane(C);
            const KTile &K = P->kt[u];
            new_tile<V, FNS>(P, K, u, R, C, ks[u], bv, bk, bs, (V *)smem_raw, nrec);
            TT_STAMP_ADD(rec, 10, 1);
            if (tid == 0) {
                const gptr_t<Cand> c = as_global(K.cand) + (R * CT + C);
                c->v = bv; c->key = bk; c->sv = bs;
            }
            lds_barrier();
        } else {
            // the wavefront index is uniform across the wavefront: saying so
            // keeps the tile's descriptor reads and geometry scalar
            const int st = (t - nnew) * (NT / 64) + __builtin_amdgcn_readfirstlane(wid);
            if (st < nst) {
                int u = 0;
                while (u + 1 < nk && st >= sh.soff[u + 1]) ++u;
                const int idx = st - sh.soff[u], CTs = sh.CTs[u];
                // the tile is the wavefront's (values read from LDS are
                // per-lane to the compiler): uniform geometry and loop counts
                u = __builtin_amdgcn_readfirstlane(u);
                const int R = __builtin_amdgcn_readfirstlane(idx / CTs);
                const int C = __builtin_amdgcn_readfirstlane(idx - R * CTs);
                const KTile &K = P->kt[u];
                const TileGeom g = tile_geom(K, u, R, C);
#ifdef TT_STAMPS
                // wave 0's first stored tile: geometry known, tile done
                const bool first_st = rec && wid == 0 && rec[11] == 0;
                if (first_st && lane == 0) rec[7] = __builtin_amdgcn_s_memrealtime();
#endif
                // 8 rows per batch of loads: more would cost occupancy
                stored_tile_wave<V, 8>(K, ks[u], g, bv, bk, bs);
                wave_best(bv, bk, bs);
                if (lane == 0) {
                    const gptr_t<Cand> c = as_global(K.cand) + (R * sh.CT[u] + C);
                    c->v = bv; c->key = bk; c->sv = bs;
                }
#ifdef TT_STAMPS
                if (first_st && lane == 0) rec[8] = __builtin_amdgcn_s_memrealtime();
                if (rec && wid == 0 && lane == 0) rec[11] += 1;
#endif
            }
        }
    }
#ifdef TT_STAMPS
    __syncthreads();
    TT_STAMP(rec, 9);
#endif
}

template <typename V, int FNS = 0>
static __global__ void __launch_bounds__(NT, 4) k_sweep(const ProbDev *__restrict__ P, SweepArgs a)
{
    sweep_body<V, FNS>(P, a.S, a.nk, blockIdx.x, gridDim.x, a.sweep);
}

// ---------------------------------------------------------------------------
// FP64 value of the residual at (row, col) of superblock k from FP64 entries
// and the FP64 factors of the pivot block (checks an FP32 candidate).  One
// wavefront; lane z ends with the FP64 row factor w = R(row, gamma_z) before
// pivot z and the column factor v = R(rho_z, col) before pivot z, over p64_z.
// ---------------------------------------------------------------------------
template <int FNS>
__device__ inline double fp64_check_wave(const ProbDev *P, const KDev &K, int u, int rk, int row, int col,
                                         double &w, double &v)
{
    const int d = P->d, k = u + 1, lane = threadIdx.x & 63;
    const int nk = K.nk, nk1 = K.nk1;
    const int p = row / nk, q = col / nk1, ik = row - p * nk, ik1 = col - q * nk1;
    const int npre = k - 1, nsuf = d - k - 1, nj = d - k;
    const gptr_t<const int> preI = as_global((const int *)((k >= 2) ? P->kd[u - 1].Ifull + p * npre : nullptr));
    const gptr_t<const int> sufJ = as_global((const int *)((nsuf > 0) ? P->kd[u + 1].Jfull + q * nsuf : nullptr));
    w = 0.0;
    v = 0.0;
    if (lane < rk) {
        const gptr_t<const int> Jz = as_global((const int *)K.Jfull) + lane * nj;
        const gptr_t<const int> Iz = as_global((const int *)K.Ifull) + lane * k;
        w = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < npre ? preI[j] : (j == k - 1 ? ik : Jz[j - k]); });
        v = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < k ? Iz[j] : (j == k ? ik1 : sufJ[j - k - 1]); });
    }
    const double xrc = fn_value_ix<double, FNS>(P->F, [&](int j) {
        return j < npre ? preI[j] : (j == k - 1 ? ik : (j == k ? ik1 : sufJ[j - k - 1]));
    });
    const int rc = P->rcap;
    for (int zp = 0; zp + 1 < rk; ++zp) {
        const double wzp = __shfl(w, zp, 64);
        const double uu = __shfl(v, zp, 64) / as_global((const double *)K.piv64)[zp];
        if (lane > zp && lane < rk) {
            w = __fma_rn(-wzp, as_global((const double *)K.Up64)[zp * rc + lane], w);
            v = __fma_rn(-as_global((const double *)K.Wp64)[lane * rc + zp], uu, v);
        }
    }
    if (lane < rk) v = v / as_global((const double *)K.piv64)[lane];
    double x = xrc;
    for (int z = 0; z < rk; ++z) x = __fma_rn(-__shfl(w, z, 64), __shfl(v, z, 64), x);
    return x;
}

// The commit, one workgroup of NTC threads for every unfolding: wavefronts
// reduce the tile candidates (best of the local pivots, Sec. 3.2.1), a
// wavefront per unfolding decides and commits it, and thread 0 publishes the
// outcome.  (A commit placed in the search launch's last workgroup would need
// every search workgroup to make its candidates visible device-wide before it
// counts itself; on gfx950 that release writes back the whole L2 of the
// workgroup's XCD, full of residual updates, and the search then ran about
// three times slower.)
constexpr int NTC = 512;
constexpr int CB = 8;              // candidates per lane in one round of loads

// The state a commit reads before it starts: this sweep's shapes and tile
// counts, the committed ranks, the threshold and the counters, and the
// unfoldings' descriptors.
struct CommitIn {
    KSweep ks[TT_MAX_D];
    int ntl[TT_MAX_D];               // tiles (rook: blocks) each unfolding searched
    int rold[TT_MAX_D + 1];
    int stop;
    int err;                         // the state's error code, kept current here
    double tau;
    unsigned long long acc[3];       // alg_bytes, new_entries, pivoted
    KDev kd[TT_MAX_D];
    // the problem's fields the commit reads later, read up front
    int rook, r_max, fp32, rcap, hist_cap;
    HostMirror *hm;
};

// A candidate that loses every comparison.
__device__ inline void cand_none(Cand &c)
{
    c.v = -1.0; c.key = ~0ULL; c.sv = 0.0;
}

// Best candidate of tiles [i0, ntl) taken by lane l of wavefront sl of wpu:
// indices i0 + l + 64 * wpu * j, CB per round of loads.
__device__ inline void scan_cands(gptr_t<const Cand> cand, int i0, int ntl, int wpu, double &bv, uint64_t &bk,
                                  double &bs)
{
    const int lane = threadIdx.x & 63;
    for (; i0 < ntl; i0 += 64 * wpu * CB) {
        Cand c[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int i = i0 + lane + 64 * wpu * j;
            if (i < ntl) {
                const gptr_t<const Cand> cp = cand + i;
                c[j].v = cp->v; c[j].key = cp->key; c[j].sv = cp->sv;
            } else {
                cand_none(c[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < CB; ++j)
            if (better(c[j].v, c[j].key, bv, bk)) { bv = c[j].v; bk = c[j].key; bs = c[j].sv; }
    }
}

// PRE (single problems): a holds each unfolding's candidate array and a
// bound on its tile count, so that the first round of candidates is in
// flight with the state; batches pass PRE = false and a is not read.
template <typename V, int FNS, bool PRE>
__device__ void commit_body(const ProbDev *__restrict__ P, ProbState *S, int sweep, int nk, const SweepArgs &a)
{
    // the wavefront index is uniform across the wavefront: saying so keeps the
    // per-unfolding reads scalar
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    constexpr int NW = NTC / 64;
    const int d = nk + 1, par = sweep & 1;    // nk from the launch: no dependent read
#ifdef TT_STAMPS
    const unsigned long long t_entry = __builtin_amdgcn_s_memrealtime();
    unsigned long long *rec = stamp_commit_rec(P, sweep);
    if (rec && tid == 0) rec[0] = t_entry;
#else
    unsigned long long *const rec = nullptr;
#endif
    // wpu >= 1 wavefronts per unfolding, the groups of wpu wavefronts
    // striding over the unfoldings (one pass when nk <= NW)
    const int wpu = nk <= NW ? NW / nk : 1, ngr = NW / wpu, sl = wid % wpu;
    const int us0 = wid / wpu;
    const bool wave_on = us0 < nk && wid < ngr * wpu;
    // one round of loads: the state, the descriptors and, with a, the first
    // round of this wavefront's candidates (up to the launch's bound; those
    // past the exact count are dropped below)
    __shared__ CommitIn ci;
    Cand c0[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) cand_none(c0[j]);
    const int nmax = PRE && wave_on ? a.ntl_max[us0] : 0;
    if (PRE && wave_on) {
        const gptr_t<const Cand> cand = as_global(a.cand[us0]);
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int i = 64 * sl + lane + 64 * wpu * j;
            if (i < nmax) {
                const gptr_t<const Cand> cp = cand + i;
                c0[j].v = cp->v; c0[j].key = cp->key; c0[j].sv = cp->sv;
            }
        }
    }
    if (tid < nk) {
        load_words(ci.ks[tid], &S->ks[tid]);
        ci.ntl[tid] = as_global(&S->sh.RT[tid])[0] * as_global(&S->sh.CT[tid])[0];
    }
    if (tid <= d) ci.rold[tid] = as_global(&S->r[par][tid])[0];
    if (tid == NTC - 1) {
        ci.stop = as_global(&S->stop)[0];
        ci.tau = as_global(&S->tau)[0];
        ci.err = as_global(&S->err)[0];
    }
    if (tid == NTC - 2) {
        ci.acc[0] = as_global(&S->alg_bytes)[0];
        ci.acc[1] = as_global(&S->new_entries)[0];
        ci.acc[2] = as_global(&S->pivoted)[0];
    }
    if (tid == NTC - 3) {
        ci.rook = P->rook; ci.r_max = P->r_max; ci.fp32 = P->fp32; ci.rcap = P->rcap;
        ci.hist_cap = P->hist_cap; ci.hm = P->hm;
    }
    constexpr int KW = (int)(sizeof(KDev) / 4);
    static_assert(sizeof(KDev) % 4 == 0, "word-sized descriptor");
    for (int w = tid; w < nk * KW; w += NTC) ((int *)ci.kd)[w] = as_global((const int *)P->kd)[w];
    __syncthreads();
    TT_STAMP(rec, 1);
    if (ci.stop) return;
    KSweep *const ks = ci.ks;
    const KDev *const kd = ci.kd;
    const int *const s_rold = ci.rold;
    const double s_tau = ci.tau;
    const bool rook = ci.rook != 0;
    __shared__ unsigned long long s_rcnt[TT_MAX_D];
    __shared__ int s_prop[TT_MAX_D], s_rnew[TT_MAX_D + 1];
    __shared__ unsigned long long s_bytes[TT_MAX_D], s_new[TT_MAX_D], s_piv[TT_MAX_D];
    __shared__ int s_geo[TT_MAX_D][4];

    // best candidate of unfolding us over this wavefront's share of the
    // tiles, in every lane
    auto scan = [&](int us, double &bv, uint64_t &bk, double &bs) {
        const KDev &K = kd[us];
        const int ntl = rook ? K.nrb * K.ncb : ci.ntl[us];
        bv = -1.0; bs = 0.0; bk = ~0ULL;
        if (rook && sl == 0) {
            // residuals the block searches looked at
            unsigned long long c = 0;
            for (int i = lane; i < ntl; i += 64) c += as_global((unsigned long long *)K.bcnt)[i];
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
            if (lane == 0) s_rcnt[us] = c;
        }
        int i0 = 64 * sl;
        if (PRE && us == us0 && ntl <= nmax) {      // the first round is in registers
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int i = i0 + lane + 64 * wpu * j;
                if (i < ntl && better(c0[j].v, c0[j].key, bv, bk)) { bv = c0[j].v; bk = c0[j].key; bs = c0[j].sv; }
            }
            i0 += 64 * wpu * CB;
        }
        scan_cands(as_global((const Cand *)K.cand), i0, ntl, wpu, bv, bk, bs);
        wave_best(bv, bk, bs);
    };

    // decide and commit unfolding u from its best candidate (one wavefront)
    auto decide = [&](int u, double bv, uint64_t bk, double bs) {
        const int k = u + 1;
        const KDev &K = kd[u];
        const int rk = ks[u].rk, nr = ks[u].nr, nc = ks[u].nc;
        const bool found = bv >= 0.0;
        const int row = (int)(bk >> 32), col = (int)(bk & 0xffffffffULL);
        double e = found ? bv : 0.0, p64 = 0.0, w64 = 0.0, v64 = 0.0;
        if constexpr (sizeof(V) == 4) {
            if (found) {
                // FP64 check of the FP32 candidate: stop test and pivot block in FP64
                p64 = fp64_check_wave<FNS>(P, K, u, rk, row, col, w64, v64);
                e = fabs(p64);
            }
        }
        const bool over = found && e > s_tau;
        const bool propose = over && rk < ci.r_max && rk < K.rk_cap;
        if (propose) {
            const int z = rk;
            const int p = row / K.nk, ik = row - p * K.nk;
            const int q = col / K.nk1, ik1 = col - q * K.nk1;
            if (lane == 0) {
                as_global((int *)K.rho)[z] = row;
                as_global((int *)K.gam)[z] = col;
                as_global((double *)K.piv)[z] = bs;
                as_global((double *)K.piv64)[z] = ci.fp32 ? p64 : bs;
                as_global((uint8_t *)K.rpiv)[row] = (uint8_t)(z + 1);
                as_global((uint8_t *)K.cpiv)[col] = (uint8_t)(z + 1);
                as_global((int *)K.Ifull)[z * k + k - 1] = ik;
                as_global((int *)K.Jfull)[z * (d - k)] = ik1;
            }
            if (lane < k - 1)
                as_global((int *)K.Ifull)[z * k + lane] = as_global((const int *)kd[u - 1].Ifull)[p * (k - 1) + lane];
            if (lane < d - k - 1)
                as_global((int *)K.Jfull)[z * (d - k) + 1 + lane] =
                    as_global((const int *)kd[u + 1].Jfull)[q * (d - k - 1) + lane];
            if (ci.fp32 && lane < z) {
                as_global((double *)K.Wp64)[z * ci.rcap + lane] = w64;
                as_global((double *)K.Up64)[lane * ci.rcap + z] = v64;
            }
        }
        if (lane == 0) {
            if (sweep < ci.hist_cap) as_global((double *)K.hist)[sweep] = e;
            S->last_best[u] = e;
            if (over && !propose) S->capped = 1;
            if (propose && bs == 0.0) {
                S->err = TT_ESINGULAR;
                ci.err = TT_ESINGULAR;
            }
            // traffic accounting of this sweep's tiles
            const unsigned long long nst = (unsigned long long)ks[u].nr_st, cst = (unsigned long long)ks[u].nc_st;
            const unsigned long long all = (unsigned long long)nr * (unsigned long long)nc;
            // (a restarted run's first sweep stores nothing)
            const unsigned long long live =
                (nst > (unsigned long long)rk && cst > (unsigned long long)rk) ? (nst - rk) * (cst - rk) : 0ull;
            if (rook) {
                // every residual looked at streams one factor vector of rk
                // values (the other is shared by the whole scan)
                s_bytes[u] = s_rcnt[u] * 8ull * (unsigned long long)rk;
                s_new[u] = 0;
                s_piv[u] = s_rcnt[u];
            } else {
                s_bytes[u] = live * sizeof(V) * (ks[u].apply ? 2ull : 1ull) + (all - nst * cst) * sizeof(V);
                s_new[u] = all - nst * cst;
                s_piv[u] = all;
            }
            s_prop[u] = propose ? 1 : 0;
            s_rnew[k] = rk + (propose ? 1 : 0);
            if (propose) {
                ks[u].arho = row;
                ks[u].agam = col;
                ks[u].apiv = bs;
            }
            // the descriptor fields the next shapes need
            s_geo[u][0] = K.nk;
            s_geo[u][1] = K.nk1;
            s_geo[u][2] = K.RTp;
            s_geo[u][3] = K.CTq;
        }
    };

    if (tid == 0) { s_rnew[0] = 1; s_rnew[d] = 1; }
    if (wpu == 1) {
        // a wavefront per unfolding: it decides as soon as its scan is done
        for (int u = wid; u < nk; u += NW) {
            double bv, bs;
            uint64_t bk;
            scan(u, bv, bk, bs);
            TT_STAMP(rec, 2);
            decide(u, bv, bk, bs);
        }
    } else {
        // several wavefronts per unfolding: partial result (u, sl) in slot
        // u * wpu + sl < NW, combined in wavefront order (the comparison
        // decides; the order only matters for equal keys, which cannot occur)
        __shared__ double s_pv[NW], s_psv[NW];
        __shared__ uint64_t s_pk[NW];
        __shared__ double s_wv[TT_MAX_D], s_wsv[TT_MAX_D];
        __shared__ uint64_t s_wk[TT_MAX_D];
        if (wave_on) {
            double bv, bs;
            uint64_t bk;
            scan(us0, bv, bk, bs);
            const int slot = us0 * wpu + sl;
            if (lane == 0) { s_pv[slot] = bv; s_pk[slot] = bk; s_psv[slot] = bs; }
        }
        __syncthreads();
        if (tid < nk) {
            double bv = -1.0, bs = 0.0;
            uint64_t bk = ~0ULL;
            for (int w = tid * wpu; w < (tid + 1) * wpu; ++w)
                if (better(s_pv[w], s_pk[w], bv, bk)) { bv = s_pv[w]; bk = s_pk[w]; bs = s_psv[w]; }
            s_wv[tid] = bv; s_wk[tid] = bk; s_wsv[tid] = bs;
        }
        __syncthreads();
        TT_STAMP(rec, 2);
        for (int u = wid; u < nk; u += NW) decide(u, s_wv[u], s_wk[u], s_wsv[u]);
    }
    lds_barrier();
    TT_STAMP(rec, 3);
    // the next sweep's shapes and tile counts: lane u of wavefront 0 prepares
    // unfolding u, and the tile offsets are prefix sums over the lanes
    if (tid < 64) {
        const int u = tid;
        int nn = 0, ns = 0;
        if (u < nk) {
            const int k = u + 1;
            const int knk = s_geo[u][0], knk1 = s_geo[u][1], kRTp = s_geo[u][2], kCTq = s_geo[u][3];
            KSweep n;
            n.rk = s_rnew[k];
            n.apply = s_prop[u];
            n.nr_st = ks[u].nr;
            n.nc_st = ks[u].nc;
            n.nr = s_rnew[k - 1] * knk;
            n.nc = knk1 * s_rnew[k + 1];
            n.arho = ks[u].arho;
            n.agam = ks[u].agam;
            n.apiv = ks[u].apiv;
            S->ks[u] = n;
            S->r[par ^ 1][k] = s_rnew[k];
            // tile counts from the ranks (rows r_{k-1} n_k, columns n_{k+1} r_{k+1})
            const int RT = s_rnew[k - 1] * kRTp, CT = s_rnew[k + 1] * kCTq;
            const int RTs = s_rold[k - 1] * kRTp, CTs = s_rold[k + 1] * kCTq;
            S->sh.RT[u] = RT;
            S->sh.CT[u] = CT;
            S->sh.RTs[u] = RTs;
            S->sh.CTs[u] = CTs;
            nn = RT * CT - RTs * CTs;
            ns = RTs * CTs;
        }
        // inclusive scans over the first 16 lanes (nk <= 15 carry counts)
        const int pn = row_scan_incl(nn), ps = row_scan_incl(ns);
        if (u < nk) {
            S->sh.noff[u] = pn - nn;
            S->sh.soff[u] = ps - ns;
        }
        if (u == nk - 1) {
            S->sh.noff[nk] = pn;
            S->sh.soff[nk] = ps;
        }
    }
    if (tid == 0) {
        // (every LDS read in flight at once; the error code is the one kept
        // in LDS, so that nothing here waits on device memory)
        int any = 0;
        unsigned long long ab = ci.acc[0], ne = ci.acc[1], pv = ci.acc[2];
#pragma unroll
        for (int u = 0; u < TT_MAX_D; ++u) {
            if (u < nk) {
                any |= s_prop[u];
                ab += s_bytes[u];
                ne += s_new[u];
                pv += s_piv[u];
            }
        }
        const int err = ci.err;
        S->alg_bytes = ab;
        S->new_entries = ne;
        S->pivoted = pv;
        const int stop = (!any || err) ? 1 : 0;
        S->stop = stop;
        S->sweeps = sweep + 1;
        HostMirror *hm = ci.hm;
        if (stop) {
            // final sweep: ranks and status must be visible before the count
            for (int j = 0; j <= d; ++j) hm->r[j] = s_rold[j];
            hm->err = err;
            hm->stop = stop;
            __threadfence_system();
            __hip_atomic_store(&hm->sweeps_done, sweep + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        } else {
            for (int j = 0; j <= d; ++j)
                __hip_atomic_store(&hm->r[j], s_rnew[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&hm->sweeps_done, sweep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        TT_STAMP(rec, 4);
    }
}

template <typename V, int FNS = 0>
static __global__ void __launch_bounds__(NTC) k_commit(const ProbDev *__restrict__ P, SweepArgs a)
{
    commit_body<V, FNS, true>(P, a.S, a.sweep, a.nk, a);
}

// ---------------------------------------------------------------------------
// Setup: samples, rms, first pivot, initial superblocks.
// ---------------------------------------------------------------------------
// Evaluates the sample entries and clears the pivot maps of every unfolding.
// Per-workgroup partial results of the sample pass: the sum of the squares of
// its NT samples as a complete binary tree over adjacent pairs (zeros past
// ns), and its largest |sample| (lowest index on ties).  Workgroup sums are
// the subtrees of the tree over all samples, so combining them pairwise gives
// that tree's value exactly.
template <int FNS>
__device__ inline void samples_body(const ProbDev *__restrict__ P, uint64_t seed, int ns, double *vals,
                                    SamplePart *part, int blk, int nblk)
{
    const int tid = threadIdx.x, s = blk * NT + tid;
    const int d = P->d, nk = P->nk;
    // the maps' places in one round of loads: a byte store may alias the
    // descriptor, so reading it between the stores would serialise them
    __shared__ uint8_t *s_rp[TT_MAX_D], *s_cp[TT_MAX_D];
    __shared__ int s_rc[TT_MAX_D], s_cc[TT_MAX_D];
    if (tid < nk) {
        const KDev &K = P->kd[tid];
        s_rp[tid] = K.rpiv; s_cp[tid] = K.cpiv;
        s_rc[tid] = K.rowcap; s_cc[tid] = K.colcap;
    }
    __syncthreads();
    for (int u = 0; u < nk; ++u) {
        for (int i = s; i < s_rc[u]; i += nblk * NT) s_rp[u][i] = 0;
        for (int j = s; j < s_cc[u]; j += nblk * NT) s_cp[u][j] = 0;
    }
    double v = 0.0;
    if (s < ns) {
        int idx[TT_MAX_D];
        for (int j = 0; j < d; ++j)
            idx[j] = (int)(sm64_at(seed, (uint64_t)s * d + j) % (uint64_t)P->F.n[j]);
        v = fn_value<double, FNS>(P->F, idx);
        vals[s] = v;
    }
    const double a = fabs(v);
    const int bad = (s < ns && !(a <= 1.7976931348623157e308)) ? 1 : 0;
    // adjacent-pair tree: within the wavefront by shuffles, then over the
    // four wavefronts
    double q = __dmul_rn(v, v);
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_down(q, off, 64);
        if ((tid & (2 * off - 1)) == 0) q = __dadd_rn(q, o);
    }
    __shared__ double wsum[NT / 64];
    __shared__ int sbad;
    if (tid == 0) sbad = 0;
    __syncthreads();
    if ((tid & 63) == 0) wsum[tid >> 6] = q;
    if (bad) atomicOr(&sbad, 1);
    double bv = (s < ns) ? a : -1.0, bs = v;
    uint64_t bk = (s < ns) ? (uint64_t)s : ~0ULL;
    block_best(bv, bk, bs);             // synchronises the workgroup
    if (tid == 0 && blk < sample_blocks(ns)) {     // a batched launch may run more workgroups
        SamplePart &o = part[blk];
        o.sumsq = __dadd_rn(__dadd_rn(wsum[0], wsum[1]), __dadd_rn(wsum[2], wsum[3]));
        o.bv = bv;
        o.bs = bs;
        o.bk = bk;
        o.bad = sbad;
    }
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_samples(const ProbDev *__restrict__ P, uint64_t seed, int ns,
                                                  double *vals, SamplePart *part)
{
    samples_body<FNS>(P, seed, ns, vals, part, blockIdx.x, gridDim.x);
}

// Pairwise sum of x(lo..lo+c) over a complete binary tree (c a power of two,
// entries at or past hi are zero), 64 leaves at a time in registers.
template <typename X> __device__ inline double tree64_sum(X x, int lo, int hi)
{
    double q[64];
#pragma unroll
    for (int b = 0; b < 64; ++b) q[b] = (lo + b < hi) ? x(lo + b) : 0.0;
#pragma unroll
    for (int w = 64; w > 1; w >>= 1) {
#pragma unroll
        for (int i = 0; i < w / 2; ++i) q[i] = __dadd_rn(q[2 * i], q[2 * i + 1]);
    }
    return q[0];
}

template <typename X> __device__ inline double chunk_pairwise_sum(X x, int lo, int c, int n)
{
    // a chunk of c <= 64 leaves is the left subtree of a 64-leaf tree whose
    // other leaves are zero, so it is summed exactly with them
    if (c <= 64) return tree64_sum(x, lo, min(lo + c, n));
    double st[32];
    int lv[32];
    int top = 0;
    for (int i = 0; i < c; i += 64) {
        double y = tree64_sum(x, lo + i, min(lo + i + 64, n));
        int level = 6;
        while (top > 0 && lv[top - 1] == level) {
            y = __dadd_rn(st[top - 1], y);
            --top;
            ++level;
        }
        st[top] = y;
        lv[top] = level;
        ++top;
    }
    return st[0];
}

// ---------------------------------------------------------------------------
// Restarts after false convergence (not in the paper; tt_options.restarts).
// A restarted run starts from several initial pivots per unfolding (the
// SeedPlan): the rank-1 recursion of eq. (aca_approx_E) restricted to the
// pivot rows and columns gives each pivot's residual and the frozen values
// on the pivot block; an entry of the pivot rows and columns depends on
// nothing else.  Step z updates the entries (a, b) with a, b > z only (the
// others are never read again), so every value the runs use matches a
// recursion over the whole superblock.
// ---------------------------------------------------------------------------
constexpr int MSP = TT_MAX_SEEDS + 2;    // pivot-block side: the points and one candidate

// One wavefront: the m x m pivot block of unfolding u in P (FP64), where row
// a is point ra(a)'s prefix (i_1..i_k) and column b point cb(b)'s suffix
// (i_{k+1}..i_d).  Then steps z < zend of the recursion; before step z,
// frozen(a, b, value) is called for row z from column z on and for column z
// below row z.
template <int FNS, typename RA, typename CB, typename FR>
__device__ inline void pivot_block_wave(const ProbDev *__restrict__ P, int k, int m, RA ra, CB cb, double (*Pm)[MSP],
                                        int zend, FR frozen)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < m * m; e += 64) {
        const int a = e / m, b = e - a * m;
        const int *pa = ra(a), *pb = cb(b);
        Pm[a][b] = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < k ? pa[j] : pb[j]; });
    }
    __builtin_amdgcn_wave_barrier();
    for (int z = 0; z < zend; ++z) {
        double nv[(MSP * MSP + 63) / 64];
#pragma unroll
        for (int i = 0; i < (MSP * MSP + 63) / 64; ++i) {
            const int e = lane + 64 * i, a = e / m, b = e - a * m;
            nv[i] = 0.0;
            if (e < m * m) {
                if ((a == z && b >= z) || (b == z && a > z)) frozen(a, b, Pm[a][b]);
                if (a > z && b > z) nv[i] = __fma_rn(-Pm[a][z], Pm[z][b] / Pm[z][z], Pm[a][b]);
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < (MSP * MSP + 63) / 64; ++i) {
            const int e = lane + 64 * i, a = e / m, b = e - a * m;
            if (e < m * m && a > z && b > z) Pm[a][b] = nv[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// The initial pivots of a restarted run (whole workgroup, after the samples'
// part of the setup): pivot data, masks, index tuples, the pivot block's
// frozen values in E, and shapes in which every tile of the first sweep is
// new (nothing stored yet).
template <typename V, int FNS>
__device__ void seeded_pivots(const ProbDev *__restrict__ P, ProbState *S, const SeedPlan *plan)
{
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, d = P->d, nk = P->nk;
    __shared__ double sP[NT / 64][MSP][MSP];
    for (int u = wid; u < nk; u += NT / 64) {
        const KDev &K = P->kd[u];
        const int k = u + 1, m = plan->m[u];
        const gptr_t<V> E = as_global((V *)K.E);
        const int64_t ld = K.ld;
        auto pt = [&](int z) { return plan->pts[plan->mem[u][z]]; };
        pivot_block_wave<FNS>(P, k, m, pt, pt, sP[wid], m, [&](int a, int b, double v) {
            E[(int64_t)plan->rho[u][a] * ld + plan->gam[u][b]] = (V)v;
        });
        if (lane < m) {
            const int z = lane, *pz = pt(z);
            const int rz = plan->rho[u][z], gz = plan->gam[u][z];
            K.rho[z] = rz;
            K.gam[z] = gz;
            K.piv[z] = (double)(V)sP[wid][z][z];
            K.piv64[z] = sP[wid][z][z];
            K.rpiv[rz] = (uint8_t)(z + 1);
            K.cpiv[gz] = (uint8_t)(z + 1);
            for (int j = 0; j < k; ++j) K.Ifull[z * k + j] = pz[j];
            for (int j = 0; j < d - k; ++j) K.Jfull[z * (d - k) + j] = pz[k + j];
        }
        if (lane == 0) {
            const int mp = u >= 1 ? plan->m[u - 1] : 1, mn = u + 1 < nk ? plan->m[u + 1] : 1;
            KSweep ks;
            ks.rk = m;
            ks.apply = 0;
            ks.nr_st = 0;
            ks.nc_st = 0;
            ks.nr = mp * K.nk;
            ks.nc = K.nk1 * mn;
            ks.arho = 0;
            ks.agam = 0;
            ks.apiv = 0.0;
            S->ks[u] = ks;
            S->r[0][k] = m;
            S->r[1][k] = m;
            P->hm->r[k] = m;
        }
    }
    if (tid == 0) {
        int no = 0;
        for (int u = 0; u < nk; ++u) {
            const KDev &K = P->kd[u];
            const int mp = u >= 1 ? plan->m[u - 1] : 1, mn = u + 1 < nk ? plan->m[u + 1] : 1;
            S->sh.RT[u] = mp * K.RTp;
            S->sh.CT[u] = mn * K.CTq;
            S->sh.RTs[u] = 0;
            S->sh.CTs[u] = 0;
            S->sh.noff[u] = no;
            S->sh.soff[u] = 0;
            no += S->sh.RT[u] * S->sh.CT[u];
        }
        S->sh.noff[nk] = no;
        S->sh.soff[nk] = 0;
        P->hm->r[0] = 1;
        P->hm->r[d] = 1;
    }
}

// |residual| of every candidate point as the next pivot of every unfolding it
// enters, after that unfolding's pivots in the plan: one wavefront per
// (candidate, unfolding); out[c * TT_MAX_D + u] (-1 where it does not enter).
template <int FNS>
static __global__ void __launch_bounds__(NT) k_point_resid(const ProbDev *__restrict__ P, const SeedPlan *plan,
                                                          const PointCheck *pc, double *out)
{
    const int nk = P->nk, wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (NT / 64) + wid, c = gw / nk, u = gw - c * nk;
    if (c >= pc->nc) return;
    if (!((pc->cin[c] >> u) & 1)) {
        if (lane == 0) out[c * TT_MAX_D + u] = -1.0;
        return;
    }
    __shared__ double sP[NT / 64][MSP][MSP];
    const int m = plan->m[u] + 1;
    auto pt = [&](int z) { return z < m - 1 ? plan->pts[plan->mem[u][z]] : pc->cand[c]; };
    pivot_block_wave<FNS>(P, u + 1, m, pt, pt, sP[wid], m - 1, [](int, int, double) {});
    if (lane == 0) out[c * TT_MAX_D + u] = fabs(sP[wid][m - 1][m - 1]);
}

template <typename V, int FNS>
__device__ void setup_body(const ProbDev *__restrict__ P, uint64_t seed, int ns, const SamplePart *part, double eps)
{
    ProbState *S = P->S;
    const int tid = threadIdx.x, d = P->d, nk = P->nk;
    const int nb = (ns + NT - 1) / NT;                 // workgroups that saw samples
    // One round of loads: the sample partials and what does not depend on
    // them -- the restart plan's size, the descriptor fields of the first
    // pivot's stores (16 threads per unfolding), the first sweep's shapes and
    // the mode sizes -- all requested before anything is stored (a byte
    // store may alias the descriptor, so a read after it would wait for it).
    const int npts = P->plan->npts;
    const int u = tid >> 4, l = tid & 15;
    const bool uk = u < nk;
    const KDev &K = P->kd[uk ? u : 0];
    const int knk = K.nk, knk1 = K.nk1;
    int *const kIfull = K.Ifull, *const kJfull = K.Jfull, *const krho = K.rho, *const kgam = K.gam;
    double *const kpiv = K.piv, *const kpiv64 = K.piv64;
    uint8_t *const krpiv = K.rpiv, *const kcpiv = K.cpiv;
    static_assert(SHAPE_WORDS <= NT && TT_MAX_D <= NT, "one shape word and one mode per thread");
    const int shw = ((const int *)&P->sh0)[min(tid, SHAPE_WORDS - 1)];
    const int nmode = P->F.n[min(tid, d - 1)];
    double bv = -1.0, bs = 0.0;
    uint64_t bk = ~0ULL;
    int bad = 0;
    for (int b = tid; b < nb; b += NT) {
        const SamplePart &o = part[b];
        bad |= o.bad;
        if (better(o.bv, o.bk, bv, bk)) { bv = o.bv; bk = o.bk; bs = o.bs; }
    }
    __shared__ int sbad, s_n[TT_MAX_D];
    if (tid == 0) sbad = 0;
    if (tid < d) s_n[tid] = nmode;
    __syncthreads();
    if (bad) atomicOr(&sbad, 1);
    block_best(bv, bk, bs);
    // the workgroup sums are the level-log2(NT) nodes of the tree over the
    // zero-padded samples; the rest of the tree runs over them
    int m = 1;
    while (m < nb) m <<= 1;
    const int c = (m >= NT) ? m / NT : 1;
    double q = 0.0;
    if (tid * c < m) q = chunk_pairwise_sum([&](int i) { return part[i].sumsq; }, tid * c, c, nb);
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_down(q, off, 64);
        if ((tid & (2 * off - 1)) == 0) q = __dadd_rn(q, o);
    }
    __shared__ double wsum[NT / 64];
    if ((tid & 63) == 0) wsum[tid >> 6] = q;
    __shared__ int i0[TT_MAX_D];
    __shared__ double p0s, p64;
    __syncthreads();
    if (tid == 0) {
        const double ss = __dadd_rn(__dadd_rn(wsum[0], wsum[1]), __dadd_rn(wsum[2], wsum[3]));
        const double rms = sqrt(ss / (double)ns);
        S->rms = rms;
        S->tau = eps * rms;
        for (int j = 0; j < d; ++j) i0[j] = (int)(sm64_at(seed, bk * d + j) % (uint64_t)s_n[j]);
        for (int j = 0; j < d; ++j) S->i0[j] = i0[j];
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j <= d; ++j) S->r[b][j] = 1;
        S->stop = 0; S->capped = 0; S->sweeps = 0; S->pivoted = 0;
        S->alg_bytes = 0; S->new_entries = 0;
        S->rook_rounds = 0; S->rook_long = 0;
        S->err = sbad ? TT_EFN : 0;
        p0s = (double)fn_value<V, FNS>(P->F, i0);
        p64 = (double)fn_value<double, FNS>(P->F, i0);
        if (p0s == 0.0) S->err = TT_ESINGULAR;
        if (S->err) S->stop = 1;
    }
    __syncthreads();
    // the first pivot of every unfolding: 16 threads per unfolding
    if (npts > 0) {
        seeded_pivots<V, FNS>(P, S, P->plan);
    } else if (uk) {
        const int k = u + 1;
        if (l < k) kIfull[l] = i0[l];
        if (l < d - k) kJfull[l] = i0[k + l];
        if (l == 0) {
            krho[0] = i0[k - 1];
            kgam[0] = i0[k];
            kpiv[0] = p0s;
            kpiv64[0] = p64;
            krpiv[i0[k - 1]] = 1;
            kcpiv[i0[k]] = 1;
            KSweep ks;
            ks.rk = 1;
            ks.apply = 1;                 // the first pivot is applied by the first sweep
            ks.nr_st = ks.nr = knk;
            ks.nc_st = ks.nc = knk1;
            ks.arho = i0[k - 1];
            ks.agam = i0[k];
            ks.apiv = p0s;
            S->ks[u] = ks;
        }
    }
    if (npts == 0) {
        if (tid < SHAPE_WORDS) ((int *)&S->sh)[tid] = shw;
        if (tid == 0)
            for (int j = 0; j <= d; ++j) P->hm->r[j] = 1;
    }
    if (tid == 0) {
        HostMirror *hm = P->hm;
        hm->stop = S->stop;
        __threadfence_system();
    }
}

template <typename V, int FNS = 0>
static __global__ void __launch_bounds__(NT) k_setup(const ProbDev *__restrict__ P, uint64_t seed, int ns,
                                                const SamplePart *part, double eps)
{
    setup_body<V, FNS>(P, seed, ns, part, eps);
}

// ---------------------------------------------------------------------------
// Rook mode: Alg. 1 run inside every subtensor block (the local pivot of
// Alg. 3) on residual factors instead of a stored residual.  For pivot z at
// (rho_z, gamma_z) with value p_z,
//   W(i, z) = residual of row i at column gamma_z before pivot z,
//   U(z, j) = residual of row rho_z at column j before pivot z, over p_z,
// each formed from the generating function and the earlier factors by the
// same fma chain as the in-place elimination, so that the residual at (i, j)
// after rk pivots, X(i, j) - sum_z W(i, z) U(z, j) in pivot order, carries
// the same bits as the stored residual of the greedy search.  Memory is
// (rows + columns) x rank instead of rows x columns.
// ---------------------------------------------------------------------------

// Piece of index i when n indices are split evenly into C pieces: piece b
// holds [floor(b n / C), floor((b+1) n / C)), so b = floor(((i+1) C - 1) / n).
__device__ inline int grid_piece(int i, int n, int C)
{
    return (int)(((int64_t)(i + 1) * C - 1) / n);
}

__device__ inline int piece_start(int b, int n, int C) { return (int)((int64_t)b * n / C); }

// Values z .. z+7 of a rook factor vector: one aligned 64-byte load from
// device memory (the chunk lies inside the vector's pitch; values at rk and
// beyond are read but not used), or eight LDS reads of a workgroup copy.
typedef double dvec8 __attribute__((ext_vector_type(8)));
__device__ inline dvec8 factor_chunk(gptr_t<const double> v, int z) { return *(gptr_t<const dvec8>)(v + z); }
__device__ inline dvec8 factor_chunk(const double *v, int z)
{
    dvec8 r;
#pragma unroll
    for (int m = 0; m < 8; ++m) r[m] = v[z + m];
    return r;
}

// x minus the products Wrow[z] * Ucol[z] for z = 0 .. rk-1 in that order, the
// fma chain of the in-place elimination.  Each vector is read chunk by chunk
// and every chunk is used as soon as it arrives: read value by value, a lane
// touches a new cache line per value of a random row, and with many lanes on
// many rows the lines are evicted before the next value is read.
template <typename TW, typename TU>
__device__ inline double factor_chain(double x, TW Wrow, TU Ucol, int rk)
{
    for (int z = 0; z < rk; z += 8) {
        const dvec8 w = factor_chunk(Wrow, z), v = factor_chunk(Ucol, z);
        const int m_end = rk - z;
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (m < m_end) x = __fma_rn(-w[m], v[m], x);
    }
    return x;
}

// The generating function at superblock entry (row, col) of unfolding u.
template <int FNS>
__device__ inline double rook_entry(const ProbDev *__restrict__ P, int u, int row, int col)
{
    const KDev &K = P->kd[u];
    const int k = u + 1, d = P->d;
    const int p = row / K.nk, ik = row - p * K.nk;
    const int q = col / K.nk1, ik1 = col - q * K.nk1;
    const gptr_t<const int> Ip = as_global((const int *)((k > 1) ? P->kd[u - 1].Ifull + p * (k - 1) : nullptr));
    const gptr_t<const int> Jq = as_global((const int *)((k < d - 1) ? P->kd[u + 1].Jfull + q * (d - k - 1) : nullptr));
    return fn_value_ix<double, FNS>(P->F, [&](int j) {
        return j < k - 1 ? Ip[j] : (j == k - 1 ? ik : (j == k ? ik1 : Jq[j - k - 1]));
    });
}

// Factors for this sweep: the newest pivot's column of W on the rows of the
// previous superblock and row of U on its columns, and every pivot's factor
// on the rows and columns that are new.  One thread per superblock row or
// column; every value read was written by an earlier sweep or earlier in the
// same thread.
template <int FNS>
__device__ void rook_factor_body(const ProbDev *__restrict__ P, int nk, int blk, int nblk)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    __shared__ KSweep ks[TT_MAX_D];
    __shared__ int off[TT_MAX_D + 1];
    if (threadIdx.x < nk) ks[threadIdx.x] = S->ks[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        int o = 0;
        for (int u = 0; u < nk; ++u) { off[u] = o; o += ks[u].nr + ks[u].nc; }
        off[nk] = o;
    }
    __syncthreads();
    const int tot = off[nk];
    for (int t = blk * NT + (int)threadIdx.x; t < tot; t += nblk * NT) {
        int u = 0;
        while (u + 1 < nk && t >= off[u + 1]) ++u;
        const KDev &K = P->kd[u];
        const KSweep &s = ks[u];
        const int e = t - off[u], rk = s.rk, wp = factor_pitch(K.rk_cap);
        const gptr_t<double> W = as_global(K.Wf), U = as_global(K.Uf);
        if (e < s.nr) {
            const int i = e;
            const int z0 = (i < s.nr_st) ? (s.apply ? rk - 1 : rk) : 0;
            const gptr_t<double> Wi = W + (int64_t)i * wp;
            for (int z = z0; z < rk; ++z) {
                const int gz = as_global((const int *)K.gam)[z];
                Wi[z] = factor_chain(rook_entry<FNS>(P, u, i, gz), gptr_t<const double>(Wi), gptr_t<const double>(U + (int64_t)gz * wp), z);
            }
        } else {
            const int j = e - s.nr;
            const int z0 = (j < s.nc_st) ? (s.apply ? rk - 1 : rk) : 0;
            const gptr_t<double> Uj = U + (int64_t)j * wp;
            for (int z = z0; z < rk; ++z) {
                const int rz = as_global((const int *)K.rho)[z];
                const double x = factor_chain(rook_entry<FNS>(P, u, rz, j), gptr_t<const double>(W + (int64_t)rz * wp), gptr_t<const double>(Uj), z);
                Uj[z] = x / as_global((const double *)K.piv)[z];
            }
        }
    }
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_rook_factors(const ProbDev *__restrict__ P, SweepArgs a)
{
    rook_factor_body<FNS>(P, a.nk, blockIdx.x, gridDim.x);
}

// Workgroup sum of a count; the result is valid in every thread.
__device__ inline unsigned long long block_sum_u64(unsigned long long c)
{
    __shared__ unsigned long long s_c[NT / 64];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    unsigned long long t = 0;
    for (int i = 0; i < NT / 64; ++i) t += s_c[i];
    __syncthreads();
    return t;
}

// Workgroup minimum of an int; valid in every thread.
__device__ inline int block_min_int(int c)
{
    __shared__ int s_m[NT / 64];
    for (int off = 32; off > 0; off >>= 1) c = min(c, __shfl_xor(c, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = c;
    __syncthreads();
    int t = s_m[0];
    for (int i = 1; i < NT / 64; ++i) t = min(t, s_m[i]);
    __syncthreads();
    return t;
}

// Rows and columns of one subtensor block of superblock u in this sweep, in
// ascending position: row t = pref[t / len] * n_k + lo + t % len, column t =
// suf[t / len1] * n_{k+1} + lo1 + t % len1, with pref (suf) the prefixes
// (suffixes) whose indices lie in the block.
struct RookGeom {
    int np, nq, lo, len, lo1, len1;
};

// Filled by one thread into workgroup-shared pref, suf and g.
__device__ inline void rook_block_geom(const ProbDev *__restrict__ P, int u, int b, const KSweep &ks, int *pref,
                                       int *suf, RookGeom &g)
{
    const KDev &K = P->kd[u];
    const int k = u + 1, d = P->d;
    const int rb = b % K.nrb, cb = b / K.nrb;
    int c[TT_MAX_D];
    int x = rb;
    for (int j = 0; j < k; ++j) { c[j] = x % P->grid[j]; x /= P->grid[j]; }
    x = cb;
    for (int j = k; j < d; ++j) { c[j] = x % P->grid[j]; x /= P->grid[j]; }
    const int rp = ks.nr / K.nk, rq = ks.nc / K.nk1;
    int np = 0;
    for (int p = 0; p < rp; ++p) {
        bool ok = true;
        for (int j = 0; j < k - 1 && ok; ++j)
            ok = grid_piece(as_global((const int *)P->kd[u - 1].Ifull)[p * (k - 1) + j], P->F.n[j], P->grid[j]) == c[j];
        if (ok) pref[np++] = p;
    }
    int nq = 0;
    for (int q = 0; q < rq; ++q) {
        bool ok = true;
        for (int j = 0; j < d - k - 1 && ok; ++j)
            ok = grid_piece(as_global((const int *)P->kd[u + 1].Jfull)[q * (d - k - 1) + j], P->F.n[k + 1 + j], P->grid[k + 1 + j]) ==
                 c[k + 1 + j];
        if (ok) suf[nq++] = q;
    }
    g.np = np;
    g.nq = nq;
    g.lo = piece_start(c[k - 1], K.nk, P->grid[k - 1]);
    g.len = piece_start(c[k - 1] + 1, K.nk, P->grid[k - 1]) - g.lo;
    g.lo1 = piece_start(c[k], K.nk1, P->grid[k]);
    g.len1 = piece_start(c[k] + 1, K.nk1, P->grid[k]) - g.lo1;
}

// One subtensor block of superblock u in this sweep, staged in LDS: its
// prefixes and suffixes with their index tuples, and the positions of the
// unfolding's pivots.  An entry at a position of the block then needs no
// index reads from memory, and whether a sampled row or column holds a
// pivot is a comparison against the rk pivot positions, so a residual at a
// random position reads only its two factor vectors.
struct RookBlock {
    KSweep ks;
    RookGeom g;
    int nk, nk1, npre, nsuf;
    int pref[TT_MAX_RANK], suf[TT_MAX_RANK];
    int rho[TT_MAX_RANK], gam[TT_MAX_RANK];
    int ptup[TT_MAX_RANK * TT_MAX_D], stup[TT_MAX_RANK * TT_MAX_D];

    __device__ int nR() const { return g.np * g.len; }
    __device__ int nC() const { return g.nq * g.len1; }
    __device__ int rowpos(int t) const { return pref[t / g.len] * nk + g.lo + t % g.len; }
    __device__ int colpos(int t) const { return suf[t / g.len1] * nk1 + g.lo1 + t % g.len1; }
    // local prefix (suffix) index of a superblock row (column) of the block
    __device__ int row_pref(int row) const
    {
        const int p = row / nk;
        int t = 0;
        while (t + 1 < g.np && pref[t] != p) ++t;
        return t;
    }
    __device__ int col_suf(int col) const
    {
        const int q = col / nk1;
        int t = 0;
        while (t + 1 < g.nq && suf[t] != q) ++t;
        return t;
    }
    __device__ bool pivot_row(int row) const
    {
        bool hit = false;
        for (int z = 0; z < ks.rk; ++z) hit |= rho[z] == row;
        return hit;
    }
    __device__ bool pivot_col(int col) const
    {
        bool hit = false;
        for (int z = 0; z < ks.rk; ++z) hit |= gam[z] == col;
        return hit;
    }
};

// Thread 0 reads the sweep's shapes and finds the block's geometry, then
// every thread stages the tuples and the pivot positions.  Ends with a
// barrier.
__device__ inline void rook_block_load(const ProbDev *__restrict__ P, int u, int b, RookBlock &B)
{
    const KDev &K = P->kd[u];
    const int k = u + 1, npre = k - 1, nsuf = P->d - k - 1;
    if (threadIdx.x == 0) {
        B.ks = P->S->ks[u];
        rook_block_geom(P, u, b, B.ks, B.pref, B.suf, B.g);
        B.nk = K.nk;
        B.nk1 = K.nk1;
        B.npre = npre;
        B.nsuf = nsuf;
    }
    __syncthreads();
    for (int z = threadIdx.x; z < B.ks.rk; z += NT) {
        B.rho[z] = as_global((const int *)K.rho)[z];
        B.gam[z] = as_global((const int *)K.gam)[z];
    }
    if (npre > 0) {
        const gptr_t<const int> I = as_global((const int *)P->kd[u - 1].Ifull);
        for (int e = threadIdx.x; e < B.g.np * npre; e += NT) {
            const int t = e / npre, j = e - t * npre;
            B.ptup[e] = I[B.pref[t] * npre + j];
        }
    }
    if (nsuf > 0) {
        const gptr_t<const int> J = as_global((const int *)P->kd[u + 1].Jfull);
        for (int e = threadIdx.x; e < B.g.nq * nsuf; e += NT) {
            const int t = e / nsuf, j = e - t * nsuf;
            B.stup[e] = J[B.suf[t] * nsuf + j];
        }
    }
    __syncthreads();
}

// The generating function at the block's local row (prefix tp, index ik of
// mode k) and column (index ik1 of mode k+1, suffix tq).
template <int FNS>
__device__ inline double rook_entry_loc(const ProbDev *__restrict__ P, const RookBlock &B, int tp, int ik, int tq,
                                        int ik1)
{
    const int npre = B.npre, k = npre + 1;
    const int *pt = B.ptup + tp * npre;
    const int *st = B.stup + tq * B.nsuf;
    return fn_value_ix<double, FNS>(P->F, [&](int j) {
        return j < npre ? pt[j] : (j == npre ? ik : (j == k ? ik1 : st[j - k - 1]));
    });
}

// Residual at a position of the block after rk pivots: the entry minus the
// factor products in pivot order.  Wrow: W(row, :); Ucol: U(:, col).  Both
// factors are stored as contiguous vectors of rk_cap values per row (W) and
// per column (U).
template <int FNS, typename TW, typename TU>
__device__ inline double rook_residual_loc(const ProbDev *__restrict__ P, const RookBlock &B, int tp, int ik, int tq,
                                           int ik1, TW Wrow, TU Ucol, int rk)
{
    return factor_chain(rook_entry_loc<FNS>(P, B, tp, ik, tq, ik1), Wrow, Ucol, rk);
}

// The loop of Alg. 1 run by one workgroup from (ci, cj), whose |residual| is
// bv: a column step (largest |residual| in column cj), then a row step (in
// row ci), each moving only to a strictly larger |residual|, until a round
// moves neither.  Among equal values the lowest position wins.  The loop ends
// by itself: every move raises |residual|, and a column step leaves the
// position at the largest |residual| of its column (a row step, of its row),
// so a column (row) that a step has searched is never entered again; hence
// at most min(rows, columns) + 1 rounds, the bound written below.
// Adds the residuals looked at to cnt; returns the rounds run.
template <int FNS>
__device__ int rook_walk(const ProbDev *__restrict__ P, const KDev &K, const RookBlock &B, double *s_f, double &bv,
                         double &bs, int &ci, int &cj, unsigned long long &cnt)
{
    const int tid = threadIdx.x, wp = factor_pitch(K.rk_cap), rk = B.ks.rk, nR = B.nR(), nC = B.nC();
    const int len = B.g.len, len1 = B.g.len1, lo = B.g.lo, lo1 = B.g.lo1;
    const gptr_t<const double> W = as_global((const double *)K.Wf), U = as_global((const double *)K.Uf);
    const gptr_t<const uint8_t> rpiv = as_global((const uint8_t *)K.rpiv), cpiv = as_global((const uint8_t *)K.cpiv);
    const int cap = min(nR, nC) + 1;
    int rounds = 0;
    while (rounds < cap) {
        ++rounds;
        bool moved = false;
        // column step: U(:, cj) shared by every row
        for (int z = tid; z < rk; z += NT) s_f[z] = U[(int64_t)cj * wp + z];
        const int tq = B.col_suf(cj), ik1 = cj - B.suf[tq] * B.nk1;
        __syncthreads();
        double tv = -1.0, ts = 0.0;
        uint64_t tk = ~0ULL;
        for (int t = tid; t < nR; t += NT) {
            const int row = B.rowpos(t);
            if (rpiv[row]) continue;
            ++cnt;
            const double x = rook_residual_loc<FNS>(P, B, t / len, lo + t % len, tq, ik1, W + (int64_t)row * wp, s_f, rk);
            if (better(fabs(x), (uint64_t)row, tv, tk)) { tv = fabs(x); tk = (uint64_t)row; ts = x; }
        }
        block_best(tv, tk, ts);
        if (tv > bv) { bv = tv; bs = ts; ci = (int)tk; moved = true; }
        // row step: W(ci, :) shared by every column
        for (int z = tid; z < rk; z += NT) s_f[z] = W[(int64_t)ci * wp + z];
        const int tp = B.row_pref(ci), ik = ci - B.pref[tp] * B.nk;
        __syncthreads();
        tv = -1.0;
        ts = 0.0;
        tk = ~0ULL;
        for (int t = tid; t < nC; t += NT) {
            const int col = B.colpos(t);
            if (cpiv[col]) continue;
            ++cnt;
            const double x = rook_residual_loc<FNS>(P, B, tp, ik, t / len1, lo1 + t % len1, s_f, U + (int64_t)col * wp, rk);
            if (better(fabs(x), (uint64_t)col, tv, tk)) { tv = fabs(x); tk = (uint64_t)col; ts = x; }
        }
        block_best(tv, tk, ts);
        if (tv > bv) { bv = tv; bs = ts; cj = (int)tk; moved = true; }
        if (!moved) break;
    }
    return rounds;
}

// Walk statistics of one block search (one thread per block).
__device__ inline void rook_note_rounds(const ProbDev *__restrict__ P, int rounds)
{
    ProbState *S = P->S;
    atomicMax(&S->rook_rounds, rounds);
    if (rounds > TT_ROOK_ITERS) atomicAdd(&S->rook_long, 1);
}

// The random set of Alg. 1 for block b of unfolding u in this sweep: pair s
// takes draws 2s (row) and 2s+1 (column) of the stream seeded with seed XOR
// mix(k | sweep << 8 | b << 32); pairs on a pivot row or column are
// skipped.  Samples s0, s0 + ds, ... below L = max(64, rows + columns).
template <int FNS>
__device__ inline void rook_samples(const ProbDev *__restrict__ P, const KDev &K, const RookBlock &B, int u, int b,
                                    int sweep, uint64_t seed, int s0, int ds, double &bv, uint64_t &bk, double &bs,
                                    unsigned long long &cnt)
{
    const int k = u + 1, wp = factor_pitch(K.rk_cap), rk = B.ks.rk, nR = B.nR(), nC = B.nC();
    const int len = B.g.len, len1 = B.g.len1, lo = B.g.lo, lo1 = B.g.lo1;
    const gptr_t<const double> W = as_global((const double *)K.Wf), U = as_global((const double *)K.Uf);
    const uint64_t tag = (uint64_t)k | ((uint64_t)sweep << 8) | ((uint64_t)b << 32);
    const uint64_t sig = seed ^ sm64_mix(tag);
    const int L = max(64, nR + nC);
    for (int s = s0; s < L; s += ds) {
        const uint64_t ra = sm64_at(sig, 2 * (uint64_t)s), ca = sm64_at(sig, 2 * (uint64_t)s + 1);
        const int tr = (int)(ra % (uint64_t)nR), tc = (int)(ca % (uint64_t)nC);
        const int row = B.rowpos(tr), col = B.colpos(tc);
        if (B.pivot_row(row) || B.pivot_col(col)) continue;
        ++cnt;
        const double x = rook_residual_loc<FNS>(P, B, tr / len, lo + tr % len, tc / len1, lo1 + tc % len1,
                                                W + (int64_t)row * wp, U + (int64_t)col * wp, rk);
        const uint64_t key = ((uint64_t)row << 32) | (uint32_t)col;
        if (better(fabs(x), key, bv, bk)) { bv = fabs(x); bk = key; bs = x; }
    }
}

// No sample off the pivot rows and columns: the block's first row and first
// column without a pivot (every thread gets the same answer; fr = nR or
// fc = nC when there is none).
__device__ inline void rook_first_free(const KDev &K, const RookBlock &B, int &fr, int &fc)
{
    const int nR = B.nR(), nC = B.nC();
    fr = nR;
    fc = nC;
    for (int t = threadIdx.x; t < nR; t += NT) if (!K.rpiv[B.rowpos(t)]) { fr = min(fr, t); break; }
    for (int t = threadIdx.x; t < nC; t += NT) if (!K.cpiv[B.colpos(t)]) { fc = min(fc, t); break; }
    fr = block_min_int(fr);
    fc = block_min_int(fc);
}

// One subtensor block of one superblock per workgroup: the random start of
// Alg. 1 from the block's seeded sample stream, then its loop (rook_walk).
// Ties go to the lowest position, as in the greedy search.
template <int FNS>
__device__ void rook_search_body(const ProbDev *__restrict__ P, int nk, int sweep, uint64_t seed, int wg)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int tid = threadIdx.x;
    int u = 0, b = wg;
    while (u < nk && b >= P->kd[u].nrb * P->kd[u].ncb) { b -= P->kd[u].nrb * P->kd[u].ncb; ++u; }
    if (u >= nk) return;
    const KDev &K = P->kd[u];
    __shared__ RookBlock B;
    __shared__ double s_f[TT_MAX_RANK];
    rook_block_load(P, u, b, B);
    const int nR = B.nR(), nC = B.nC(), rk = B.ks.rk, wp = factor_pitch(K.rk_cap);
    const gptr_t<const double> W = as_global((const double *)K.Wf), U = as_global((const double *)K.Uf);
    double bv = -1.0, bs = 0.0;
    uint64_t bk = ~0ULL;
    unsigned long long cnt = 0;
    int rounds = 0;
    if (nR > 0 && nC > 0) {
        rook_samples<FNS>(P, K, B, u, b, sweep, seed, tid, NT, bv, bk, bs, cnt);
        block_best(bv, bk, bs);
        if (bv < 0.0) {
            int fr, fc;
            rook_first_free(K, B, fr, fc);
            if (fr < nR && fc < nC) {
                const int row = B.rowpos(fr), col = B.colpos(fc);
                const double x = rook_residual_loc<FNS>(P, B, fr / B.g.len, B.g.lo + fr % B.g.len, fc / B.g.len1,
                                                        B.g.lo1 + fc % B.g.len1, W + (int64_t)row * wp,
                                                        U + (int64_t)col * wp, rk);
                bv = fabs(x);
                bs = x;
                bk = ((uint64_t)row << 32) | (uint32_t)col;
                if (tid == 0) ++cnt;
            }
        }
        if (bv >= 0.0) {
            int ci = (int)(bk >> 32), cj = (int)(bk & 0xffffffffULL);
            rounds = rook_walk<FNS>(P, K, B, s_f, bv, bs, ci, cj, cnt);
            bk = ((uint64_t)ci << 32) | (uint32_t)cj;
        }
    }
    cnt = block_sum_u64(cnt);
    if (tid == 0) {
        Cand &c = K.cand[b];
        c.v = bv; c.key = bk; c.sv = bs;
        K.bcnt[b] = cnt;
        if (rounds > 0) rook_note_rounds(P, rounds);
    }
}

// ---------------------------------------------------------------------------
// The same search with G workgroups per block, for large blocks.  The random
// set and every column or row scan are split over the G workgroups; each
// writes its partial best, and the next launch reduces the partials (every
// workgroup the same way) and moves the block's state.  Phase 0 draws the
// samples, phase p = 1..2 TT_ROOK_ITERS is a column step (p odd) or a row
// step (p even), and a finishing launch applies the last step and completes
// any walk still moving.  A block whose round moved nothing is done; its
// later launches return at once.  Values, order of comparisons and counts
// are those of the one-workgroup search.
// ---------------------------------------------------------------------------
__device__ inline bool rook_wg_of(const ProbDev *__restrict__ P, int nk, int G, int wg, int &u, int &b, int &g)
{
    u = 0;
    int r = wg;
    while (u < nk && r >= P->kd[u].nrb * P->kd[u].ncb * G) { r -= P->kd[u].nrb * P->kd[u].ncb * G; ++u; }
    if (u >= nk) return false;
    b = r / G;
    g = r - b * G;
    return true;
}

template <int FNS>
__device__ void rook_wsample_body(const ProbDev *__restrict__ P, int nk, int sweep, uint64_t seed, int wg)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int tid = threadIdx.x, G = P->rook_g;
    int u, b, g;
    if (!rook_wg_of(P, nk, G, wg, u, b, g)) return;
    const KDev &K = P->kd[u];
    __shared__ RookBlock B;
    rook_block_load(P, u, b, B);
    double bv = -1.0, bs = 0.0;
    uint64_t bk = ~0ULL;
    unsigned long long cnt = 0;
    if (B.nR() > 0 && B.nC() > 0) rook_samples<FNS>(P, K, B, u, b, sweep, seed, g * NT + tid, G * NT, bv, bk, bs, cnt);
    block_best(bv, bk, bs);
    cnt = block_sum_u64(cnt);
    if (tid == 0) {
        const int nb = K.nrb * K.ncb;
        Cand &c = K.rpart[(int64_t)0 * nb * G + (int64_t)b * G + g];
        c.v = bv; c.key = bk; c.sv = bs;
        K.rcnt[(int64_t)b * G + g] = cnt;
    }
}

// Best of the G partials of block b in partial buffer buf.
__device__ inline void rook_reduce_parts(const KDev &K, int G, int buf, int b, double &pv, uint64_t &pk, double &psv)
{
    const int nb = K.nrb * K.ncb;
    pv = -1.0; psv = 0.0; pk = ~0ULL;
    for (int i = threadIdx.x; i < G; i += NT) {
        const Cand c = K.rpart[(int64_t)buf * nb * G + (int64_t)b * G + i];
        if (better(c.v, c.key, pv, pk)) { pv = c.v; pk = c.key; psv = c.sv; }
    }
    block_best(pv, pk, psv);
}

// The block's state entering phase p >= 2, from the state entering p-1 and
// the partials p-1 left.
__device__ inline RookState rook_advance(RookState s, int p, double pv, uint64_t pk, double psv)
{
    if (!s.active) return s;
    if ((p - 1) & 1) {                          // p-1 was a column step
        if (pv > s.v) { s.v = pv; s.sv = psv; s.ci = (int)pk; s.moved = 1; }
    } else {                                    // p-1 was a row step: a round ends
        if (pv > s.v) { s.v = pv; s.sv = psv; s.cj = (int)pk; s.moved = 1; }
        ++s.rounds;
        if (!s.moved) s.active = 0;
        s.moved = 0;
    }
    return s;
}

template <int FNS>
__device__ void rook_wstep_body(const ProbDev *__restrict__ P, int nk, int p, int wg)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int tid = threadIdx.x, G = P->rook_g;
    int u, b, g;
    if (!rook_wg_of(P, nk, G, wg, u, b, g)) return;
    const KDev &K = P->kd[u];
    const int nb = K.nrb * K.ncb;
    __shared__ RookBlock B;
    __shared__ RookState st;
    __shared__ double s_f[TT_MAX_RANK];
    rook_block_load(P, u, b, B);
    double pv, psv;
    uint64_t pk;
    rook_reduce_parts(K, G, (p - 1) & 1, b, pv, pk, psv);
    const int nR = B.nR(), nC = B.nC(), rk = B.ks.rk, wp = factor_pitch(K.rk_cap);
    const int len = B.g.len, len1 = B.g.len1, lo = B.g.lo, lo1 = B.g.lo1;
    const gptr_t<const double> W = as_global((const double *)K.Wf), U = as_global((const double *)K.Uf);
    unsigned long long cnt = 0;
    if (tid == 0) {
        RookState s;
        if (p == 1) {
            s.valid = pv >= 0.0 ? 1 : 0;
            s.active = s.valid;
            s.moved = 0;
            s.rounds = 0;
            s.v = pv;
            s.sv = psv;
            s.ci = (int)(pk >> 32);
            s.cj = (int)(pk & 0xffffffffULL);
        } else {
            s = rook_advance(K.rst[(int64_t)((p - 1) & 1) * nb + b], p, pv, pk, psv);
        }
        st = s;
    }
    __syncthreads();
    if (p == 1 && !st.valid && nR > 0 && nC > 0) {
        int fr, fc;
        rook_first_free(K, B, fr, fc);
        if (fr < nR && fc < nC && tid == 0) {
            const int row = B.rowpos(fr), col = B.colpos(fc);
            const double x = rook_residual_loc<FNS>(P, B, fr / len, lo + fr % len, fc / len1, lo1 + fc % len1,
                                                    W + (int64_t)row * wp, U + (int64_t)col * wp, rk);
            st.v = fabs(x);
            st.sv = x;
            st.ci = row;
            st.cj = col;
            st.valid = 1;
            st.active = 1;
            if (g == 0) cnt = 1;
        }
        __syncthreads();
    }
    if (g == 0 && tid == 0) K.rst[(int64_t)(p & 1) * nb + b] = st;
    double tv = -1.0, ts = 0.0;
    uint64_t tk = ~0ULL;
    if (st.active) {
        if (p & 1) {
            // column step
            for (int z = tid; z < rk; z += NT) s_f[z] = U[(int64_t)st.cj * wp + z];
            const int tq = B.col_suf(st.cj), ik1 = st.cj - B.suf[tq] * B.nk1;
            __syncthreads();
            for (int t = g * NT + tid; t < nR; t += G * NT) {
                const int row = B.rowpos(t);
                if (K.rpiv[row]) continue;
                ++cnt;
                const double x = rook_residual_loc<FNS>(P, B, t / len, lo + t % len, tq, ik1, W + (int64_t)row * wp,
                                                        s_f, rk);
                if (better(fabs(x), (uint64_t)row, tv, tk)) { tv = fabs(x); tk = (uint64_t)row; ts = x; }
            }
        } else {
            // row step
            for (int z = tid; z < rk; z += NT) s_f[z] = W[(int64_t)st.ci * wp + z];
            const int tp = B.row_pref(st.ci), ik = st.ci - B.pref[tp] * B.nk;
            __syncthreads();
            for (int t = g * NT + tid; t < nC; t += G * NT) {
                const int col = B.colpos(t);
                if (K.cpiv[col]) continue;
                ++cnt;
                const double x = rook_residual_loc<FNS>(P, B, tp, ik, t / len1, lo1 + t % len1, s_f,
                                                        U + (int64_t)col * wp, rk);
                if (better(fabs(x), (uint64_t)col, tv, tk)) { tv = fabs(x); tk = (uint64_t)col; ts = x; }
            }
        }
    }
    block_best(tv, tk, ts);
    cnt = block_sum_u64(cnt);
    if (tid == 0) {
        Cand &c = K.rpart[(int64_t)(p & 1) * nb * G + (int64_t)b * G + g];
        c.v = tv; c.key = tk; c.sv = ts;
        K.rcnt[(int64_t)b * G + g] += cnt;
    }
}

// After the last step: the block's pivot and count.  One workgroup per block.
// A walk still moving after the fixed TT_ROOK_ITERS rounds is not cut short:
// this workgroup runs the rest of Alg. 1's loop (rook_walk, the comparisons
// and counts of the split steps) until it stops.
template <int FNS>
__device__ void rook_wfinish_body(const ProbDev *__restrict__ P, int nk, int wg)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int tid = threadIdx.x, G = P->rook_g, p = 2 * TT_ROOK_ITERS + 1;
    int u, b, g;
    if (!rook_wg_of(P, nk, 1, wg, u, b, g)) return;
    const KDev &K = P->kd[u];
    const int nb = K.nrb * K.ncb;
    __shared__ RookState st;
    __shared__ RookBlock B;
    __shared__ double s_f[TT_MAX_RANK];
    double pv, psv;
    uint64_t pk;
    rook_reduce_parts(K, G, (p - 1) & 1, b, pv, pk, psv);
    unsigned long long c = 0;
    for (int i = tid; i < G; i += NT) c += K.rcnt[(int64_t)b * G + i];
    c = block_sum_u64(c);
    if (tid == 0) st = rook_advance(K.rst[(int64_t)((p - 1) & 1) * nb + b], p, pv, pk, psv);
    __syncthreads();
    if (st.active) {                            // uniform: read after the barrier
        rook_block_load(P, u, b, B);
        double bv = st.v, bs = st.sv;
        int ci = st.ci, cj = st.cj;
        unsigned long long more = 0;
        const int r = rook_walk<FNS>(P, K, B, s_f, bv, bs, ci, cj, more);
        more = block_sum_u64(more);
        if (tid == 0) {
            st.v = bv;
            st.sv = bs;
            st.ci = ci;
            st.cj = cj;
            st.rounds += r;
            c += more;
        }
    }
    if (tid == 0) {
        Cand &o = K.cand[b];
        if (st.valid) {
            o.v = st.v;
            o.key = ((uint64_t)st.ci << 32) | (uint32_t)st.cj;
            o.sv = st.sv;
            rook_note_rounds(P, st.rounds);
        } else {
            o.v = -1.0;
            o.key = ~0ULL;
            o.sv = 0.0;
        }
        K.bcnt[b] = c;
    }
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_rook_wsample(const ProbDev *__restrict__ P, SweepArgs a, uint64_t seed)
{
    rook_wsample_body<FNS>(P, a.nk, a.sweep, seed, blockIdx.x);
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_rook_wstep(const ProbDev *__restrict__ P, SweepArgs a, int phase)
{
    rook_wstep_body<FNS>(P, a.nk, phase, blockIdx.x);
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_rook_wfinish(const ProbDev *__restrict__ P, SweepArgs a)
{
    rook_wfinish_body<FNS>(P, a.nk, blockIdx.x);
}

template <int FNS = 0>
static __global__ void __launch_bounds__(NT) k_rook_search(const ProbDev *__restrict__ P, SweepArgs a, uint64_t seed)
{
    rook_search_body<FNS>(P, a.nk, a.sweep, seed, blockIdx.x);
}

// E = X on the initial superblocks (one prefix, one suffix: the first pivot's).
template <typename V, int FNS>
__device__ void init_eval_body(const ProbDev *__restrict__ P, int u, int blk, int nblk)
{
    const ProbState *S = P->S;
    if (S->stop) return;
    const int k = u + 1, d = P->d;
    const KDev &K = P->kd[u];
    const int64_t tot = (int64_t)K.nk * K.nk1;
    for (int64_t e = (int64_t)blk * NT + threadIdx.x; e < tot; e += (int64_t)nblk * NT) {
        const int i = (int)(e / K.nk1), j = (int)(e - (int64_t)i * K.nk1);
        int idx[TT_MAX_D];
        for (int jj = 0; jj < d; ++jj) idx[jj] = S->i0[jj];
        idx[k - 1] = i;
        idx[k] = j;
        ((V *)K.E)[(int64_t)i * K.ld + j] = fn_value<V, FNS>(P->F, idx);
    }
}

template <typename V, int FNS = 0>
static __global__ void __launch_bounds__(NT) k_init_eval(const ProbDev *__restrict__ P)
{
    init_eval_body<V, FNS>(P, blockIdx.y, blockIdx.x, gridDim.x);
}

// Copies n ints from device memory to LDS with NTH threads, U loads per
// thread in flight before any store (a plain loop would wait a round trip per
// pass).
template <int U, int NTH> __device__ inline void copy_to_lds(int *dst, gptr_t<const int> src, int n)
{
    for (int e0 = (int)threadIdx.x; e0 < n; e0 += U * NTH) {
        int v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = src[min(e0 + j * NTH, n - 1)];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (e0 + j * NTH < n) dst[e0 + j * NTH] = v[j];
    }
}

// ---------------------------------------------------------------------------
// Cores by Alg. 4 (FP64), one 64-thread workgroup per 64 rows of
// A_k = X(I_{<=k-1} x [n_k], J_{>k}) (the sliced fibers of eq. corereshape).
// Each workgroup evaluates its rows' fibers and the pivot rows' fibers
// A(I_{<=k}, J_{>k}), runs the pivot rows' recursion (lane t = pivot row t,
// lock-step within the wavefront) and, step by step, applies
// eq. (aca_approx_T_sub) to its own rows:
//   s = T(:, 0..z-1) A(I_z, j_z) - A(:, j_z),  delta^{-1} = -s(i_z),
//   T <- [T + delta s T(i_z, :), -delta s].
// Workgroups past the last unfolding's rows evaluate G_d = X(I_{<=d-1}, :).
// ---------------------------------------------------------------------------
// The core workgroups are one wavefront each: its lanes run in lockstep and
// the LDS serves one wavefront's accesses in order, so ordering the accesses
// in the compiler is all a barrier has to do.
__device__ inline void wave_sync() { __builtin_amdgcn_wave_barrier(); }

struct CoreArgs {
    int nk;
    int ranks[TT_MAX_D + 1];
    int64_t goff[TT_MAX_D + 1]; // offset of G_k in the cores buffer
    int rowblocks[TT_MAX_D + 1];// prefix sum of 64-row blocks per unfolding; [nk] = start of G_d blocks
};

constexpr int A4W = 64;         // rows per workgroup (one wavefront)

// Offsets of the cores and their workgroup ranges for final ranks r[0..d];
// returns the number of workgroups (row blocks of G_1..G_{d-1}, then G_d).
__host__ __device__ inline int make_core_args(int d, const int *n, const int *r, CoreArgs &a, int64_t &len)
{
    a.nk = d - 1;
    for (int k = 0; k <= d; ++k) a.ranks[k] = r[k];
    int64_t go = 0;
    int rb = 0;
    for (int u = 0; u < d - 1; ++u) {
        const int k = u + 1;
        const int nr = r[k - 1] * n[k - 1], rk = r[k];
        a.goff[u] = go;
        a.rowblocks[u] = rb;
        go += (int64_t)nr * rk;
        rb += (nr + A4W - 1) / A4W;
    }
    a.rowblocks[d - 1] = rb;
    a.goff[d - 1] = go;
    const int64_t gd = (int64_t)r[d - 1] * n[d - 1];
    len = go + gd;
    return rb + (int)((gd + A4W - 1) / A4W);
}

// Alg. 4 on one wavefront's rows with T in registers (rk <= RM; RM = 16 fits
// the register file, 32 does not): lane i holds
// row i of T for the workgroup's rows, and lanes z < rk also row z of T for
// the pivot rows (the recursion on those rows gives every delta).  The
// operations and their order are those of the LDS version below; T(i_z, :)
// reaches the other lanes by shuffles before lane z updates it.
template <int RM>
__device__ bool core_alg4_regs(const double *Ap, const double *Ab, int st, int rk, int nr, int i0, double *Gk0)
{
    bool singular = false;
    const int lane = threadIdx.x;
    const bool piv = lane < rk;
    double ab[RM], tb[RM], tp[RM];
    const double a11 = Ap[0];
#pragma unroll
    for (int z = 0; z < RM; ++z) {
        ab[z] = (z < rk) ? Ab[z * A4W + lane] : 0.0;
        tb[z] = 0.0;
        tp[z] = 0.0;
    }
    tb[0] = ab[0] / a11;
    if (piv) tp[0] = Ap[lane * st] / a11;
#pragma unroll
    for (int z = 1; z < RM; ++z) {
        if (z >= rk) continue;                  // uniform: every lane skips
        double dotb = 0.0, dotp = 0.0;
#pragma unroll
        for (int zz = 0; zz < z; ++zz) {
            const double az = Ap[zz * st + z];
            dotb = __fma_rn(tb[zz], az, dotb);
            dotp = __fma_rn(tp[zz], az, dotp);
        }
        const double sb = dotb - ab[z];
        const double sp = piv ? dotp - Ap[lane * st + z] : 0.0;
        const double dinv = -__shfl(sp, z, 64);
        singular |= dinv == 0.0;
        const double delta = 1.0 / dinv;
        const double cb = delta * sb, cp = delta * sp;
#pragma unroll
        for (int zz = 0; zz < z; ++zz) {
            const double tr = __shfl(tp[zz], z, 64);   // T(i_z, zz) before this step
            tb[zz] = __fma_rn(cb, tr, tb[zz]);
            if (piv) tp[zz] = __fma_rn(cp, tr, tp[zz]);
        }
        tb[z] = -cb;
        if (piv) tp[z] = -cp;
    }
    if (i0 + lane < nr) {
        double *row = Gk0 + (int64_t)(i0 + lane) * rk;
#pragma unroll
        for (int z = 0; z < RM; ++z)
            if (z < rk) row[z] = tb[z];
    }
    return singular;
}

// G_d = X(I_{<=d-1}, :): the workgroups past the last unfolding's rows, one
// entry per lane.
template <int FNS>
__device__ void core_last_fiber(const ProbDev *__restrict__ P, const CoreArgs &a, double *G, int bid)
{
    const int lane = threadIdx.x, d = P->d;
    const KDev &K = P->kd[d - 2];
    const int rd = a.ranks[d - 1], nd = P->F.n[d - 1];
    const int64_t e = (int64_t)(bid - a.rowblocks[a.nk]) * A4W + lane;
    if (e >= (int64_t)rd * nd) return;
    const int pp = (int)(e / nd), i = (int)(e - (int64_t)pp * nd);
    const gptr_t<const int> Ip = as_global((const int *)K.Ifull) + pp * (d - 1);
    // the lane's index tuple, every entry in flight at once
    int pv[TT_MAX_D];
#pragma unroll
    for (int j = 0; j < TT_MAX_D; ++j) pv[j] = Ip[min(j, d - 2)];
    if constexpr (FNS == TT_FN_HILBERT) {
        // the entry depends on the integer index sum only
        long long s = (long long)i + 1;
#pragma unroll
        for (int j = 0; j < TT_MAX_D; ++j)
            if (j < d - 1) s += (long long)pv[j] + 1;
        G[a.goff[d - 1] + e] = 1.0 / ((double)s + P->F.shift);
    } else {
        // through LDS: the function reads the tuple by a runtime index
        __shared__ int sIp[A4W * TT_MAX_D];
#pragma unroll
        for (int j = 0; j < TT_MAX_D; ++j)
            if (j < d - 1) sIp[lane * TT_MAX_D + j] = pv[j];
        G[a.goff[d - 1] + e] = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < d - 1 ? sIp[lane * TT_MAX_D + j] : i; });
    }
}

template <int FNS>
__device__ void cores_body(const ProbDev *__restrict__ P, const CoreArgs &a, double *G, int bid)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x, d = P->d;
    if (bid >= a.rowblocks[a.nk]) {
        core_last_fiber<FNS>(P, a, G, bid);
        return;
    }
    int u = 0;
    while (u + 1 < a.nk && bid >= a.rowblocks[u + 1]) ++u;
    const int k = u + 1;
    const KDev &K = P->kd[u];
    const int rk = a.ranks[k], nr = a.ranks[k - 1] * K.nk, st = rk + 1, nj = d - k;
    double *Tp = (double *)smem_raw;            // Tp[t*st + z]: T of pivot row t
    double *Ap = Tp + rk * st;                  // Ap[t*st + z] = A(rho_t, z)
    double *Tb = Ap + rk * st;                  // Tb[z*A4W + lane]: T of this lane's row
    double *Ab = Tb + rk * A4W;                 // Ab[z*A4W + lane] = A(row, z)
    const int i0 = (bid - a.rowblocks[u]) * A4W, i = i0 + lane;
    const bool act = i < nr;
    const int p = act ? i / K.nk : 0, ik = act ? i - p * K.nk : 0;
    // one round of loads: the pivots' index tuples and every lane's prefix
    __shared__ int sJ[TT_MAX_RANK * TT_MAX_D], sI[TT_MAX_RANK * TT_MAX_D], sPre[A4W * TT_MAX_D];
    const gptr_t<const int> Jf = as_global((const int *)K.Jfull), If = as_global((const int *)K.Ifull);
    copy_to_lds<4, A4W>(sJ, Jf, rk * nj);
    copy_to_lds<4, A4W>(sI, If, rk * k);
    if (k >= 2) {
        // the lane's prefix, every entry in flight at once
        const gptr_t<const int> preI = as_global((const int *)P->kd[u - 1].Ifull) + p * (k - 1);
        int pv[TT_MAX_D];
#pragma unroll
        for (int j = 0; j < TT_MAX_D; ++j) pv[j] = preI[min(j, k - 2)];
#pragma unroll
        for (int j = 0; j < TT_MAX_D; ++j)
            if (j < k - 1) sPre[lane * TT_MAX_D + j] = pv[j];
    }
    wave_sync();
    if constexpr (FNS == TT_FN_HILBERT) {
        // the Hilbert entry depends on the integer index sum only: add the
        // prefix, suffix and pivot-tuple parts once, exactly, in integers
        __shared__ long long sJs[TT_MAX_RANK];
        long long is = 0;
        if (lane < rk) {
            long long js = 0;
            for (int j = 0; j < nj; ++j) js += sJ[lane * nj + j] + 1;
            for (int j = 0; j < k; ++j) is += sI[lane * k + j] + 1;
            sJs[lane] = js;
        }
        long long ps = ik + 1;
        for (int j = 0; j < k - 1; ++j) ps += sPre[lane * TT_MAX_D + j] + 1;
        wave_sync();
        const double sh = P->F.shift;
        for (int z = 0; z < rk; ++z) {
            const long long js = sJs[z];
            Ab[z * A4W + lane] = act ? 1.0 / ((double)(ps + js) + sh) : 0.0;
            if (lane < rk) Ap[lane * st + z] = 1.0 / ((double)(is + js) + sh);
        }
    } else {
        for (int z = 0; z < rk; ++z) {
            const int *Jz = sJ + z * nj;
            Ab[z * A4W + lane] = act ? fn_value_ix<double, FNS>(P->F, [&](int j) {
                return j < k - 1 ? sPre[lane * TT_MAX_D + j] : (j == k - 1 ? ik : Jz[j - k]);
            }) : 0.0;
            if (lane < rk) {
                const int *It = sI + lane * k;
                Ap[lane * st + z] = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < k ? It[j] : Jz[j - k]; });
            }
        }
    }
    wave_sync();
    if (rk <= 16) {
        // a zero pivot-block residual (delta^{-1} = 0): singular, as in the oracle
        if (core_alg4_regs<16>(Ap, Ab, st, rk, nr, i0, G + a.goff[u]) && lane == 0) P->S->err = TT_ESINGULAR;
        return;
    }
    bool singular = false;
    const double a11 = Ap[0];
    for (int z = 0; z < rk; ++z) {
        Tb[z * A4W + lane] = (z == 0) ? Ab[lane] / a11 : 0.0;
        if (lane < rk) Tp[lane * st + z] = (z == 0) ? Ap[lane * st] / a11 : 0.0;
    }
    wave_sync();
    for (int z = 1; z < rk; ++z) {
        // the two dot products, each summed in ascending zz, side by side
        // and unrolled so that their LDS reads overlap
        double dotb = 0.0, dotp = 0.0;
        const bool piv_lane = lane < rk;
#pragma unroll 4
        for (int zz = 0; zz < z; ++zz) {
            const double az = Ap[zz * st + z];
            dotb = __fma_rn(Tb[zz * A4W + lane], az, dotb);
            if (piv_lane) dotp = __fma_rn(Tp[lane * st + zz], az, dotp);
        }
        const double sb = dotb - Ab[z * A4W + lane];
        const double sp = piv_lane ? dotp - Ap[lane * st + z] : 0.0;
        const double dinv = -__shfl(sp, z, 64);
        singular |= dinv == 0.0;
        const double delta = 1.0 / dinv;
        const double cb = delta * sb, cp = delta * sp;
        wave_sync();                            // every lane has read T before it changes
        // every lane reads T(i_z, zz) in the same instruction before lane z
        // (the only writer of that entry) updates it, and the other entries
        // each lane touches are its own, so no barrier is needed in here
#pragma unroll 4
        for (int zz = 0; zz < z; ++zz) {
            const double tr = Tp[z * st + zz];  // T(i_z, zz) before this step
            Tb[zz * A4W + lane] = __fma_rn(cb, tr, Tb[zz * A4W + lane]);
            if (lane < rk) Tp[lane * st + zz] = __fma_rn(cp, tr, Tp[lane * st + zz]);
        }
        Tb[z * A4W + lane] = -cb;
        if (lane < rk) Tp[lane * st + z] = -cp;
        wave_sync();
    }
    const int rows = min(A4W, nr - i0);
    double *Gk = G + a.goff[u] + (int64_t)i0 * rk;
    for (int e = lane; e < rows * rk; e += A4W) {
        const int ii = e / rk, z = e - ii * rk;
        Gk[e] = Tb[z * A4W + ii];
    }
    if (singular && lane == 0) P->S->err = TT_ESINGULAR;
}

template <int FNS = 0>
static __global__ void __launch_bounds__(A4W) k_cores(const ProbDev *__restrict__ P, CoreArgs a, double *G)
{
    cores_body<FNS>(P, a, G, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Cores with the pivot rows' recursion run once.  Alg. 4's steps on the pivot
// rows do not depend on the fiber rows, so k_core_piv runs them once per
// unfolding (one wavefront, lane t = pivot row t, as in cores_body) and
// records what every row's step reads; k_cores_t then applies the steps to 64
// rows per workgroup with each row's T in registers.  The operations and
// their order are those of cores_body, so the cores are the same bits.
// Table of unfolding u at tab + u * CT_STRIDE:
//   At[z * CT_LD + t] = A(rho_t, gam_z) for t < z, and At[0] = A(rho_0, gam_0)
//   Tr[z * CT_LD + t] = T(i_z, t) before step z, for t < z
//   Dl[z]             = delta of step z
// ---------------------------------------------------------------------------
constexpr int CT_LD = TT_MAX_RANK;
constexpr int CT_STRIDE = 2 * CT_LD * CT_LD + CT_LD;

template <int FNS>
__device__ void core_piv_body(const ProbDev *__restrict__ P, const CoreArgs &a, double *tab, int u)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x, d = P->d, k = u + 1;
    const KDev &K = P->kd[u];
    const int rk = a.ranks[k], st = rk + 1, nj = d - k;
    double *Tp = (double *)smem_raw;            // Tp[t*st + z]: T of pivot row t
    double *Ap = Tp + rk * st;                  // Ap[t*st + z] = A(rho_t, z)
    __shared__ int sJ[TT_MAX_RANK * TT_MAX_D], sI[TT_MAX_RANK * TT_MAX_D];
    copy_to_lds<4, A4W>(sJ, as_global((const int *)K.Jfull), rk * nj);
    copy_to_lds<4, A4W>(sI, as_global((const int *)K.Ifull), rk * k);
    wave_sync();
    const bool piv = lane < rk;
    if constexpr (FNS == TT_FN_HILBERT) {
        __shared__ long long sJs[TT_MAX_RANK];
        long long is = 0;
        if (piv) {
            long long js = 0;
            for (int j = 0; j < nj; ++j) js += sJ[lane * nj + j] + 1;
            for (int j = 0; j < k; ++j) is += sI[lane * k + j] + 1;
            sJs[lane] = js;
        }
        wave_sync();
        const double sh = P->F.shift;
        if (piv)
            for (int z = 0; z < rk; ++z) Ap[lane * st + z] = 1.0 / ((double)(is + sJs[z]) + sh);
    } else if (piv) {
        const int *It = sI + lane * k;
        for (int z = 0; z < rk; ++z) {
            const int *Jz = sJ + z * nj;
            Ap[lane * st + z] = fn_value_ix<double, FNS>(P->F, [&](int j) { return j < k ? It[j] : Jz[j - k]; });
        }
    }
    wave_sync();
    double *At = tab + (int64_t)u * CT_STRIDE, *Tr = At + CT_LD * CT_LD, *Dl = Tr + CT_LD * CT_LD;
    const double a11 = Ap[0];
    if (piv)
        for (int z = 0; z < rk; ++z) Tp[lane * st + z] = (z == 0) ? Ap[lane * st] / a11 : 0.0;
    wave_sync();
    bool singular = false;
    for (int z = 1; z < rk; ++z) {
        double dotp = 0.0;
        if (piv)
            for (int zz = 0; zz < z; ++zz) dotp = __fma_rn(Tp[lane * st + zz], Ap[zz * st + z], dotp);
        const double sp = piv ? dotp - Ap[lane * st + z] : 0.0;
        const double dinv = -__shfl(sp, z, 64);
        singular |= dinv == 0.0;
        const double delta = 1.0 / dinv;
        const double cp = delta * sp;
        // T(i_z, :) as every row's step reads it, before lane z updates it
        if (lane < z) Tr[z * CT_LD + lane] = Tp[z * st + lane];
        if (lane == 0) Dl[z] = delta;
        wave_sync();
        for (int zz = 0; zz < z; ++zz) {
            const double tr = Tp[z * st + zz];
            if (piv) Tp[lane * st + zz] = __fma_rn(cp, tr, Tp[lane * st + zz]);
        }
        if (piv) Tp[lane * st + z] = -cp;
        wave_sync();
    }
    for (int z = 1; z < rk; ++z)
        if (lane < z) At[z * CT_LD + lane] = Ap[lane * st + z];
    if (lane == 0) At[0] = a11;
    // a zero pivot-block residual (delta^{-1} = 0): singular, as in the oracle
    if (singular && lane == 0) P->S->err = TT_ESINGULAR;
}

template <int FNS = 0>
static __global__ void __launch_bounds__(A4W) k_core_piv(const ProbDev *__restrict__ P, CoreArgs a, double *tab)
{
    core_piv_body<FNS>(P, a, tab, blockIdx.x);
}

// Rows of A_k by the recorded steps; RM >= the largest rank (registers per
// row's T).  Workgroups past the last unfolding's rows evaluate G_d.
template <int FNS, int RM>
__device__ void cores_t_body(const ProbDev *__restrict__ P, const CoreArgs &a, double *G,
                             const double *__restrict__ tab, int bid)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x, d = P->d;
    if (bid >= a.rowblocks[a.nk]) {
        core_last_fiber<FNS>(P, a, G, bid);
        return;
    }
    int u = 0;
    while (u + 1 < a.nk && bid >= a.rowblocks[u + 1]) ++u;
    const int k = u + 1;
    const KDev &K = P->kd[u];
    const int rk = a.ranks[k], nr = a.ranks[k - 1] * K.nk, nj = d - k;
    const int i0 = (bid - a.rowblocks[u]) * A4W, i = i0 + lane;
    const bool act = i < nr;
    const int p = act ? i / K.nk : 0, ik = act ? i - p * K.nk : 0;
    __shared__ int sJ[TT_MAX_RANK * TT_MAX_D];
    copy_to_lds<4, A4W>(sJ, as_global((const int *)K.Jfull), rk * nj);
    // the lane's prefix, every entry in flight at once
    int pv[TT_MAX_D];
    if (k >= 2) {
        const gptr_t<const int> preI = as_global((const int *)P->kd[u - 1].Ifull) + p * (k - 1);
#pragma unroll
        for (int j = 0; j < TT_MAX_D; ++j) pv[j] = preI[min(j, k - 2)];
    }
    // x(z): A(row, gam_z).  Hilbert: from the integer index sums, at the step
    // that reads it; else evaluated up front into LDS (Ab[z*A4W + lane]),
    // where the function can read the prefix by a runtime index
    [[maybe_unused]] double *Ab = (double *)smem_raw;
    [[maybe_unused]] long long ps = ik + 1;
    __shared__ long long sJs[TT_MAX_RANK];
    if constexpr (FNS == TT_FN_HILBERT) {
        if (k >= 2) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j)
                if (j < k - 1) ps += (long long)pv[j] + 1;
        }
        wave_sync();
        if (lane < rk) {
            long long js = 0;
            for (int j = 0; j < nj; ++j) js += sJ[lane * nj + j] + 1;
            sJs[lane] = js;
        }
    } else {
        __shared__ int sPre[A4W * TT_MAX_D];
        if (k >= 2) {
#pragma unroll
            for (int j = 0; j < TT_MAX_D; ++j)
                if (j < k - 1) sPre[lane * TT_MAX_D + j] = pv[j];
        }
        wave_sync();
        for (int z = 0; z < rk; ++z) {
            const int *Jz = sJ + z * nj;
            Ab[z * A4W + lane] = act ? fn_value_ix<double, FNS>(P->F, [&](int j) {
                return j < k - 1 ? sPre[lane * TT_MAX_D + j] : (j == k - 1 ? ik : Jz[j - k]);
            }) : 0.0;
        }
    }
    wave_sync();
    const double sh = P->F.shift;
    auto x = [&](int z) -> double {
        if constexpr (FNS == TT_FN_HILBERT) return act ? 1.0 / ((double)(ps + sJs[z]) + sh) : 0.0;
        else return Ab[z * A4W + lane];
    };
    const double *At = tab + (int64_t)u * CT_STRIDE, *Tr = At + CT_LD * CT_LD, *Dl = Tr + CT_LD * CT_LD;
    double tb[RM];
#pragma unroll
    for (int z = 0; z < RM; ++z) tb[z] = 0.0;
    tb[0] = x(0) / At[0];
#pragma unroll
    for (int z = 1; z < RM; ++z) {
        if (z < rk) {
            double dot = 0.0;
#pragma unroll
            for (int zz = 0; zz < z; ++zz) dot = __fma_rn(tb[zz], At[z * CT_LD + zz], dot);
            const double cb = Dl[z] * (dot - x(z));
#pragma unroll
            for (int zz = 0; zz < z; ++zz) tb[zz] = __fma_rn(cb, Tr[z * CT_LD + zz], tb[zz]);
            tb[z] = -cb;
        }
    }
    if (act) {
        double *row = G + a.goff[u] + (int64_t)i * rk;
#pragma unroll
        for (int z = 0; z < RM; ++z)
            if (z < rk) row[z] = tb[z];
    }
}

template <int FNS, int RM>
static __global__ void __launch_bounds__(A4W) k_cores_t(const ProbDev *__restrict__ P, CoreArgs a, double *G,
                                                        const double *__restrict__ tab)
{
    cores_t_body<FNS, RM>(P, a, G, tab, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sampled-error check (Sec. 5): over R multi-indices drawn from
// SplitMix64(seed), the sums of (X - X~)^2 and X^2, one wavefront per sample
// (lane b carries entry b of the running row vector of the TT product).
// Workgroup blk of nblk writes its two partial sums to part[2*blk..]; the
// caller adds the nblk pairs in order, so the result does not depend on
// which launch computed it.
// ---------------------------------------------------------------------------
constexpr int NBV = 128;        // workgroups per checked problem

// serr (optional): |X - X~| of every sample, in sample order.
__device__ void verify_body(const ProbDev *__restrict__ P, const double *__restrict__ G, const int *r, int64_t R,
                            uint64_t seed, double *part, int blk, int nblk, double *serr = nullptr)
{
    const int d = P->d, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // ranks, mode sizes and core offsets in LDS (indexed by the mode, they
    // would otherwise be read from scratch at every step)
    __shared__ int s_r[TT_MAX_D + 1], s_n[TT_MAX_D];
    __shared__ int64_t s_go[TT_MAX_D + 1];
    if (threadIdx.x == 0) {
        CoreArgs ca;
        int64_t len;
        make_core_args(d, P->F.n, r, ca, len);
        for (int k = 0; k <= d; ++k) { s_r[k] = r[k]; s_go[k] = ca.goff[k]; }
        for (int k = 0; k < d; ++k) s_n[k] = P->F.n[k];
    }
    __syncthreads();
    // a lane group of GL lanes per sample (GL >= every rank and >= d), so a
    // wavefront carries 64 / GL samples at once
    int rmax = d;
    for (int k = 1; k < d; ++k) rmax = max(rmax, s_r[k]);
    const int GL = rmax <= 16 ? 16 : (rmax <= 32 ? 32 : 64), spw = 64 / GL;
    const int gsub = lane / GL, gl = lane - gsub * GL;
    double num = 0.0, den = 0.0;
    const int64_t waves = (int64_t)nblk * (NT / 64), wave = (int64_t)blk * (NT / 64) + wid;
    for (int64_t t0 = wave * spw; t0 < R; t0 += waves * spw) {
        const int64_t t = t0 + gsub;
        const bool ok = t < R;
        const int ix = (ok && gl < d) ? (int)(sm64_at(seed, (uint64_t)t * d + gl) % (uint64_t)s_n[gl]) : 0;
        double v = (gl == 0) ? 1.0 : 0.0;
        for (int k = 0; k < d; ++k) {
            const int ik = __shfl(ix, k, GL), ra = s_r[k], rb = s_r[k + 1], nn = s_n[k];
            // G_k(a, i_k, b) for b = the lane (clamped to a valid column: the
            // lanes past rb drop their sums)
            const gptr_t<const double> Gk = as_global(G + s_go[k] + (int64_t)ik * rb + min(gl, rb - 1));
            const int64_t sa = (int64_t)nn * rb;
            double acc = 0.0;
            // VU terms at a time: their core entries and row-vector values are
            // all requested before the first fma (one term per round trip
            // otherwise); the fmas keep ascending a
            constexpr int VU = 8;
            for (int a0 = 0; a0 < ra; a0 += VU) {
                double g[VU], va[VU];
#pragma unroll
                for (int j = 0; j < VU; ++j) g[j] = Gk[(int64_t)min(a0 + j, ra - 1) * sa];
#pragma unroll
                for (int j = 0; j < VU; ++j) va[j] = __shfl(v, min(a0 + j, ra - 1), GL);
#pragma unroll
                for (int j = 0; j < VU; ++j)
                    if (a0 + j < ra) acc = __fma_rn(va[j], g[j], acc);
            }
            v = (gl < rb) ? acc : 0.0;
        }
        const double x = fn_value_ix<double>(P->F, [&](int j) { return __shfl(ix, j, GL); });
        if (gl == 0 && ok) {
            const double dx = x - v;
            num = __fma_rn(dx, dx, num);
            den = __fma_rn(x, x, den);
            if (serr) serr[t] = fabs(dx);
        }
    }
    // the group leaders' sums in lane order, then the wavefronts in order
    __shared__ double sn[NT / 64][64], sd[NT / 64][64];
    sn[wid][lane] = num;
    sd[wid][lane] = den;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NT / 64; ++w)
            for (int g = 0; g < spw; ++g) { a += sn[w][g * GL]; b += sd[w][g * GL]; }
        part[2 * blk] = a;
        part[2 * blk + 1] = b;
    }
}

__device__ inline void final_ranks(const ProbDev *P, int *r)
{
    const ProbState *S = P->S;
    for (int k = 0; k <= P->d; ++k) r[k] = S->r[S->sweeps & 1][k];
}

static __global__ void __launch_bounds__(NT) k_verify(const ProbDev *__restrict__ P, const double *G, int64_t R,
                                                      uint64_t seed, double *part, double *serr)
{
    int r[TT_MAX_D + 1];
    final_ranks(P, r);
    verify_body(P, G, r, R, seed, part, blockIdx.x, gridDim.x, serr);
}

// ---------------------------------------------------------------------------
// Batched launches: many independent problems in one launch.  Their
// descriptors lie contiguously in device memory; the kernel arguments name
// the problems of the launch and, for the grid-strided kernels, the range of
// workgroups each one gets.  Every problem runs the same bodies as a single
// solve, so its results are the same bit for bit.
// ---------------------------------------------------------------------------
constexpr int MAXB = 512;       // problems per batched launch

struct BatchMap {
    int na;                     // problems in this launch
    int boff[MAXB + 1];         // problem i owns workgroups [boff[i], boff[i+1])
    uint16_t p[MAXB];           // index of problem i in the descriptor array
};

__device__ inline int batch_find(const BatchMap &bm, int b)
{
    int lo = 0, hi = bm.na;     // boff[lo] <= b < boff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bm.boff[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

static __global__ void __launch_bounds__(NT) k_samples_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const ProbDev *P = Pa + bm.p[blockIdx.y];
    samples_body<0>(P, P->run.seed, P->run.ns, P->run.vals, P->run.spart, blockIdx.x, gridDim.x);
}

template <typename V>
static __global__ void __launch_bounds__(NT) k_setup_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const ProbDev *P = Pa + bm.p[blockIdx.x];
    setup_body<V, 0>(P, P->run.seed, P->run.ns, P->run.spart, P->run.eps);
}

template <typename V>
static __global__ void __launch_bounds__(NT) k_init_eval_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const ProbDev *P = Pa + bm.p[blockIdx.z];
    if ((int)blockIdx.y >= P->nk) return;
    init_eval_body<V, 0>(P, blockIdx.y, blockIdx.x, gridDim.x);
}

template <typename V>
static __global__ void __launch_bounds__(NT, 4) k_sweep_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const int i = batch_find(bm, blockIdx.x);
    const ProbDev *P = Pa + bm.p[i];
    sweep_body<V, 0>(P, P->S, P->nk, blockIdx.x - bm.boff[i], bm.boff[i + 1] - bm.boff[i]);
}

template <typename V>
static __global__ void __launch_bounds__(NTC) k_commit_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const ProbDev *P = Pa + bm.p[blockIdx.x];
    const SweepArgs none{};
    commit_body<V, 0, false>(P, P->S, P->S->sweeps, P->nk, none);
}

// Cores of every problem from its final ranks (those of its last commit).
static __global__ void __launch_bounds__(A4W) k_cores_b(const ProbDev *__restrict__ Pa, BatchMap bm)
{
    const int i = batch_find(bm, blockIdx.x);
    const ProbDev *P = Pa + bm.p[i];
    int r[TT_MAX_D + 1];
    final_ranks(P, r);
    CoreArgs a;
    int64_t len;
    make_core_args(P->d, P->F.n, r, a, len);
    cores_body<0>(P, a, P->run.cores, blockIdx.x - bm.boff[i]);
}

// Sampled-error check of every listed problem: NBV workgroups each (grid.y =
// problem), partial sums to part + 2*NBV*slot, R and the seed in run.
// The device state of each named problem copied to host memory (mapped),
// one workgroup per problem: one launch instead of a copy per problem.
static __global__ void __launch_bounds__(64) k_state_out_b(const ProbState *__restrict__ dS, ProbState *hS, BatchMap bm)
{
    if ((int)blockIdx.x >= bm.na) return;
    const int i = bm.p[blockIdx.x];
    const uint32_t *src = reinterpret_cast<const uint32_t *>(dS + i);
    uint32_t *dst = reinterpret_cast<uint32_t *>(hS + i);
    for (int w = threadIdx.x; w < (int)(sizeof(ProbState) / 4); w += 64) dst[w] = src[w];
}

static __global__ void __launch_bounds__(NT) k_verify_b(const ProbDev *__restrict__ Pa, BatchMap bm, double *part)
{
    const int slot = bm.p[blockIdx.y];
    const ProbDev *P = Pa + slot;
    int r[TT_MAX_D + 1];
    final_ranks(P, r);
    verify_body(P, P->run.cores, r, P->run.verify_R, P->run.seed + 1, part + (int64_t)2 * NBV * slot, blockIdx.x,
                gridDim.x);
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

// A lane group of GL lanes per multi-index (GL >= every rank and >= d, so a
// wavefront takes 64 / GL of them at once); lane b of a group accumulates
// entry b of the row vector, the terms in ascending a.  A step's core
// entries and row-vector values are requested TU terms at a time before the
// first fma (one term per round trip otherwise).
static __global__ void __launch_bounds__(NT) k_tt_eval(TTArgs a, const double *__restrict__ G, int64_t m,
                                                  const int *__restrict__ idx, double *__restrict__ out)
{
    const int lane = threadIdx.x & 63, d = a.d;
    int rmax = d;
    for (int k = 1; k < d; ++k) rmax = max(rmax, a.ranks[k]);
    const int GL = rmax <= 16 ? 16 : (rmax <= 32 ? 32 : 64), spw = 64 / GL;
    const int gsub = lane / GL, gl = lane - gsub * GL;
    const int64_t wave = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * NT) >> 6;
    const gptr_t<const int> IX = as_global(idx);
    const gptr_t<const double> Gg = as_global(G);
    constexpr int TU = 8;
    for (int64_t t0 = wave * spw; t0 < m; t0 += nw * spw) {
        const int64_t t = t0 + gsub;
        const bool ok = t < m;
        // lane j < d of the group holds index j of its multi-index
        const int ix = IX[(ok ? t : m - 1) * d + min(gl, d - 1)];
        double v = (gl == 0) ? 1.0 : 0.0;
        for (int kk = 0; kk < d; ++kk) {
            const int ra = a.ranks[kk], rb = a.ranks[kk + 1], nn = a.n[kk];
            const int i = __shfl(ix, kk, GL);
            // G_kk(a, i, b) for b = the lane (clamped to a valid column: the
            // lanes past rb drop their sums)
            const gptr_t<const double> Gk = Gg + (a.goff[kk] + (int64_t)i * rb + min(gl, rb - 1));
            const int64_t sa = (int64_t)nn * rb;
            double acc = 0.0;
            for (int a0 = 0; a0 < ra; a0 += TU) {
                double g[TU], va[TU];
#pragma unroll
                for (int j = 0; j < TU; ++j) g[j] = Gk[(int64_t)min(a0 + j, ra - 1) * sa];
#pragma unroll
                for (int j = 0; j < TU; ++j) va[j] = __shfl(v, min(a0 + j, ra - 1), GL);
#pragma unroll
                for (int j = 0; j < TU; ++j)
                    if (a0 + j < ra) acc = __fma_rn(va[j], g[j], acc);
            }
            v = (gl < rb) ? acc : 0.0;
        }
        if (gl == 0 && ok) out[t] = v;
    }
}

// The generating function at m multi-indices, in the arithmetic of V (the
// precision of the sweeps that would evaluate it).
// Bulk evaluation.  A workgroup takes rounds of ch = NT*EV_KP/d consecutive
// entries.  Their multi-indices (at most NT*EV_KP ints) are loaded with
// coalesced loads into registers one round ahead and stored to LDS at the
// start of the round, so the loads of round r+1 are in flight while round r
// is evaluated.  When the function's per-mode table fits (tab_lds) the
// workgroup first copies it to LDS, so every table read is an LDS read.
constexpr int EV_KP = 16;                   // index ints per thread and round
constexpr int EV_TAB_LDS_MAX = 32768;       // bytes of table copied to LDS, at most

__host__ __device__ inline size_t fn_eval_idx_bytes() { return (size_t)NT * EV_KP * sizeof(int); }

template <typename V>
static __global__ void __launch_bounds__(NT) k_fn_eval(FnDev F, int64_t m, const int *__restrict__ idx,
                                                       V *__restrict__ out, int tab_lds)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int d = F.d, tid = threadIdx.x;
    const int ch = (NT * EV_KP) / d;
    const int64_t stride = (int64_t)gridDim.x * ch;
    int *sidx = (int *)smem_raw;
    int pf[EV_KP];
    auto fetch = [&](int64_t b) {
        const int nint = (b < m) ? (int)min((int64_t)ch, m - b) * d : 0;
        const int *src = idx + (b < m ? b : 0) * d;
#pragma unroll
        for (int r = 0; r < EV_KP; ++r) {
            const int i = tid + r * NT;
            pf[r] = (i < nint) ? src[i] : 0;
        }
    };
    auto rounds = [&](const V *tb) {
        int64_t base = (int64_t)blockIdx.x * ch;
        fetch(base);
        for (; base < m; base += stride) {
            const int cnt = (int)min((int64_t)ch, m - base);
            __syncthreads();                // the previous round's reads of sidx are done
#pragma unroll
            for (int r = 0; r < EV_KP; ++r) sidx[tid + r * NT] = pf[r];
            __syncthreads();
            fetch(base + stride);
            for (int e = tid; e < cnt; e += NT) {
                const int *ix = sidx + e * d;
                out[base + e] = fn_value_tx<V>(F, [&](int j) { return ix[j]; }, tb);
            }
        }
    };
    if (tab_lds) {
        V *stab = (V *)(smem_raw + fn_eval_idx_bytes());
        const V *src = fn_table<V>(F);
        const int cnt = F.tab_rows * F.tab_ld;
        for (int i = tid; i < cnt; i += NT) stab[i] = src[i];
        // the first round's barriers order these writes before any read
        rounds(stab);
    } else {
        rounds(fn_table<V>(F));
    }
}

// Launch of k_fn_eval for m entries: the grid covers the chip eight
// workgroups per CU deep and strides over the rest.
template <typename V>
inline hipError_t launch_fn_eval(const FnDev &F, int64_t m, const int *idx, V *out, hipStream_t stream,
                                 hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr)
{
    if (m <= 0) return hipSuccess;
    const size_t tab_bytes = (size_t)F.tab_rows * F.tab_ld * sizeof(V);
    const int tab_lds = (fn_table<V>(F) && tab_bytes > 0 && tab_bytes <= EV_TAB_LDS_MAX) ? 1 : 0;
    const size_t lds = fn_eval_idx_bytes() + (tab_lds ? tab_bytes : 0);
    const int ch = (NT * EV_KP) / F.d;
    const int64_t rounds = (m + ch - 1) / ch;
    const unsigned g = (unsigned)std::min<int64_t>(rounds, 2048);
    if (ev_start && ev_stop) {
        // the events take the dispatch's own start and end timestamps
        hipExtLaunchKernelGGL(k_fn_eval<V>, dim3(g), dim3(NT), (uint32_t)lds, stream, ev_start, ev_stop, 0u, F, m,
                              idx, out, tab_lds);
    } else {
        k_fn_eval<V><<<g, NT, lds, stream>>>(F, m, idx, out, tab_lds);
    }
    return hipGetLastError();
}

static __global__ void __launch_bounds__(NT) k_gen_idx(int d, TTArgs a, uint64_t seed, int64_t m, int *idx)
{
    const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (t >= m) return;
    for (int j = 0; j < d; ++j) idx[t * d + j] = (int)(sm64_at(seed, (uint64_t)t * d + j) % (uint64_t)a.n[j]);
}

static __global__ void __launch_bounds__(NT) k_err_partial(int64_t m, const double *__restrict__ x,
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
