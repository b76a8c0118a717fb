// tt_cross.hip -- host driver and C ABI of the gfx950 greedy adaptive TT-cross
// library (declarations and contracts in include/tt_cross.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tt_cross.h"
#include "tt_device.h"
#include "tt_kernels.h"
#include "tt_internal.h"

using namespace ttc;

namespace ttc {

static thread_local std::string g_err;

int set_err(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}


// ---------------------------------------------------------------------------
// Generating function descriptors.
// ---------------------------------------------------------------------------
// Per-mode tables of the Maxwellians.  Every value is the FP64 result of the
// operations the formula applies to one index, in the formula's order, so an
// entry assembled from the table in FP64 (fn_value_ix) takes the same
// rounding steps as the formula evaluated term by term; only the final
// exponential runs on the device.  Constant factors (the (2 pi T)^{-3/2}
// terms) go to F.cst.
static void mode_tables(FnDev &F, FnHost &out)
{
    const int d = F.d;
    const double twopi = 2.0 * PI;
    int rows = 0;
    bool has[TT_MAX_D] = {false};
    switch (F.id) {
    case TT_FN_MAXWELL:            // x1, x2, x3: sin, cos, sin of 2 pi x; v1..v3: cell centres
    case TT_FN_MAXWELL_IL:         // the same atoms, modes x1, v1, x2, v2, x3, v3
        rows = 1;
        for (int j = 0; j < d; ++j) has[j] = true;
        F.cst[0] = std::pow(twopi * F.prm[2], -1.5);
        break;
    case TT_FN_BIMAXWELL:          // velocity modes: (v - u_{m,c})^2 for Maxwellian m = row
        rows = 2;
        for (int j = d - 3; j < d; ++j) has[j] = true;
        for (int m = 0; m < 2; ++m) F.cst[m] = F.prm[5 * m] * std::pow(twopi * F.prm[5 * m + 4], -1.5);
        break;
    default:                       // kinetic 2d2v / 3d3v: x modes rho/(2 sqrt(2 pi T)), 2T;
        rows = 2;                  // v modes (v - 3/4)^2, (v + 3/4)^2
        for (int j = 0; j < d; ++j) has[j] = true;
        break;
    }
    int total = 0;
    for (int j = 0; j < d; ++j) {
        F.off[j] = has[j] ? total : 0;
        if (has[j]) total += F.n[j];
    }
    F.tab_ld = total;
    F.tab_rows = rows;
    out.table.assign((size_t)rows * total, 0.0);
    double *t0 = out.table.data(), *t1 = rows > 1 ? t0 + total : nullptr;
    for (int j = 0; j < d; ++j) {
        if (!has[j]) continue;
        const int n = F.n[j];
        double *a = t0 + F.off[j], *b = t1 ? t1 + F.off[j] : nullptr;
        for (int i = 0; i < n; ++i) {
            switch (F.id) {
            case TT_FN_MAXWELL:
            case TT_FN_MAXWELL_IL: {
                // position w (0-based) of mode j, or -1 for a velocity mode
                const int w = F.id == TT_FN_MAXWELL ? (j < 3 ? j : -1) : ((j & 1) == 0 ? j / 2 : -1);
                if (w >= 0) {
                    const double x = (double)i / (double)n;
                    a[i] = (w == 1) ? std::cos(twopi * x) : std::sin(twopi * x);
                } else {
                    a[i] = vel<double>(i, n, F.prm[3]);
                }
                break;
            }
            case TT_FN_BIMAXWELL: {
                const double v = vel<double>(i, n, F.prm[10]);
                const int c = j - (d - 3);
                a[i] = (v - F.prm[1 + c]) * (v - F.prm[1 + c]);
                b[i] = (v - F.prm[6 + c]) * (v - F.prm[6 + c]);
                break;
            }
            default:
                if ((j & 1) == 0) {
                    const double x = cell<double>(i, n, -0.5, 0.5);
                    const double sx = std::sin(twopi * x);
                    const double rho = 1.0 + 0.875 * sx;
                    const double T = 0.5 + 0.4 * sx;
                    a[i] = rho / (2.0 * std::sqrt(twopi * T));
                    b[i] = 2.0 * T;
                } else {
                    const double v = cell<double>(i, n, -3.0, 3.0);
                    a[i] = (v - 0.75) * (v - 0.75);
                    b[i] = (v + 0.75) * (v + 0.75);
                }
                break;
            }
        }
    }
}

int build_fn(int fn_id, int d, const int32_t *n, const double *params, int nparams, FnHost &out)
{
    FnDev &F = out.dev;
    std::memset(&F, 0, sizeof F);
    if (d < 2 || d > TT_MAX_D) return set_err(TT_EINVAL, "d=%d outside [2,%d]", d, TT_MAX_D);
    if (!n) return set_err(TT_EINVAL, "n is NULL");
    for (int j = 0; j < d; ++j)
        if (n[j] < 1 || n[j] > (1 << 20)) return set_err(TT_EINVAL, "n[%d]=%d out of range", j, n[j]);
    if (nparams < 0 || (nparams > 0 && !params)) return set_err(TT_EINVAL, "bad params");
    F.id = fn_id;
    F.d = d;
    for (int j = 0; j < d; ++j) F.n[j] = n[j];
    out.table.clear();
    switch (fn_id) {
    case TT_FN_HILBERT:
        F.shift = (nparams >= 1) ? params[0] : (double)(1 - d);
        if (!((double)d + F.shift > 0.0)) return set_err(TT_EFN, "Hilbert denominator can be <= 0");
        break;
    case TT_FN_MAXWELL:
    case TT_FN_MAXWELL_IL:
        if (d != 6) return set_err(TT_EFN, "Maxwellian needs d=6");
        if (nparams == 0) { F.prm[0] = 0.5; F.prm[1] = 0.3; F.prm[2] = 1.0; F.prm[3] = 8.0; }
        else if (nparams >= 4) for (int i = 0; i < 4; ++i) F.prm[i] = params[i];
        else return set_err(TT_EFN, "Maxwellian params: [a,b,T,vmax]");
        if (!(F.prm[2] > 0.0) || !(F.prm[3] > 0.0)) return set_err(TT_EFN, "Maxwellian needs T>0, vmax>0");
        break;
    case TT_FN_BIMAXWELL:
        if (d < 3) return set_err(TT_EFN, "bi-Maxwellian needs d>=3");
        if (nparams < 10) return set_err(TT_EFN, "bi-Maxwellian needs 10 params");
        for (int i = 0; i < 10; ++i) F.prm[i] = params[i];
        F.prm[10] = (nparams >= 11) ? params[10] : 8.0;
        if (!(F.prm[4] > 0.0) || !(F.prm[9] > 0.0) || !(F.prm[10] > 0.0))
            return set_err(TT_EFN, "bi-Maxwellian needs T>0, vmax>0");
        break;
    case TT_FN_SEPSUM: {
        if (nparams < 1) return set_err(TT_EFN, "separable sum needs [r, g...]");
        int r = (int)params[0];
        int total = 0;
        for (int j = 0; j < d; ++j) { F.off[j] = total; total += n[j]; }
        if (r < 1 || (double)r != params[0] || nparams < 1 + r * total)
            return set_err(TT_EFN, "separable sum needs 1 + r*sum(n) params");
        F.sep_r = r;
        F.tab_ld = total;
        F.tab_rows = r;
        out.table.assign(params + 1, params + 1 + (size_t)r * total);
        break;
    }
    case TT_FN_MAXWELL_2D2V:
        if (d != 4) return set_err(TT_EFN, "2d2v Maxwellian needs d=4");
        break;
    case TT_FN_MAXWELL_3D3V:
        if (d != 6) return set_err(TT_EFN, "3d3v Maxwellian needs d=6");
        break;
    default:
        return set_err(TT_EFN, "unknown fn_id %d", fn_id);
    }
    if (fn_id != TT_FN_HILBERT && fn_id != TT_FN_SEPSUM) mode_tables(F, out);
    return TT_OK;
}

void FnHost::free_device()
{
    if (d_table) (void)hipFree(d_table);
    if (d_table32) (void)hipFree(d_table32);
    d_table = nullptr;
    d_table32 = nullptr;
    d_cap = 0;
}

int upload_fn(FnHost &fh, hipStream_t stream)
{
    fh.dev.tab = nullptr;
    fh.dev.tab32 = nullptr;
    if (fh.table.empty()) return TT_OK;
    const size_t m = fh.table.size();
    fh.table32.resize(m);
    for (size_t i = 0; i < m; ++i) fh.table32[i] = (float)fh.table[i];
    if (m > fh.d_cap) {
        // a larger table: the old buffers may still be read by queued work
        if (stream) HIPCHK(hipStreamSynchronize(stream));
        fh.free_device();
        HIPCHK(hipMalloc(&fh.d_table, m * sizeof(double)));
        HIPCHK(hipMalloc(&fh.d_table32, m * sizeof(float)));
        fh.d_cap = m;
    }
    if (stream) {
        // ordered after earlier work on the stream; the host vectors live as
        // long as the holder and change only at its next upload
        HIPCHK(hipMemcpyAsync(fh.d_table, fh.table.data(), m * sizeof(double), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(fh.d_table32, fh.table32.data(), m * sizeof(float), hipMemcpyHostToDevice, stream));
    } else {
        HIPCHK(hipMemcpy(fh.d_table, fh.table.data(), m * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(fh.d_table32, fh.table32.data(), m * sizeof(float), hipMemcpyHostToDevice));
    }
    fh.dev.tab = fh.d_table;
    fh.dev.tab32 = fh.d_table32;
    return TT_OK;
}

static int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Split one mode into tiles: blocks b = [b*n/C, (b+1)*n/C) (Sec. 3: n_j split
// evenly into C_j pieces), each cut into chunks of at most T entries.
static void mode_tiles(int n, int C, int T, std::vector<int> &start, std::vector<int> &len,
                       std::vector<int> &blk)
{
    start.clear(); len.clear(); blk.clear();
    for (int b = 0; b < C; ++b) {
        const int lo = (int)((int64_t)b * n / C), hi = (int)((int64_t)(b + 1) * n / C);
        for (int s = lo; s < hi; s += T) {
            start.push_back(s);
            len.push_back(std::min(T, hi - s));
            blk.push_back(b);
        }
    }
}

// ---------------------------------------------------------------------------
// Problem lifetime.
// ---------------------------------------------------------------------------
Problem::~Problem() { release(); }

void Problem::release()
{
    for (void *p : allocs) (void)hipFree(p);
    allocs.clear();
    for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
    prof_events.clear();
    if (hm) { (void)hipHostFree(hm); hm = nullptr; }
    if (hS_pinned) { (void)hipHostFree(hS_pinned); hS_pinned = nullptr; }
    if (h_part) { (void)hipHostFree(h_part); h_part = nullptr; }
    for (hipEvent_t &e : run_ev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
    fn.free_device();
    if (own_stream && stream) { (void)hipStreamDestroy(stream); }
    stream = nullptr;
    own_stream = false;
    allocated = false;
    dP = nullptr;
}

int Problem::dalloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_err(TT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    allocs.push_back(*p);
    return TT_OK;
}

size_t Problem::device_bytes() const
{
    size_t tot = 0;
    const size_t w = fp32 ? 4 : 8;
    for (int u = 0; u < d - 1; ++u) {
        const int k = u + 1;
        const size_t rows = (size_t)rc[k - 1] * n[k - 1], cols = (size_t)n[k] * rc[k + 1];
        tot += rows * cols * w + (size_t)rc[k] * (rows + cols) * w + rows + cols;
    }
    return tot;
}

int Problem::allocate()
{
    if (allocated) return TT_OK;
    int st;
    if (!stream) {
        if (opt.stream) {
            stream = (hipStream_t)opt.stream;
            own_stream = false;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            own_stream = true;
        }
    }
    if ((st = upload_fn(fn)) != TT_OK) return st;
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        // the search kernel's static LDS (shapes, commit scratch) comes off the top
        // (the larger of the Hilbert kernel's and the general one's)
        hipFuncAttributes fa, fh;
        if (fp32) {
            HIPCHK(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_sweep<float, 0>)));
            HIPCHK(hipFuncGetAttributes(&fh, reinterpret_cast<const void *>(&k_sweep<float, TT_FN_HILBERT>)));
        } else {
            HIPCHK(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_sweep<double, 0>)));
            HIPCHK(hipFuncGetAttributes(&fh, reinterpret_cast<const void *>(&k_sweep<double, TT_FN_HILBERT>)));
        }
        lds_static = (int)std::max(fa.sharedSizeBytes, fh.sharedSizeBytes);
    }
    const size_t w = fp32 ? 4 : 8;
    ProbDev &H = hP;
    std::memset(&H, 0, sizeof H);
    H.d = d;
    H.nk = d - 1;
    H.r_max = opt.r_max;
    H.fp32 = fp32;
    const bool rook = opt.pivot_mode == TT_PIVOT_ROOK;
    H.rook = rook ? 1 : 0;
    for (int j = 0; j < d; ++j) H.grid[j] = grid[j];
    rook_g = 1;
    if (rook) {
        // workgroups per block of the search: the option, else enough that a
        // block's rows and columns at full rank give each about 4096
        int64_t ext = 0, nblk = 0;
        for (int k = 1; k <= d - 1; ++k) {
            int64_t rb = 1, cb = 1;
            for (int j = 0; j < k; ++j) rb *= grid[j];
            for (int j = k; j < d; ++j) cb *= grid[j];
            ext = std::max(ext, (int64_t)rc[k - 1] * n[k - 1] / rb + (int64_t)n[k] * rc[k + 1] / cb);
            nblk += rb * cb;
        }
        if (opt.rook_split > 0) {
            rook_g = opt.rook_split;
        } else if (ext >= 8192) {
            rook_g = (int)std::min<int64_t>(64, ext / 4096);
            rook_g = (int)std::max<int64_t>(2, std::min<int64_t>(rook_g, 8192 / std::max<int64_t>(1, nblk)));
        }
        if (nblk * rook_g > ((int64_t)1 << 30))
            return set_err(TT_EINVAL, "%lld subtensor blocks x %d workgroups each is too many for one launch",
                           (long long)nblk, rook_g);
    }
    H.rook_g = rook_g;
    H.F = fn.dev;
    int rcmax = 1;
    for (int k = 0; k <= d; ++k) rcmax = std::max(rcmax, rc[k]);
    H.rcap = rcmax;
    hist_cap = 2;
    for (int k = 1; k <= d - 1; ++k) hist_cap += rc[k];
    H.hist_cap = hist_cap;
    max_sweeps = hist_cap;
    int64_t cores_cap = 0;
    for (int u = 0; u < d - 1; ++u) {
        const int k = u + 1;
        KDev &K = H.kd[u];
        K.k = k;
        K.nk = n[k - 1];
        K.nk1 = n[k];
        // positions are 32-bit (and a search key packs a row and a column)
        if ((int64_t)rc[k - 1] * n[k - 1] > INT32_MAX || (int64_t)n[k] * rc[k + 1] > INT32_MAX)
            return set_err(TT_EINVAL, "superblock %d would have more than 2^31-1 rows or columns", k);
        K.rowcap = rc[k - 1] * n[k - 1];
        K.colcap = n[k] * rc[k + 1];
        {
            // rows of E start 256 bytes past a multiple of 512, so that the
            // rows of a tile spread over the HBM channels instead of landing
            // on one when the capacity is a power of two
            const int per256 = (int)(256 / w);
            K.ld = ((K.colcap + 2 * per256 - 1) / (2 * per256)) * (2 * per256) + per256;
        }
        K.rk_cap = rc[k];
        // tile geometry: rows of mode k, columns of mode k+1.  A tile lies in
        // one run of i_k (i_{k+1}) inside a subtensor block.  Default height,
        // from measured sweeps of shapes: 256 rows when both runs are long
        // (>= 400), where a stored tile (one wavefront's work) gains from
        // streaming longer and the new-entry tiles are still many; 64 rows
        // for d >= 4 with runs >= 100; else 32.  (With d = 3, each new prefix
        // adds a whole row of long new-entry tiles, which taller tiles make
        // fewer and slower.)  Other shapes are found by tt_autotune.
        auto longest_run = [&](int nn, int C) {
            int m = 1;
            for (int b = 0; b < C; ++b) m = std::max(m, (int)((int64_t)(b + 1) * nn / C - (int64_t)b * nn / C));
            return m;
        };
        const int runr = longest_run(n[k - 1], grid[k - 1]), maxrun = longest_run(n[k], grid[k]);
        int TR = req_tr > 0 ? req_tr : ((runr >= 400 && maxrun >= 400) ? 256 : (d >= 4 && runr >= 100) ? 64 : 32);
        // stored tiles put 64 / TC rows on a wavefront: TC <= 64
        int TC = req_tc > 0 ? req_tc : std::min(64, pow2_at_least(maxrun));
        TC = std::min(pow2_at_least(TC), 64);
        if (req_tr <= 0 && req_tc <= 0) {
            // shrink the default tile until its LDS fits next to the rank
            // cap: the height first down to 32 rows, then the width
            while (sweep_lds_bytes(rc[k], TR, TC, w) + lds_static > (size_t)lds_limit && (TC > 16 || TR > 8)) {
                if (TR > 32) TR /= 2;
                else if (TC > 16) TC /= 2;
                else TR /= 2;
            }
        }
        std::vector<int> rs, rl, rb, cs, cl, cb;
        mode_tiles(n[k - 1], grid[k - 1], TR, rs, rl, rb);
        mode_tiles(n[k], grid[k], TC, cs, cl, cb);
        if (!rook && sweep_lds_bytes(rc[k], TR, TC, w) + lds_static > (size_t)lds_limit)
            return set_err(TT_EINVAL, "tile %dx%d with rank cap %d needs more LDS than a workgroup has (%d B)",
                           TR, TC, rc[k], lds_limit);
        K.RTp = (int)rs.size();
        K.CTq = (int)cs.size();
        K.TR = TR;
        K.TC = TC;
        tileTR[u] = TR;
        tileTC[u] = TC;
        int *tabs;
        if ((st = dalloc((void **)&tabs, sizeof(int) * 3 * (rs.size() + cs.size()))) != TT_OK) return st;
        std::vector<int> all;
        all.insert(all.end(), rs.begin(), rs.end());
        all.insert(all.end(), rl.begin(), rl.end());
        all.insert(all.end(), rb.begin(), rb.end());
        all.insert(all.end(), cs.begin(), cs.end());
        all.insert(all.end(), cl.begin(), cl.end());
        all.insert(all.end(), cb.begin(), cb.end());
        HIPCHK(hipMemcpy(tabs, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice));
        const int R = K.RTp, Cc = K.CTq;
        K.rt_start = tabs; K.rt_len = tabs + R; K.rt_blk = tabs + 2 * R;
        K.ct_start = tabs + 3 * R; K.ct_len = tabs + 3 * R + Cc; K.ct_blk = tabs + 3 * R + 2 * Cc;
        const int rk = rc[k];
        if (rook) {
            // factors W (rows x rank) and U (rank x columns) instead of the residual
            K.E = nullptr;
            const size_t fp = (size_t)factor_pitch(rk);
            if ((st = dalloc((void **)&K.Wf, sizeof(double) * K.rowcap * fp)) != TT_OK) return st;
            if ((st = dalloc((void **)&K.Uf, sizeof(double) * fp * K.colcap)) != TT_OK) return st;
            K.nrb = 1;
            K.ncb = 1;
            for (int j = 0; j < k; ++j) K.nrb *= grid[j];
            for (int j = k; j < d; ++j) K.ncb *= grid[j];
            if ((int64_t)K.nrb * K.ncb > (1 << 24)) return set_err(TT_EINVAL, "more than 2^24 subtensor blocks");
            if ((st = dalloc((void **)&K.bcnt, sizeof(unsigned long long) * K.nrb * K.ncb)) != TT_OK) return st;
            if (rook_g > 1) {
                const size_t nb = (size_t)K.nrb * K.ncb;
                if ((st = dalloc((void **)&K.rpart, sizeof(Cand) * 2 * nb * rook_g)) != TT_OK) return st;
                if ((st = dalloc((void **)&K.rst, sizeof(RookState) * 2 * nb)) != TT_OK) return st;
                if ((st = dalloc((void **)&K.rcnt, sizeof(unsigned long long) * nb * rook_g)) != TT_OK) return st;
            }
        } else if ((st = dalloc(&K.E, (size_t)K.rowcap * K.ld * w)) != TT_OK) {
            return st;
        }
        // whole 32-bit words: the search reads row masks as aligned words
        if ((st = dalloc((void **)&K.rpiv, ((size_t)K.rowcap + 3) & ~(size_t)3)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.cpiv, ((size_t)K.colcap + 3) & ~(size_t)3)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.Ifull, sizeof(int) * rk * k)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.Jfull, sizeof(int) * rk * (d - k))) != TT_OK) return st;
        if ((st = dalloc((void **)&K.rho, sizeof(int) * rk)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.gam, sizeof(int) * rk)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.piv, sizeof(double) * rk)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.piv64, sizeof(double) * rk)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.Wp64, sizeof(double) * rcmax * rcmax)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.Up64, sizeof(double) * rcmax * rcmax)) != TT_OK) return st;
        K.cand_cap = rook ? K.nrb * K.ncb : (rc[k - 1] * K.RTp) * (rc[k + 1] * K.CTq);
        if ((st = dalloc((void **)&K.cand, sizeof(Cand) * K.cand_cap)) != TT_OK) return st;
        if ((st = dalloc((void **)&K.hist, sizeof(double) * hist_cap)) != TT_OK) return st;
        cores_cap += (int64_t)rc[k - 1] * n[k - 1] * rc[k];
    }
    cores_cap += (int64_t)rc[d - 1] * n[d - 1];
    if ((st = dalloc((void **)&d_cores, sizeof(double) * cores_cap)) != TT_OK) return st;
    if ((st = dalloc((void **)&d_ctab, sizeof(double) * CT_STRIDE * (d - 1))) != TT_OK) return st;
    if ((st = dalloc((void **)&d_vals, sizeof(double) * opt.n_samples)) != TT_OK) return st;
    if ((st = dalloc((void **)&d_spart, sizeof(SamplePart) * sample_blocks(opt.n_samples))) != TT_OK) return st;
    if ((st = dalloc((void **)&d_part, sizeof(double) * 2 * NBV)) != TT_OK) return st;
    if ((st = dalloc((void **)&d_plan, sizeof(SeedPlan))) != TT_OK) return st;
    HIPCHK(hipMemset(d_plan, 0, sizeof(SeedPlan)));
    dev_plan_npts = 0;
    H.plan = d_plan;
    if ((st = dalloc((void **)&d_pc, sizeof(PointCheck))) != TT_OK) return st;
    if ((st = dalloc((void **)&d_pres, sizeof(double) * TT_RESTART_TRIES * TT_MAX_D)) != TT_OK) return st;
    serr_cap = 0;
    d_serr = nullptr;
    if ((st = dalloc((void **)&H.S, sizeof(ProbState))) != TT_OK) return st;
#ifdef TT_STAMPS
    // phase stamps: one record per search workgroup and sweep, one per commit
    H.stamp_wgs = sweep_grid_cap;
    H.stamp_sweeps = max_sweeps;
    stamp_words = (size_t)max_sweeps * (sweep_grid_cap + 1) * STAMP_WORDS;
    if ((st = dalloc((void **)&H.stamps, sizeof(unsigned long long) * stamp_words)) != TT_OK) return st;
#endif
    HIPCHK(hipHostMalloc((void **)&hm, sizeof(HostMirror), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&H.hm, hm, 0));
    for (int u = 0; u < d - 1; ++u) {
        const KDev &K = H.kd[u];
        KTile &T = H.kt[u];
        T.nk = K.nk; T.nk1 = K.nk1; T.ld = K.ld; T.RTp = K.RTp; T.CTq = K.CTq; T.TR = K.TR; T.TC = K.TC;
        T.pad = 0;
        T.rt_start = K.rt_start; T.rt_len = K.rt_len; T.ct_start = K.ct_start; T.ct_len = K.ct_len;
        T.E = K.E; T.rpiv = K.rpiv; T.cpiv = K.cpiv; T.rho = K.rho; T.gam = K.gam; T.piv = K.piv;
        T.Ifull = K.Ifull; T.Jfull = K.Jfull;
        T.Ipre = u >= 1 ? H.kd[u - 1].Ifull : nullptr;
        T.Jsuf = u + 1 < d - 1 ? H.kd[u + 1].Jfull : nullptr;
        T.cand = K.cand;
    }
    // the first sweep searches the initial superblocks (one prefix, one
    // suffix, every tile stored): its tile counts are fixed by the geometry
    std::memset(&H.sh0, 0, sizeof H.sh0);
    for (int u = 0, acc = 0; u < d - 1; ++u) {
        const KDev &K = H.kd[u];
        H.sh0.RT[u] = H.sh0.RTs[u] = K.RTp;
        H.sh0.CT[u] = H.sh0.CTs[u] = K.CTq;
        H.sh0.soff[u] = acc;
        acc += K.RTp * K.CTq;
        H.sh0.soff[u + 1] = acc;
    }
    if ((st = dalloc((void **)&dP, sizeof(ProbDev))) != TT_OK) return st;
    HIPCHK(hipMemcpy(dP, &H, sizeof(ProbDev), hipMemcpyHostToDevice));
    allocated = true;
    return TT_OK;
}

void Problem::resolve_geometry()
{
    // rank capacity per unfolding: r_k <= min(prod n_{<=k}, prod n_{>k}, r_max)
    rc[0] = rc[d] = 1;
    for (int k = 1; k <= d - 1; ++k) {
        double left = 1, right = 1;
        for (int j = 0; j < k; ++j) left *= n[j];
        for (int j = k; j < d; ++j) right *= n[j];
        double m = std::min(std::min(left, right), (double)opt.r_max);
        if (kcap[k] > 0) m = std::min(m, (double)kcap[k]);
        rc[k] = (int)m;
    }
    for (int j = 0; j < d; ++j) grid[j] = std::max(1, std::min(opt.grid[j], n[j]));
    int prec = opt.precision;
    if (prec == TT_PREC_AUTO) prec = (eps >= 1e-6) ? TT_PREC_FP32 : TT_PREC_FP64;
    if (force_fp64 || opt.pivot_mode == TT_PIVOT_ROOK) prec = TT_PREC_FP64;
    fp32 = (prec == TT_PREC_FP32) ? 1 : 0;
    req_tr = opt.tile_rows;
    req_tc = opt.tile_cols;
    if (req_tr == 0 && req_tc == 0 && use_table) tuned_tiles(*this, req_tr, req_tc);
}

// ---------------------------------------------------------------------------
// A run as a sequence of steps.  tt_cross_run_async starts it, tt_cross_query
// advances it without blocking, tt_cross_wait advances it to the end;
// tt_cross_run is the first and the last in a row, so every run issues the
// same launches in the same order.  The steps:
//   1. samples, setup and the initial superblocks, then sweeps queued up to
//      opt.lookahead ahead of the host's view of the device's progress (the
//      commit kernels write it to mapped host memory);
//   2. once the device reports the stop (or the sweep cap is reached): the
//      cores (Alg. 4) and a copy of the final state to pinned host memory;
//   3. the sampled-error check of the precision policy, if this run has one;
//      an FP32 run that misses eps is escalated to FP64 sweeps (back to 1).
// advance(wait = false) returns as soon as the next step needs the device to
// get further than it has.
// ---------------------------------------------------------------------------
template <typename V> int Problem::begin_sweeps()
{
    const int nk = d - 1;
    // events and the pinned copies are kept with the problem: nothing is
    // created or destroyed per run
    if (!run_ev[0]) HIPCHK(hipEventCreate(&run_ev[0]));
    if (!run_ev[1]) HIPCHK(hipEventCreate(&run_ev[1]));
    if (!run_ev[2]) HIPCHK(hipEventCreateWithFlags(&run_ev[2], hipEventDisableTiming));
    if (!hS_pinned) HIPCHK(hipHostMalloc((void **)&hS_pinned, sizeof(ProbState), hipHostMallocDefault));
    if (!h_part) HIPCHK(hipHostMalloc((void **)&h_part, sizeof(double) * 2 * NBV, hipHostMallocDefault));
    hm->sweeps_done = 0;
    hm->stop = 0;
    hm->err = 0;
    std::atomic_thread_fence(std::memory_order_seq_cst);
#ifdef TT_STAMPS
    HIPCHK(hipMemsetAsync(hP.stamps, 0, sizeof(unsigned long long) * stamp_words, stream));
#endif
    // a restarted run's initial pivots (the device copy says npts = 0 for a
    // plain run; it changes only when the run's kind does)
    if (h_plan.npts > 0 || dev_plan_npts != 0) {
        HIPCHK(hipMemcpyAsync(d_plan, &h_plan, sizeof(SeedPlan), hipMemcpyHostToDevice, stream));
        dev_plan_npts = h_plan.npts;
    }
    HIPCHK(hipEventRecord(run_ev[0], stream));
    // a1: samples -> rms, tau, first pivot; initial superblocks (the sample
    // kernel also clears the pivot maps)
    const int ns = opt.n_samples;
    const bool hil = fn.dev.id == TT_FN_HILBERT;     // kernels built for the Hilbert tensor alone
    if (hil) {
        k_samples<TT_FN_HILBERT><<<sample_blocks(ns), NT, 0, stream>>>(dP, opt.seed, ns, d_vals, d_spart);
        k_setup<V, TT_FN_HILBERT><<<1, NT, 0, stream>>>(dP, opt.seed, ns, d_spart, eps);
    } else {
        k_samples<0><<<sample_blocks(ns), NT, 0, stream>>>(dP, opt.seed, ns, d_vals, d_spart);
        k_setup<V, 0><<<1, NT, 0, stream>>>(dP, opt.seed, ns, d_spart, eps);
    }
    if (opt.pivot_mode != TT_PIVOT_ROOK && h_plan.npts == 0) {     // a restarted run's first sweep evaluates them
        int maxe = 1;
        for (int u = 0; u < nk; ++u) maxe = std::max(maxe, n[u] * n[u + 1]);
        dim3 g((unsigned)std::min(1024, (maxe + NT - 1) / NT), (unsigned)nk);
        if (hil) k_init_eval<V, TT_FN_HILBERT><<<g, NT, 0, stream>>>(dP);
        else k_init_eval<V, 0><<<g, NT, 0, stream>>>(dP);
    }
    HIPCHK(hipGetLastError());
    // rank bounds of the first sweep: 1, or a restarted run's initial pivot
    // counts (and nothing stored yet)
    for (int k = 0; k <= d; ++k) rub[k] = rst[k] = 1;
    if (h_plan.npts > 0)
        for (int k = 1; k <= d - 1; ++k) {
            rub[k] = h_plan.m[k - 1];
            rst[k] = 0;
        }
    launched = 0;
    done_known = 0;
    if (opt.profile) {
        while ((int)prof_events.size() < 3 * max_sweeps) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            prof_events.push_back(e);
        }
    }
    return launch_ahead<V>();
}

// Queue sweeps (search + commit) until opt.lookahead of them are ahead of the
// last one the device reported done.  rub bounds each unfolding's rank in the
// sweep being queued; rst that of its stored region.
template <typename V> int Problem::launch_ahead()
{
    const int nk = d - 1;
    const bool hil = fn.dev.id == TT_FN_HILBERT;
    const bool rook = opt.pivot_mode == TT_PIVOT_ROOK;
    const bool prof = opt.profile != 0;
    int rook_wgs = 0;                          // search workgroups: G per subtensor block
    if (rook)
        for (int u = 0; u < nk; ++u) rook_wgs += hP.kd[u].nrb * hP.kd[u].ncb;
    const int rook_blocks = rook_wgs;
    rook_wgs *= rook_g;
    const int L = std::max(1, opt.lookahead);
    while (launched < done_known + L && launched < max_sweeps) {
        SweepArgs a;
        std::memset(&a, 0, sizeof a);
        a.sweep = launched;
        a.nk = nk;
        a.S = hP.S;
        int units = 0;
        size_t lds = 0;
        for (int u = 0; u < nk; ++u) {
            const int k = u + 1;
            const KDev &K = hP.kd[u];
            const int all = rub[k - 1] * K.RTp * rub[k + 1] * K.CTq;
            // the commit's first round of candidates: at most this many
            a.cand[u] = K.cand;
            a.ntl_max[u] = rook ? K.nrb * K.ncb : all;
            const int st = std::min(all, rst[k - 1] * K.RTp * rst[k + 1] * K.CTq);
            units += (all - st) + (st + NT / 64 - 1) / (NT / 64);
            lds = std::max(lds, sweep_lds_bytes(rub[k], K.TR, K.TC, sizeof(V)));
        }
        // one workgroup per expected work unit (new tiles one each, stored
        // tiles four each); the kernel strides over the exact unit count it
        // reads on the device, so a wrong estimate costs time only
        const int grid = std::max(1, std::min(units, sweep_grid_cap));
        for (int k = 0; k <= d; ++k) rst[k] = rub[k];
        // the Hilbert tensor gets a kernel built for it alone (fewer
        // registers, more workgroups resident); the others share one
        auto kern = hil ? k_sweep<V, TT_FN_HILBERT> : k_sweep<V, 0>;
        if (rook) {
            // factors: one thread per superblock row and column (bounded by
            // the ranks this sweep can have), then one workgroup per block
            int items = 0;
            for (int u = 0; u < nk; ++u) items += rub[u] * n[u] + n[u + 1] * rub[u + 2];
            const int gf = std::max(1, std::min((items + NT - 1) / NT, 4096));
            if (hil) k_rook_factors<TT_FN_HILBERT><<<gf, NT, 0, stream>>>(dP, a);
            else k_rook_factors<0><<<gf, NT, 0, stream>>>(dP, a);
            // profiling: events around the search launches of the sweep
            if (prof) HIPCHK(hipEventRecord(prof_events[3 * launched], stream));
            if (rook_g == 1) {
                if (hil) k_rook_search<TT_FN_HILBERT><<<rook_wgs, NT, 0, stream>>>(dP, a, opt.seed);
                else k_rook_search<0><<<rook_wgs, NT, 0, stream>>>(dP, a, opt.seed);
            } else {
                // split search: samples, then a fixed sequence of column
                // and row steps (blocks that are done return at once)
                if (hil) k_rook_wsample<TT_FN_HILBERT><<<rook_wgs, NT, 0, stream>>>(dP, a, opt.seed);
                else k_rook_wsample<0><<<rook_wgs, NT, 0, stream>>>(dP, a, opt.seed);
                for (int ph = 1; ph <= 2 * TT_ROOK_ITERS; ++ph) {
                    if (hil) k_rook_wstep<TT_FN_HILBERT><<<rook_wgs, NT, 0, stream>>>(dP, a, ph);
                    else k_rook_wstep<0><<<rook_wgs, NT, 0, stream>>>(dP, a, ph);
                }
                // the finishing launch also completes any walk still moving
                if (hil) k_rook_wfinish<TT_FN_HILBERT><<<rook_blocks, NT, 0, stream>>>(dP, a);
                else k_rook_wfinish<0><<<rook_blocks, NT, 0, stream>>>(dP, a);
            }
            if (prof) HIPCHK(hipEventRecord(prof_events[3 * launched + 1], stream));
        } else if (prof) {
            // the events take the dispatch's own start and end timestamps
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(NT), (uint32_t)lds, stream,
                                  prof_events[3 * launched], prof_events[3 * launched + 1], 0u, dP, a);
        } else {
            kern<<<grid, NT, lds, stream>>>(dP, a);
        }
        ++launched;
        for (int k = 1; k <= d - 1; ++k) rub[k] = std::min(rub[k] + 1, rc[k]);
        if (hil) k_commit<V, TT_FN_HILBERT><<<1, NTC, 0, stream>>>(dP, a);
        else k_commit<V, 0><<<1, NTC, 0, stream>>>(dP, a);
    }
    HIPCHK(hipGetLastError());
    return TT_OK;
}

// Step 1: follow the device's sweeps and keep the queue filled.  Returns 0
// while sweeping (wait = false only), 1 once the cores and the final-state
// copy are queued, or an error.
template <typename V> int Problem::poll_sweeps(bool wait)
{
    // the mapped counter is read in a tight loop; the stream itself (to see
    // that it drained without a new count, or failed) is queried only after
    // 50 us without progress, so that a waiting host reacts to the device
    // at the speed of a memory read
    auto t_last = std::chrono::steady_clock::now();
    for (;;) {
        bool progressed = false, stopped = false;
        const int sd = __atomic_load_n(&hm->sweeps_done, __ATOMIC_ACQUIRE);
        if (sd > done_known) {
            done_known = sd;
            progressed = true;
            t_last = std::chrono::steady_clock::now();
        } else if (wait && std::chrono::steady_clock::now() - t_last < std::chrono::microseconds(50)) {
            continue;
        } else {
            t_last = std::chrono::steady_clock::now();
            hipError_t q = hipStreamQuery(stream);
            if (q != hipErrorNotReady) {
                if (q != hipSuccess) return set_err(TT_EDEVICE, "sweep failed: %s", hipGetErrorString(q));
                const int sd2 = __atomic_load_n(&hm->sweeps_done, __ATOMIC_ACQUIRE);
                if (sd2 > done_known) {
                    done_known = sd2;
                    progressed = true;
                } else {
                    stopped = true;      // stream idle: every queued sweep has run
                }
            }
        }
        if (!progressed && !stopped) {
            if (!wait) return 0;
            continue;
        }
        if (__atomic_load_n(&hm->stop, __ATOMIC_ACQUIRE)) stopped = true;
        if (launched >= max_sweeps && done_known >= launched) stopped = true;
        if (stopped) return launch_tail<V>();
        for (int k = 1; k <= d - 1; ++k)
            rub[k] = std::min(rc[k], __atomic_load_n(&hm->r[k], __ATOMIC_RELAXED) + (launched - done_known));
        const int st = launch_ahead<V>();
        if (st != TT_OK) return st;
    }
}

// Step 2: the cores by Alg. 4 in FP64, then the final state's copy.
template <typename V> int Problem::launch_tail()
{
    // ranks of the final sweep come from the host mirror; without the stop
    // flag's release they are read only after the stream has drained
    if (!__atomic_load_n(&hm->stop, __ATOMIC_ACQUIRE)) HIPCHK(hipStreamSynchronize(stream));
    for (int k = 0; k <= d; ++k) ranks_now[k] = __atomic_load_n(&hm->r[k], __ATOMIC_RELAXED);
    ranks_now[0] = ranks_now[d] = 1;
    if (hm->err) {
        HIPCHK(hipStreamSynchronize(stream));
        return set_err(hm->err, "device reported error %d during the sweeps", hm->err);
    }
    CoreArgs ca;
    std::memset(&ca, 0, sizeof ca);
    int maxr = 1;
    for (int k = 1; k <= d - 1; ++k) maxr = std::max(maxr, ranks_now[k]);
    const int blocks = make_core_args(d, n, ranks_now, ca, cores_len);
    const bool hil = fn.dev.id == TT_FN_HILBERT;
    if (maxr > 16) {
        // above rank 16 the pivot rows' recursion runs once per unfolding and
        // the fiber rows keep their T in registers (same operations, same bits)
        const size_t lp = sizeof(double) * (size_t)2 * maxr * (maxr + 1),
                     lt = hil ? 0 : sizeof(double) * (size_t)maxr * A4W;
        if (lp > (size_t)lds_limit) return set_err(TT_EINVAL, "rank %d too large for the core kernel", maxr);
        if (hil) k_core_piv<TT_FN_HILBERT><<<d - 1, A4W, lp, stream>>>(dP, ca, d_ctab);
        else k_core_piv<0><<<d - 1, A4W, lp, stream>>>(dP, ca, d_ctab);
        HIPCHK(hipGetLastError());
        if (maxr <= 32) {
            if (hil) k_cores_t<TT_FN_HILBERT, 32><<<blocks, A4W, lt, stream>>>(dP, ca, d_cores, d_ctab);
            else k_cores_t<0, 32><<<blocks, A4W, lt, stream>>>(dP, ca, d_cores, d_ctab);
        } else {
            if (hil) k_cores_t<TT_FN_HILBERT, TT_MAX_RANK><<<blocks, A4W, lt, stream>>>(dP, ca, d_cores, d_ctab);
            else k_cores_t<0, TT_MAX_RANK><<<blocks, A4W, lt, stream>>>(dP, ca, d_cores, d_ctab);
        }
    } else {
        const size_t lc = sizeof(double) * ((size_t)2 * maxr * (maxr + 1) + (size_t)2 * maxr * A4W);
        if (hil) k_cores<TT_FN_HILBERT><<<blocks, A4W, lc, stream>>>(dP, ca, d_cores);
        else k_cores<0><<<blocks, A4W, lc, stream>>>(dP, ca, d_cores);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(run_ev[1], stream));
    HIPCHK(hipMemcpyAsync(hS_pinned, hP.S, sizeof(ProbState), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipEventRecord(run_ev[2], stream));
    phase = PH_TAIL;
    return 1;
}

// Waits for (wait = true) or checks run_ev[2]: 1 done, 0 not yet, < 0 error.
int Problem::tail_event(bool wait)
{
    if (wait) {
        HIPCHK(hipEventSynchronize(run_ev[2]));
        return 1;
    }
    const hipError_t q = hipEventQuery(run_ev[2]);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return set_err(TT_EDEVICE, "run failed: %s", hipGetErrorString(q));
    return 1;
}

// Step 2 done: results from the final state; then step 3 is queued if the
// run has a sampled-error check.
int Problem::poll_tail(bool wait)
{
    int st = tail_event(wait);
    if (st <= 0) return st;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, run_ev[0], run_ev[1]));
    time_to_eps = ms * 1e-3 + t_first;
    const ProbState S = *hS_pinned;
    if (S.err) return set_err(S.err, "device reported error %d", S.err);
    finalize(S, ranks_now);
    sweep_launches = 0;
    sweep_kernel_s = sweep_phase_s = 0;
    if (opt.profile) {
        for (int s = 0; s < S.sweeps && s < launched; ++s) {
            float a = 0.f;
            HIPCHK(hipEventElapsedTime(&a, prof_events[3 * s], prof_events[3 * s + 1]));
            sweep_kernel_s += a * 1e-3;
            ++sweep_launches;
        }
        if (sweep_launches > 0) {
            float c = 0.f;
            HIPCHK(hipEventElapsedTime(&c, prof_events[0], prof_events[3 * (sweep_launches - 1) + 1]));
            sweep_phase_s = c * 1e-3;
        }
    }
    const int64_t R = verify_samples();
    if (R > 0) {
        // a13: sampled relative error over an independent SplitMix64(seed + 1)
        // set; with restarts on, every sample's error as well
        double *serr = nullptr;
        if (restarts_on()) {
            if (serr_cap < R) {
                if ((st = dalloc((void **)&d_serr, sizeof(double) * R)) != TT_OK) return st;
                serr_cap = R;
            }
            serr = d_serr;
        }
        k_verify<<<NBV, NT, 0, stream>>>(dP, d_cores, R, opt.seed + 1, d_part, serr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h_part, d_part, sizeof(double) * 2 * NBV, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipEventRecord(run_ev[2], stream));
        phase = PH_VERIFY;
    } else {
        phase = PH_DONE;
    }
    return 1;
}

// Step 3 done: the check's error; an FP32 run that missed eps starts again
// with FP64 sweeps.
int Problem::poll_verify(bool wait)
{
    int st = tail_event(wait);
    if (st <= 0) return st;
    // partial sums of the NBV workgroups, added in order on the host
    double num = 0.0, den = 0.0;
    for (int b = 0; b < NBV; ++b) { num += h_part[2 * b]; den += h_part[2 * b + 1]; }
    const double err = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
    sampled_err = err;
    if (err > eps && auto_fp32()) {
        // a13: the FP32 sweeps missed eps; solve again with FP64 sweeps
        t_first = time_to_eps;
        force_fp64 = true;
        escalated = 1;
        if ((st = prepare()) != TT_OK) return st;
        cur_fp32 = false;
        if ((st = begin_sweeps<double>()) != TT_OK) return st;
        phase = PH_SWEEPS;
        return 1;
    }
    if (err > eps && status == TT_OK && restarts_on()) {
        bool restarted = false;
        if ((st = try_restart(restarted)) != TT_OK) return st;
        if (restarted) return 1;
    }
    if (err > eps && status == TT_OK) status = TT_WARN_SAMPLED_ERR;
    phase = PH_DONE;
    return 1;
}

// ---------------------------------------------------------------------------
// Restarts after false convergence (not in the paper; the rule is written
// out with tt_options.restarts).  Host work is index bookkeeping only: which
// unfoldings a point enters, pivot positions, the order of the candidates;
// every value (residuals, errors) comes from the kernels.
// ---------------------------------------------------------------------------
// Index sets of h_plan's point list: unfolding u holds the points that
// entered it, in list order, and their pivot positions.  Returns an error if
// a position is missing (nested sets rule that out; the plan is then not
// used).
int Problem::plan_from_points()
{
    SeedPlan &pl = h_plan;
    const int nk = d - 1;
    for (int u = 0; u < nk; ++u) pl.m[u] = 0;
    for (int p = 0; p < pl.npts; ++p) {
        const int in = point_levels(pl.pts[p]);
        for (int u = 0; u < nk; ++u)
            if ((in >> u) & 1) pl.mem[u][pl.m[u]++] = p;
    }
    // a prefix's place in unfolding u-1, a suffix's in unfolding u+1
    auto pre_pos = [&](int u, const int *pt) {
        if (u == 0) return 0;
        for (int z = 0; z < pl.m[u - 1]; ++z)
            if (std::equal(pt, pt + u, pl.pts[pl.mem[u - 1][z]])) return z;
        return -1;
    };
    auto suf_pos = [&](int u, const int *pt) {
        if (u == nk - 1) return 0;
        const int k = u + 1;
        for (int z = 0; z < pl.m[u + 1]; ++z)
            if (std::equal(pt + k + 1, pt + d, pl.pts[pl.mem[u + 1][z]] + k + 1)) return z;
        return -1;
    };
    for (int u = 0; u < nk; ++u) {
        const int k = u + 1;
        if (pl.m[u] < 1 || pl.m[u] > rc[k]) return set_err(TT_EINVAL, "restart plan: %d pivots in unfolding %d", pl.m[u], k);
        for (int z = 0; z < pl.m[u]; ++z) {
            const int *pt = pl.pts[pl.mem[u][z]];
            const int pp = pre_pos(u, pt), qq = suf_pos(u, pt);
            if (pp < 0 || qq < 0) return set_err(TT_EINVAL, "restart plan: index sets not nested at unfolding %d", k);
            pl.rho[u][z] = pp * n[k - 1] + pt[k - 1];
            pl.gam[u][z] = qq * n[k] + pt[k];
        }
    }
    return TT_OK;
}

// Unfoldings (bit u) point pt enters after h_plan's points: those where
// neither its prefix nor its suffix is present.  A point with unfoldings
// that are not one run, or that would pass a rank capacity, enters none.
int Problem::point_levels(const int *pt) const
{
    const SeedPlan &pl = h_plan;
    const int nk = d - 1;
    int in = 0, first = -1, last = -1, cnt = 0;
    for (int u = 0; u < nk; ++u) {
        const int k = u + 1;
        bool pre = false, suf = false;
        for (int z = 0; z < pl.m[u]; ++z) {
            const int *q = pl.pts[pl.mem[u][z]];
            pre = pre || std::equal(pt, pt + k, q);
            suf = suf || std::equal(pt + k, pt + d, q + k);
        }
        if (!pre && !suf) {
            if (pl.m[u] >= rc[k]) return 0;
            in |= 1 << u;
            if (first < 0) first = u;
            last = u;
            ++cnt;
        }
    }
    return (cnt > 0 && last - first + 1 != cnt) ? 0 : in;
}

// Residuals of nc candidate points against h_plan's index sets (device,
// k_point_resid); res[c][u] < 0 where candidate c does not enter u.
int Problem::restart_check(int nc, const int (*cand)[TT_MAX_D], const int *cin, double (*res)[TT_MAX_D])
{
    PointCheck pc;
    std::memset(&pc, 0, sizeof pc);
    pc.nc = nc;
    for (int c = 0; c < nc; ++c) {
        std::memcpy(pc.cand[c], cand[c], sizeof pc.cand[c]);
        pc.cin[c] = cin[c];
    }
    HIPCHK(hipMemcpyAsync(d_plan, &h_plan, sizeof(SeedPlan), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(d_pc, &pc, sizeof(PointCheck), hipMemcpyHostToDevice, stream));
    const int waves = nc * (d - 1), blocks = (waves + NT / 64 - 1) / (NT / 64);
    if (blocks > 0) {
        if (fn.dev.id == TT_FN_HILBERT) k_point_resid<TT_FN_HILBERT><<<blocks, NT, 0, stream>>>(dP, d_plan, d_pc, d_pres);
        else k_point_resid<0><<<blocks, NT, 0, stream>>>(dP, d_plan, d_pc, d_pres);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(res, d_pres, sizeof(double) * TT_RESTART_TRIES * TT_MAX_D, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    dev_plan_npts = h_plan.npts;
    return TT_OK;
}

// After a run whose check missed eps: the next point of the list from the
// check's worst samples, then the run again from the samples on.  restarted
// = false leaves the status to the caller (restart_cause says why).
int Problem::try_restart(bool &restarted)
{
    restarted = false;
    const int nk = d - 1;
    int st;
    if (h_plan.npts == 0) {                     // the run that just ended started from i0 alone
        h_plan.npts = 1;
        std::memcpy(h_plan.pts[0], i0, sizeof(int) * d);
        if ((st = plan_from_points()) != TT_OK) return st;
    }
    if (restarts_used >= opt.restarts || h_plan.npts > TT_MAX_SEEDS) {
        restart_cause = 1;
        return TT_OK;
    }
    // the check's samples by decreasing error (lowest sample first on ties)
    const int64_t R = verify_samples();
    std::vector<double> e((size_t)R);
    HIPCHK(hipMemcpyAsync(e.data(), d_serr, sizeof(double) * R, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<int64_t> order((size_t)R);
    for (int64_t t = 0; t < R; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return e[a] > e[b]; });
    const int nc = (int)std::min<int64_t>(R, TT_RESTART_TRIES);
    int cand[TT_RESTART_TRIES][TT_MAX_D], cin[TT_RESTART_TRIES];
    int trim[TT_RESTART_TRIES][TT_MAX_D], tin[TT_RESTART_TRIES];
    double res[TT_RESTART_TRIES][TT_MAX_D], tres[TT_RESTART_TRIES][TT_MAX_D];
    std::memset(cand, 0, sizeof cand);
    std::memset(trim, 0, sizeof trim);
    for (int c = 0; c < nc; ++c) {
        const uint64_t t = (uint64_t)order[c];
        for (int j = 0; j < d; ++j) cand[c][j] = (int)(sm64_at(opt.seed + 1, t * d + j) % (uint64_t)n[j]);
        cin[c] = point_levels(cand[c]);
    }
    if ((st = restart_check(nc, cand, cin, res)) != TT_OK) return st;
    // candidates that fail: trimmed to their longest run of unfoldings that
    // pass (the first on ties), i0's indices outside it
    for (int c = 0; c < nc; ++c) {
        tin[c] = 0;
        if (!cin[c]) continue;
        int kc = -1, kd = -1, run0 = -1;
        bool all = true;
        for (int u = 0; u < nk; ++u) {
            if (!((cin[c] >> u) & 1)) continue;
            if (res[c][u] > tau) {
                if (run0 < 0) run0 = u + 1;
                if (kc < 0 || (u + 1) - run0 > kd - kc) { kc = run0; kd = u + 1; }
            } else {
                all = false;
                run0 = -1;
            }
        }
        if (all || kc < 0) continue;
        for (int j = 0; j < d; ++j) trim[c][j] = (j < kc - 1 || j > kd) ? i0[j] : cand[c][j];
        tin[c] = point_levels(trim[c]);
    }
    if ((st = restart_check(nc, trim, tin, tres)) != TT_OK) return st;
    auto passes = [&](int in, const double *r) {
        if (!in) return false;
        for (int u = 0; u < nk; ++u)
            if (((in >> u) & 1) && !(r[u] > tau)) return false;
        return true;
    };
    const int *pick = nullptr;
    for (int c = 0; c < nc && !pick; ++c) {
        if (passes(cin[c], res[c])) pick = cand[c];
        else if (passes(tin[c], tres[c])) pick = trim[c];
    }
    if (!pick) {
        restart_cause = 2;
        return TT_OK;
    }
    std::memcpy(h_plan.pts[h_plan.npts], pick, sizeof(int) * d);
    h_plan.npts++;
    if ((st = plan_from_points()) != TT_OK) return st;
    ++restarts_used;
    // the run again, from the samples on, with the longer list
    t_first = time_to_eps;
    cur_fp32 = false;
    if ((st = begin_sweeps<double>()) != TT_OK) return st;
    phase = PH_SWEEPS;
    restarted = true;
    return TT_OK;
}

// Runs the steps; returns 1 when the run is over, 0 when wait = false and
// the device is not far enough yet, or an error (which ends the run).
int Problem::advance(bool wait)
{
    for (;;) {
        int r;
        switch (phase) {
        case PH_SWEEPS: r = cur_fp32 ? poll_sweeps<float>(wait) : poll_sweeps<double>(wait); break;
        case PH_TAIL: r = poll_tail(wait); break;
        case PH_VERIFY: r = poll_verify(wait); break;
        default: return 1;
        }
        if (r < 0) {
            // an error ends the run; nothing queued may still use the buffers
            (void)hipStreamSynchronize(stream);
            status = r;
            phase = PH_DONE;
            return r;
        }
        if (r == 0) return 0;
    }
}

// Results of a completed solve from its final device state.
void Problem::finalize(const ProbState &S, const int *ranks_now)
{
    for (int k = 0; k <= d; ++k) ranks[k] = ranks_now[k];
    CoreArgs ca;
    (void)make_core_args(d, n, ranks, ca, cores_len);
    rms = S.rms;
    tau = S.tau;
    sweeps = S.sweeps;
    pivoted = (int64_t)S.pivoted;
    evaluated = 0;
    for (int k = 1; k <= d - 1; ++k)
        evaluated += (int64_t)ranks[k - 1] * n[k - 1] * (int64_t)n[k] * ranks[k + 1];
    for (int u = 0; u < d - 1; ++u) last_best[u] = S.last_best[u];
    sweep_alg_bytes = (double)S.alg_bytes;
    new_entries = (double)S.new_entries;
    for (int j = 0; j < d; ++j) i0[j] = S.i0[j];
    rook_rounds = S.rook_rounds;
    rook_long = S.rook_long;
    ran = true;
    status = S.capped ? TT_NOT_CONVERGED : TT_OK;
}

// Geometry and device buffers for the current options (kept across runs
// while the options that shape them are unchanged).
int Problem::prepare()
{
    resolve_geometry();
    if (allocated && (alloc_fp32 != fp32 || alloc_rmax != opt.r_max || alloc_tr != req_tr ||
                      alloc_pivot != opt.pivot_mode || alloc_split != opt.rook_split ||
                      std::memcmp(alloc_kcap, kcap, sizeof kcap) != 0 ||
                      alloc_tc != req_tc || alloc_ns != opt.n_samples ||
                      std::memcmp(alloc_grid, grid, sizeof grid) != 0)) {
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
        if (hm) { (void)hipHostFree(hm); hm = nullptr; }
        allocated = false;
    }
    int st = allocate();
    if (st != TT_OK) return st;
    alloc_fp32 = fp32;
    alloc_rmax = opt.r_max;
    alloc_tr = req_tr;
    alloc_tc = req_tc;
    alloc_pivot = opt.pivot_mode;
    alloc_split = opt.rook_split;
    std::memcpy(alloc_kcap, kcap, sizeof kcap);
    alloc_ns = opt.n_samples;
    std::memcpy(alloc_grid, grid, sizeof grid);
    ran = false;
    return TT_OK;
}

// Samples of the sampled-error check for this run (see tt_options.verify).
int64_t Problem::verify_samples() const
{
    if (opt.verify > 0) return opt.verify;
    if (opt.verify == 0) return 0;
    if (opt.restarts > 0) return 4096;
    const bool policy_fp32 = opt.precision == TT_PREC_AUTO && (fp32 || force_fp64);
    return policy_fp32 ? 4096 : 0;
}

// Starts a run (step 1 queued).  On an error nothing stays queued.
int Problem::start()
{
    // an escalation sticks to the handle until its options change: the same
    // FP32 solve would miss eps again
    sampled_err = -1.0;
    escalated = force_fp64 ? 1 : 0;
    t_first = 0.0;
    restarts_used = 0;
    restart_cause = 0;
    h_plan.npts = 0;
    int st = prepare();
    if (st != TT_OK) {
        phase = PH_DONE;
        return status = st;
    }
    cur_fp32 = fp32 != 0;
    phase = PH_SWEEPS;
    st = cur_fp32 ? begin_sweeps<float>() : begin_sweeps<double>();
    if (st != TT_OK) {
        (void)hipStreamSynchronize(stream);
        phase = PH_DONE;
        return status = st;
    }
    return TT_OK;
}

int Problem::run()
{
    int st = start();
    if (st != TT_OK) return st;
    st = advance(true);
    return st < 0 ? st : status;
}

}  // namespace ttc

// Shapes and core offsets of a solved handle for the TT evaluation kernels.
static void tt_args(const Problem &P, TTArgs &a)
{
    std::memset(&a, 0, sizeof a);
    a.d = P.d;
    for (int j = 0; j < P.d; ++j) a.n[j] = P.n[j];
    for (int k = 0; k <= P.d; ++k) a.ranks[k] = P.ranks[k];
    int64_t off = 0;
    for (int k = 0; k < P.d; ++k) {
        a.goff[k] = off;
        off += (int64_t)P.ranks[k] * P.n[k] * P.ranks[k + 1];
    }
    a.goff[P.d] = off;
}

// ---------------------------------------------------------------------------
// Sampled relative error (Sec. 5) of a solved handle over R seeded indices:
// indices, f values and TT values in device buffers, then per-workgroup
// partial sums added in order on the host.
// ---------------------------------------------------------------------------
constexpr int kErrParts = 256;      // workgroups of k_err_partial

struct ErrBufs {
    int *idx = nullptr;             // R x d indices
    double *x = nullptr, *y = nullptr;   // f and TT values, R each
    double *part = nullptr;         // 2 kErrParts partial sums
};

static int sampled_error_on(Problem &P, int64_t R, uint64_t seed, const ErrBufs &b, double *err)
{
    TTArgs a;
    tt_args(P, a);
    const unsigned g = (unsigned)((R + NT - 1) / NT);
    k_gen_idx<<<g, NT, 0, P.stream>>>(P.d, a, seed, R, b.idx);
    hipError_t e = launch_fn_eval<double>(P.fn.dev, R, b.idx, b.x, P.stream);
    if (e == hipSuccess) {
        const int64_t waves = std::min<int64_t>(R, 65536);
        k_tt_eval<<<(unsigned)((waves * 64 + NT - 1) / NT), NT, 0, P.stream>>>(a, P.d_cores, R, b.idx, b.y);
        k_err_partial<<<kErrParts, NT, 0, P.stream>>>(R, b.x, b.y, b.part);
        e = hipGetLastError();
    }
    double hp[2 * kErrParts];
    if (e == hipSuccess) e = hipMemcpyAsync(hp, b.part, sizeof hp, hipMemcpyDeviceToHost, P.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
    if (e != hipSuccess) return set_err(TT_EDEVICE, "sampled error: %s", hipGetErrorString(e));
    double num = 0, den = 0;
    for (int i = 0; i < kErrParts; ++i) { num += hp[2 * i]; den += hp[2 * i + 1]; }
    *err = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
    return (*err > P.eps) ? TT_WARN_SAMPLED_ERR : TT_OK;
}

// The buffers of tt_cross_sampled_error_noalloc: one static device array
// per GPU, laid out as indices | f values | TT values | partial sums, each
// part 256-byte aligned.  Its name is a host-side stand-in: host code uses
// only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScrAlign(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kScrIdx = 0;
constexpr size_t kScrX = kScrAlign(kScrIdx + sizeof(int) * (size_t)TT_NOALLOC_MAX_SAMPLES * TT_MAX_D);
constexpr size_t kScrY = kScrAlign(kScrX + sizeof(double) * (size_t)TT_NOALLOC_MAX_SAMPLES);
constexpr size_t kScrPart = kScrAlign(kScrY + sizeof(double) * (size_t)TT_NOALLOC_MAX_SAMPLES);
constexpr size_t kScrBytes = kScrAlign(kScrPart + sizeof(double) * 2 * kErrParts);

static __device__ __align__(256) unsigned char scratch[kScrBytes];

static std::mutex g_scr_mu;
static unsigned char *g_scr_ptr[64];     // per device, from hipGetSymbolAddress

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
static int scratch_base(unsigned char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_err(TT_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(TT_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scr_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scr_ptr[dev];
    return TT_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {


const char *tt_last_error(void) { return g_err.c_str(); }

void tt_options_default(tt_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->seed = 0;
    opt->r_max = 64;
    opt->precision = TT_PREC_AUTO;
    opt->pivot_mode = TT_PIVOT_GREEDY;
    opt->n_samples = 16384;
    for (int j = 0; j < TT_MAX_D; ++j) opt->grid[j] = 1;
    opt->tile_rows = 0;
    opt->tile_cols = 0;
    opt->lookahead = 2;
    opt->stream = nullptr;
    opt->verify = -1;
    opt->restarts = 0;
}

static int check_options(const tt_options *o)
{
    if (!o) return set_err(TT_EINVAL, "options NULL");
    if (o->r_max < 1 || o->r_max > TT_MAX_RANK) return set_err(TT_EINVAL, "r_max must be in [1,%d]", TT_MAX_RANK);
    if (o->precision < TT_PREC_AUTO || o->precision > TT_PREC_FP32) return set_err(TT_EINVAL, "bad precision");
    if (o->pivot_mode != TT_PIVOT_GREEDY && o->pivot_mode != TT_PIVOT_ROOK) return set_err(TT_EINVAL, "bad pivot_mode");
    if (o->pivot_mode == TT_PIVOT_ROOK && o->precision == TT_PREC_FP32)
        return set_err(TT_EINVAL, "rook pivoting sweeps in FP64");
    if (o->rook_split < 0 || o->rook_split > 1024) return set_err(TT_EINVAL, "rook_split must be in [0,1024]");
    if (o->n_samples < 1 || o->n_samples > (1 << 26)) return set_err(TT_EINVAL, "bad n_samples");
    for (int j = 0; j < TT_MAX_D; ++j)
        if (o->grid[j] < 1) return set_err(TT_EINVAL, "grid[%d] must be >= 1", j);
    if (o->tile_rows < 0 || o->tile_rows > 256) return set_err(TT_EINVAL, "tile_rows must be in [0,256]");
    if (o->tile_cols < 0 || o->tile_cols > 64) return set_err(TT_EINVAL, "tile_cols must be in [0,64]");
    if (o->verify < -1) return set_err(TT_EINVAL, "verify must be -1, 0 or a sample count");
    if (o->restarts < 0 || o->restarts > TT_MAX_SEEDS)
        return set_err(TT_EINVAL, "restarts must be in [0,%d]", TT_MAX_SEEDS);
    if (o->restarts > 0 && o->verify == 0) return set_err(TT_EINVAL, "restarts need the sampled-error check");
    return TT_OK;
}

tt_cross_h tt_cross_create(int d, const int32_t *n, double eps, int fn_id, const double *params, int nparams)
{
    g_err.clear();
    if (!(eps >= 0.0) || !(eps < 1.0)) { set_err(TT_EINVAL, "eps must be in [0,1)"); return nullptr; }
    tt_cross_s *h = new (std::nothrow) tt_cross_s();
    if (!h) { set_err(TT_ENOMEM, "out of host memory"); return nullptr; }
    Problem &P = h->p;
    if (build_fn(fn_id, d, n, params, nparams, P.fn) != TT_OK) { delete h; return nullptr; }
    P.d = d;
    for (int j = 0; j < d; ++j) P.n[j] = n[j];
    P.eps = eps;
    tt_options_default(&P.opt);
    return h;
}

// Every call that reads or changes a handle's state refuses while a run
// started by tt_cross_run_async is in flight.
#define TT_NOT_BUSY(h)                                                                       \
    do {                                                                                     \
        if ((h)->p.busy()) return set_err(TT_ESTATE, "a run is in flight (tt_cross_wait)"); \
    } while (0)

// Use stream s (non-NULL) from now on, as tt_options.stream would.
static int adopt_stream(Problem &P, hipStream_t s)
{
    if (!s || s == P.stream) return TT_OK;
    if (P.own_stream && P.stream) (void)hipStreamDestroy(P.stream);
    P.stream = s;
    P.own_stream = false;
    P.opt.stream = s;
    return TT_OK;
}

int tt_cross_set_options(tt_cross_h h, const tt_options *opt)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    int st = check_options(opt);
    if (st) return st;
    if (h->p.allocated && opt->stream != h->p.opt.stream) {
        if (h->p.own_stream && h->p.stream) (void)hipStreamDestroy(h->p.stream);
        h->p.stream = nullptr;
        h->p.own_stream = false;
        if (h->p.allocated) {
            // a new stream needs no new buffers; keep them
            if (opt->stream) h->p.stream = (hipStream_t)opt->stream;
            else {
                if (hipStreamCreateWithFlags(&h->p.stream, hipStreamNonBlocking) != hipSuccess)
                    return set_err(TT_EDEVICE, "hipStreamCreate failed");
                h->p.own_stream = true;
            }
        }
    }
    h->p.opt = *opt;
    h->p.force_fp64 = false;
    return TT_OK;
}

int tt_cross_set_rank_caps(tt_cross_h h, const int32_t *caps)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    for (int k = 1; k <= P.d - 1; ++k) {
        const int c = caps ? caps[k - 1] : 0;
        if (c < 0 || c > TT_MAX_RANK) return set_err(TT_EINVAL, "rank cap %d of unfolding %d outside [0,%d]", c, k,
                                                      TT_MAX_RANK);
    }
    for (int k = 1; k <= P.d - 1; ++k) P.kcap[k] = caps ? caps[k - 1] : 0;
    return TT_OK;
}

int tt_cross_run(tt_cross_h h)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    g_err.clear();
    return h->p.run();
}

int tt_cross_run_async(tt_cross_h h, void *hip_stream)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    g_err.clear();
    Problem &P = h->p;
    if (hip_stream && P.allocated) adopt_stream(P, (hipStream_t)hip_stream);
    else if (hip_stream) P.opt.stream = hip_stream;     // taken up when the buffers are made
    const int st = P.start();
    if (st != TT_OK) return st;
    // take whatever steps the device already allows, without waiting
    const int a = P.advance(false);
    return a < 0 ? a : TT_OK;
}

int tt_cross_query(tt_cross_h h)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    Problem &P = h->p;
    if (!P.busy()) return 1;
    const int a = P.advance(false);
    return a < 0 ? a : (P.busy() ? 0 : 1);
}

int tt_cross_wait(tt_cross_h h)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    Problem &P = h->p;
    if (P.phase == Problem::PH_IDLE) return set_err(TT_ESTATE, "no run started");
    const int a = P.advance(true);
    return a < 0 ? a : P.status;
}

int tt_cross_get_ranks(tt_cross_h h, int32_t *ranks)
{
    if (!h || !ranks) return set_err(TT_EINVAL, "NULL argument");
    TT_NOT_BUSY(h);
    if (!h->p.ran) return set_err(TT_ESTATE, "no completed run");
    for (int k = 0; k <= h->p.d; ++k) ranks[k] = h->p.ranks[k];
    return TT_OK;
}

int tt_cross_get_tiles(tt_cross_h h, int32_t *rows, int32_t *cols)
{
    if (!h || !rows || !cols) return set_err(TT_EINVAL, "NULL argument");
    TT_NOT_BUSY(h);
    if (!h->p.ran) return set_err(TT_ESTATE, "no completed run");
    for (int u = 0; u < h->p.d - 1; ++u) {
        rows[u] = h->p.tileTR[u];
        cols[u] = h->p.tileTC[u];
    }
    return TT_OK;
}

int64_t tt_cross_get_cores(tt_cross_h h, double *out, int64_t cap, int on_device)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (!out) return P.cores_len;
    if (cap < P.cores_len) return set_err(TT_EINVAL, "cap %lld < %lld", (long long)cap, (long long)P.cores_len);
    HIPCHK(hipMemcpyAsync(out, P.d_cores, sizeof(double) * P.cores_len,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, P.stream));
    HIPCHK(hipStreamSynchronize(P.stream));
    return P.cores_len;
}


int tt_eval(tt_cross_h h, int64_t m, const int32_t *idx, double *out, int on_device)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (m < 0 || (m > 0 && (!idx || !out))) return set_err(TT_EINVAL, "bad arguments");
    if (m == 0) return TT_OK;
    TTArgs a;
    tt_args(P, a);
    const int *didx = idx;
    double *dout = out;
    void *tmp_i = nullptr, *tmp_o = nullptr;
    if (!on_device) {
        // validate indices on the host before they reach a kernel
        for (int64_t t = 0; t < m; ++t)
            for (int j = 0; j < P.d; ++j)
                if (idx[t * P.d + j] < 0 || idx[t * P.d + j] >= P.n[j])
                    return set_err(TT_EINVAL, "index %lld,%d out of range", (long long)t, j);
        HIPCHK(hipMalloc(&tmp_i, sizeof(int) * m * P.d));
        HIPCHK(hipMalloc(&tmp_o, sizeof(double) * m));
        HIPCHK(hipMemcpyAsync(tmp_i, idx, sizeof(int) * m * P.d, hipMemcpyHostToDevice, P.stream));
        didx = (const int *)tmp_i;
        dout = (double *)tmp_o;
    }
    const int64_t waves = std::min<int64_t>(m, 65536);
    k_tt_eval<<<(unsigned)((waves * 64 + NT - 1) / NT), NT, 0, P.stream>>>(a, P.d_cores, m, didx, dout);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && !on_device) e = hipMemcpyAsync(out, dout, sizeof(double) * m, hipMemcpyDeviceToHost, P.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
    if (tmp_i) (void)hipFree(tmp_i);
    if (tmp_o) (void)hipFree(tmp_o);
    if (e != hipSuccess) return set_err(TT_EDEVICE, "tt_eval: %s", hipGetErrorString(e));
    return TT_OK;
}

int tt_cross_get_pivots(tt_cross_h h, int k, int32_t *rows, int32_t *cols)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (k < 1 || k > P.d - 1) return set_err(TT_EINVAL, "k out of range");
    const KDev &K = P.hP.kd[k - 1];
    const int rk = P.ranks[k];
    if (rows) HIPCHK(hipMemcpy(rows, K.Ifull, sizeof(int) * rk * k, hipMemcpyDeviceToHost));
    if (cols) HIPCHK(hipMemcpy(cols, K.Jfull, sizeof(int) * rk * (P.d - k), hipMemcpyDeviceToHost));
    return rk;
}

int tt_cross_get_history(tt_cross_h h, int k, double *out, int cap)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (k < 1 || k > P.d - 1) return set_err(TT_EINVAL, "k out of range");
    const int m = std::min(std::min(P.sweeps, cap), P.hist_cap);
    if (out && m > 0) HIPCHK(hipMemcpy(out, P.hP.kd[k - 1].hist, sizeof(double) * m, hipMemcpyDeviceToHost));
    return P.sweeps;
}

int tt_cross_get_stats(tt_cross_h h, tt_stats *st)
{
    if (!h || !st) return set_err(TT_EINVAL, "NULL argument");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    std::memset(st, 0, sizeof *st);
    st->d = P.d;
    st->status = P.status;
    if (!P.ran) return TT_OK;
    st->evaluated = P.evaluated;
    st->pivoted = P.pivoted;
    st->samples = P.opt.n_samples;
    st->sweeps = P.sweeps;
    st->precision_used = P.fp32 ? TT_PREC_FP32 : TT_PREC_FP64;
    for (int k = 0; k <= P.d; ++k) st->ranks[k] = P.ranks[k];
    st->rms = P.rms;
    st->tau = P.tau;
    st->time_to_eps_s = P.time_to_eps;
    for (int u = 0; u < P.d - 1; ++u) st->last_best[u] = P.last_best[u];
    st->sweep_launches = P.sweep_launches;
    st->sweep_kernel_s = P.sweep_kernel_s;
    st->sweep_alg_bytes = P.sweep_alg_bytes;
    st->new_entries = P.new_entries;
    st->sweep_phase_s = P.sweep_phase_s;
    st->sampled_err = P.sampled_err;
    st->escalated = P.escalated;
    st->rook_max_rounds = P.rook_rounds;
    st->rook_long_walks = P.rook_long;
    st->restarts_used = P.restarts_used;
    st->restart_cause = P.restart_cause;
    return TT_OK;
}

int64_t tt_cross_get_stamps(tt_cross_h h, uint64_t *out, int64_t cap, int32_t *layout)
{
    if (!h) return set_err(TT_EINVAL, "NULL handle");
    TT_NOT_BUSY(h);
#ifdef TT_STAMPS
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (layout) {
        layout[0] = STAMP_WORDS;
        layout[1] = P.hP.stamp_wgs;
        layout[2] = P.hP.stamp_sweeps;
        layout[3] = P.sweeps;
    }
    if (!out) return (int64_t)P.stamp_words;
    if (cap < (int64_t)P.stamp_words) return set_err(TT_EINVAL, "cap below %zu", P.stamp_words);
    HIPCHK(hipMemcpy(out, P.hP.stamps, sizeof(uint64_t) * P.stamp_words, hipMemcpyDeviceToHost));
    return (int64_t)P.stamp_words;
#else
    (void)out; (void)cap; (void)layout;
    return set_err(TT_ESTATE, "this library was built without phase stamps (build with stamps=True)");
#endif
}

int tt_cross_sampled_error(tt_cross_h h, int64_t R, uint64_t seed, double *err)
{
    if (!h || !err) return set_err(TT_EINVAL, "NULL argument");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (R < 1) return set_err(TT_EINVAL, "R must be >= 1");
    ErrBufs b;
    hipError_t e = hipMalloc(&b.idx, sizeof(int) * R * P.d);
    if (e == hipSuccess) e = hipMalloc(&b.x, sizeof(double) * R);
    if (e == hipSuccess) e = hipMalloc(&b.y, sizeof(double) * R);
    if (e == hipSuccess) e = hipMalloc(&b.part, sizeof(double) * 2 * kErrParts);
    int st = (e == hipSuccess) ? sampled_error_on(P, R, seed, b, err)
                               : set_err(TT_ENOMEM, "sampled error: %s", hipGetErrorString(e));
    if (b.idx) (void)hipFree(b.idx);
    if (b.x) (void)hipFree(b.x);
    if (b.y) (void)hipFree(b.y);
    if (b.part) (void)hipFree(b.part);
    return st;
}

int tt_cross_sampled_error_noalloc(tt_cross_h h, int64_t R, uint64_t seed, double *err)
{
    if (!h || !err) return set_err(TT_EINVAL, "NULL argument");
    TT_NOT_BUSY(h);
    Problem &P = h->p;
    if (!P.ran) return set_err(TT_ESTATE, "no completed run");
    if (R < 1 || R > TT_NOALLOC_MAX_SAMPLES)
        return set_err(TT_EINVAL, "R = %lld outside [1, %d] (the static scratch holds %d samples)", (long long)R,
                       TT_NOALLOC_MAX_SAMPLES, TT_NOALLOC_MAX_SAMPLES);
    unsigned char *base = nullptr;
    const int st = scratch_base(&base);
    if (st != TT_OK) return st;
    ErrBufs b;
    b.idx = (int *)(base + kScrIdx);
    b.x = (double *)(base + kScrX);
    b.y = (double *)(base + kScrY);
    b.part = (double *)(base + kScrPart);
    return sampled_error_on(P, R, seed, b, err);
}

}  // extern "C"

namespace ttc {
// Device tables of the functions that bulk evaluation saw last, so that
// repeated evaluations of one function upload nothing.  A call holds the lock
// until its kernel has finished (it ends with a device synchronisation), so
// no table is replaced while a kernel reads it.  At most kEvalCacheEntries
// tables of at most kEvalCacheBytes each are kept, until the process ends.
namespace {
constexpr int kEvalCacheEntries = 4;
constexpr size_t kEvalCacheBytes = (size_t)16 << 20;
struct EvalKey {
    int fn_id = 0, d = 0;
    std::vector<int32_t> n;
    std::vector<double> params;
    bool operator==(const EvalKey &o) const
    {
        return fn_id == o.fn_id && d == o.d && n == o.n && params == o.params;
    }
};
struct EvalEntry {
    EvalKey key;
    FnHost fh;
    uint64_t used = 0;
};
std::mutex g_eval_mu;
std::vector<std::unique_ptr<EvalEntry>> g_eval_cache;
uint64_t g_eval_clock = 0;
hipEvent_t g_eval_ev[2] = {nullptr, nullptr};   // attached to the last evaluation's dispatch
double g_eval_last_ms = -1.0;
}  // namespace

// Bulk evaluation behind tt_fn_eval (V = double) and tt_fn_eval_f32.
template <typename V>
static int fn_eval_impl(int fn_id, int d, const int32_t *n, const double *params, int nparams, int64_t m,
                        const int32_t *idx, V *out, int on_device)
{
    g_err.clear();
    FnHost fresh;
    int st = build_fn(fn_id, d, n, params, nparams, fresh);
    if (st) return st;
    if (m < 0 || (m > 0 && (!idx || !out))) return set_err(TT_EINVAL, "bad arguments");
    if (m == 0) return TT_OK;
    if (!on_device)
        for (int64_t t = 0; t < m; ++t)
            for (int j = 0; j < d; ++j)
                if (idx[t * d + j] < 0 || idx[t * d + j] >= n[j])
                    return set_err(TT_EINVAL, "index %lld,%d out of range", (long long)t, j);
    std::lock_guard<std::mutex> lk(g_eval_mu);
    EvalKey key;
    key.fn_id = fn_id;
    key.d = d;
    key.n.assign(n, n + d);
    if (nparams > 0) key.params.assign(params, params + nparams);
    EvalEntry *ent = nullptr;
    for (auto &x : g_eval_cache)
        if (x->key == key) { ent = x.get(); break; }
    FnHost *fhp = &fresh;
    if (ent) {
        fhp = &ent->fh;
    } else if (fresh.table.size() * (sizeof(double) + sizeof(float)) <= kEvalCacheBytes) {
        if ((int)g_eval_cache.size() >= kEvalCacheEntries) {
            auto lru = std::min_element(g_eval_cache.begin(), g_eval_cache.end(),
                                        [](const auto &a, const auto &b) { return a->used < b->used; });
            (*lru)->fh.free_device();
            g_eval_cache.erase(lru);
        }
        auto e = std::make_unique<EvalEntry>();
        e->key = std::move(key);
        e->fh = std::move(fresh);
        if ((st = upload_fn(e->fh)) != TT_OK) { e->fh.free_device(); return st; }
        ent = e.get();
        fhp = &ent->fh;
        g_eval_cache.push_back(std::move(e));
    } else if ((st = upload_fn(fresh)) != TT_OK) {
        fresh.free_device();
        return st;
    }
    if (ent) ent->used = ++g_eval_clock;
    FnHost &fh = *fhp;
    const int *didx = idx;
    V *dout = out;
    void *ti = nullptr, *to = nullptr;
    hipError_t e = hipSuccess;
    if (!on_device) {
        e = hipMalloc(&ti, sizeof(int) * m * d);
        if (e == hipSuccess) e = hipMalloc(&to, sizeof(V) * m);
        if (e == hipSuccess) e = hipMemcpy(ti, idx, sizeof(int) * m * d, hipMemcpyHostToDevice);
        didx = (const int *)ti;
        dout = (V *)to;
    }
    for (hipEvent_t &ev : g_eval_ev)
        if (e == hipSuccess && !ev) e = hipEventCreate(&ev);
    if (e == hipSuccess) e = launch_fn_eval<V>(fh.dev, m, didx, dout, nullptr, g_eval_ev[0], g_eval_ev[1]);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_eval_ev[0], g_eval_ev[1]);
    if (e == hipSuccess) g_eval_last_ms = ms;
    if (e == hipSuccess && !on_device) e = hipMemcpy(out, dout, sizeof(V) * m, hipMemcpyDeviceToHost);
    if (ti) (void)hipFree(ti);
    if (to) (void)hipFree(to);
    if (!ent) fresh.free_device();
    if (e != hipSuccess) return set_err(TT_EDEVICE, "tt_fn_eval: %s", hipGetErrorString(e));
    return TT_OK;
}
}  // namespace ttc

extern "C" {

int tt_fn_eval(int fn_id, int d, const int32_t *n, const double *params, int nparams, int64_t m,
               const int32_t *idx, double *out, int on_device)
{
    return fn_eval_impl<double>(fn_id, d, n, params, nparams, m, idx, out, on_device);
}

int tt_fn_eval_f32(int fn_id, int d, const int32_t *n, const double *params, int nparams, int64_t m,
                   const int32_t *idx, float *out, int on_device)
{
    return fn_eval_impl<float>(fn_id, d, n, params, nparams, m, idx, out, on_device);
}

int tt_fn_eval_last_kernel_ms(double *ms)
{
    if (!ms) return set_err(TT_EINVAL, "ms is NULL");
    std::lock_guard<std::mutex> lk(g_eval_mu);
    if (g_eval_last_ms < 0.0) return set_err(TT_ESTATE, "no bulk evaluation has completed");
    *ms = g_eval_last_ms;
    return TT_OK;
}

void tt_cross_destroy(tt_cross_h h)
{
    if (!h) return;
    // a run in flight is finished first: its kernels use the buffers
    if (h->p.busy()) (void)h->p.advance(true);
    delete h;
}

}  // extern "C"
