// tt_tune.hip -- tile-shape autotuner and the process-wide table of tuned
// shapes.
//
// A tile is the search launch's unit of work: TR superblock rows by TC
// columns inside one subtensor block and one prefix (suffix).  The result of
// a solve does not depend on the tile shape -- every entry's arithmetic is
// per entry, and the tiles' local pivots are combined with the lowest
// (row, column) tie-break -- only its time does.  The tuner times complete
// solves under each candidate shape and keeps the fastest per problem class:
// mode sizes, subtensor grid, sweep precision, rank cap and the generating
// function's kernel family.  Problems whose tile options are both 0 look the
// class up when they are prepared.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tt_internal.h"

namespace ttc {
namespace {

struct ClassKey {
    int d, fp32, hil, rmax;
    std::array<int, TT_MAX_D> n, grid;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(d, fp32, hil, rmax, n, grid) < std::tie(o.d, o.fp32, o.hil, o.rmax, o.n, o.grid);
    }
};

// the problem's class, from its resolved geometry
ClassKey class_of(const Problem &P)
{
    ClassKey c{};
    c.d = P.d;
    c.fp32 = P.fp32;
    c.hil = P.fn.dev.id == TT_FN_HILBERT ? 1 : 0;
    c.rmax = P.opt.r_max;
    c.n.fill(0);
    c.grid.fill(0);
    for (int j = 0; j < P.d; ++j) {
        c.n[j] = P.n[j];
        c.grid[j] = P.grid[j];
    }
    return c;
}

std::mutex g_mu;
std::map<ClassKey, std::pair<int, int>> g_table;

int pow2_ceil(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// longest run of one mode's indices inside one subtensor block
int longest_run(int n, int C)
{
    int m = 1;
    for (int b = 0; b < C; ++b) m = std::max(m, (int)((int64_t)(b + 1) * n / C - (int64_t)b * n / C));
    return m;
}

// (0, 0) -- the library's default shape -- first, then every power-of-two
// TR in [8, 256] and TC in [8, 64] up to the longest block run (a longer
// tile would hold the same entries)
std::vector<std::pair<int, int>> candidates(const Problem &P)
{
    int mr = 1, mc = 1;
    for (int k = 1; k <= P.d - 1; ++k) {
        mr = std::max(mr, longest_run(P.n[k - 1], P.grid[k - 1]));
        mc = std::max(mc, longest_run(P.n[k], P.grid[k]));
    }
    const int tr_hi = std::max(8, pow2_ceil(mr)), tc_hi = std::max(8, pow2_ceil(mc));
    std::vector<std::pair<int, int>> out{{0, 0}};
    for (int tr = 8; tr <= std::min(256, tr_hi); tr *= 2)
        for (int tc = 8; tc <= std::min(64, tc_hi); tc *= 2) out.push_back({tr, tc});
    return out;
}

double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    const size_t m = v.size() / 2;
    return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
}

void record(const ClassKey &c, int tr, int tc)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[c] = {tr, tc};
}

// A candidate must beat the default shape by this factor to be kept (a
// batch of a few small problems is timed less steadily than one solve).
constexpr double kMargin = 0.98;
constexpr double kBatchMargin = 0.95;

}  // namespace

bool tuned_tiles(const Problem &P, int &tr, int &tc)
{
    const ClassKey c = class_of(P);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(c);
    if (it == g_table.end() || (it->second.first == 0 && it->second.second == 0)) return false;
    tr = it->second.first;
    tc = it->second.second;
    return true;
}

}  // namespace ttc

using namespace ttc;

extern "C" int tt_autotune(tt_cross_h h, int reps, int32_t *tile_rows, int32_t *tile_cols, double *best_ms)
{
    if (!h) return set_err(TT_EINVAL, "handle is NULL");
    if (reps < 1 || reps > 64) return set_err(TT_EINVAL, "reps must be in [1,64]");
    if (h->p.busy()) return set_err(TT_ESTATE, "a run is in flight");
    Problem &P = h->p;
    const tt_options saved = P.opt;
    const bool saved_force = P.force_fp64;
    P.resolve_geometry();
    const ClassKey key = class_of(P);
    const std::vector<std::pair<int, int>> cands = candidates(P);
    P.use_table = false;
    auto restore = [&]() {
        P.opt = saved;
        P.force_fp64 = saved_force;
        P.use_table = true;
    };
    double t_default = -1.0, t_best = -1.0;
    std::pair<int, int> best{0, 0};
    for (const auto &c : cands) {
        P.opt.tile_rows = c.first;
        P.opt.tile_cols = c.second;
        P.force_fp64 = saved_force;
        int st = P.prepare();
        if (st == TT_EINVAL) continue;          // the shape does not fit in LDS at this rank cap
        if (st != TT_OK) { restore(); return st; }
        std::vector<double> t;
        for (int r = 0; r <= reps; ++r) {       // the first run is not timed
            P.force_fp64 = saved_force;
            st = P.run();
            if (st < 0) { restore(); return st; }
            if (r > 0) t.push_back(P.time_to_eps);
        }
        const double m = median(t);
        if (c.first == 0 && c.second == 0) t_default = m;
        if (t_best < 0 || m < t_best) { t_best = m; best = c; }
    }
    restore();
    if (t_best < 0) return set_err(TT_EINVAL, "no tile shape fits this problem");
    if (t_default >= 0 && t_best > kMargin * t_default) { best = {0, 0}; t_best = t_default; }
    record(key, best.first, best.second);
    if (tile_rows) *tile_rows = best.first;
    if (tile_cols) *tile_cols = best.second;
    if (best_ms) *best_ms = t_best * 1e3;
    return TT_OK;
}

extern "C" int tt_batch_autotune(tt_cross_h *hs, int count, int reps, int per_class, void *hip_stream)
{
    if (count < 0 || (count > 0 && !hs)) return set_err(TT_EINVAL, "bad batch arguments");
    if (reps < 1 || reps > 64) return set_err(TT_EINVAL, "reps must be in [1,64]");
    if (per_class < 1) return set_err(TT_EINVAL, "per_class must be >= 1");
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) return set_err(TT_EINVAL, "handle %d is NULL", i);
        if (hs[i]->p.busy()) return set_err(TT_ESTATE, "handle %d has a run in flight", i);
    }
    // classes in order of first appearance
    std::map<ClassKey, int> index;
    std::vector<ClassKey> keys;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
        Problem &P = hs[i]->p;
        P.resolve_geometry();
        const ClassKey c = class_of(P);
        auto it = index.find(c);
        if (it == index.end()) {
            index.emplace(c, (int)keys.size());
            keys.push_back(c);
            members.push_back({i});
        } else if ((int)members[it->second].size() < per_class) {
            members[it->second].push_back(i);
        }
    }
    std::vector<tt_options> saved(count);
    std::vector<char> saved_force(count);
    for (int i = 0; i < count; ++i) {
        saved[i] = hs[i]->p.opt;
        saved_force[i] = hs[i]->p.force_fp64 ? 1 : 0;
    }
    auto restore = [&]() {
        for (int i = 0; i < count; ++i) {
            hs[i]->p.opt = saved[i];
            hs[i]->p.force_fp64 = saved_force[i] != 0;
            hs[i]->p.use_table = true;
        }
    };
    for (size_t g = 0; g < keys.size(); ++g) {
        std::vector<tt_cross_h> sub;
        for (int i : members[g]) sub.push_back(hs[i]);
        double t_default = -1.0, t_best = -1.0;
        std::pair<int, int> best{0, 0};
        for (const auto &c : candidates(hs[members[g][0]]->p)) {
            bool fits = true;
            for (tt_cross_h x : sub) {
                x->p.opt.tile_rows = c.first;
                x->p.opt.tile_cols = c.second;
                x->p.use_table = false;
            }
            for (size_t j = 0; j < sub.size(); ++j) {
                sub[j]->p.force_fp64 = saved_force[members[g][j]] != 0;
                const int st = sub[j]->p.prepare();
                if (st == TT_EINVAL) { fits = false; break; }
                if (st != TT_OK) { restore(); return st; }
            }
            if (!fits) continue;
            std::vector<double> t;
            for (int r = 0; r <= reps; ++r) {
                for (size_t j = 0; j < sub.size(); ++j) sub[j]->p.force_fp64 = saved_force[members[g][j]] != 0;
                const int st = tt_batch_run(sub.data(), (int)sub.size(), hip_stream);
                if (st < 0) { restore(); return st; }
                // device time of the whole batch, both passes
                if (r > 0) t.push_back(sub[0]->p.time_to_eps);
            }
            const double m = median(t);
            if (c.first == 0 && c.second == 0) t_default = m;
            if (t_best < 0 || m < t_best) { t_best = m; best = c; }
        }
        if (t_best < 0) continue;
        if (t_default >= 0 && t_best > kBatchMargin * t_default) best = {0, 0};
        record(keys[g], best.first, best.second);
    }
    restore();
    return (int)keys.size();
}

extern "C" int tt_tile_table(int32_t *out, int cap)
{
    std::lock_guard<std::mutex> lk(g_mu);
    const int n = (int)g_table.size();
    if (!out) return n;
    int i = 0;
    for (const auto &e : g_table) {
        if (i >= cap) break;
        const ClassKey &c = e.first;
        int32_t *row = out + (int64_t)i * TT_TILE_ROW_WORDS;
        row[0] = c.d;
        row[1] = c.fp32;
        row[2] = c.hil;
        row[3] = c.rmax;
        for (int j = 0; j < TT_MAX_D; ++j) {
            row[4 + j] = c.n[j];
            row[4 + TT_MAX_D + j] = c.grid[j];
        }
        row[4 + 2 * TT_MAX_D] = e.second.first;
        row[5 + 2 * TT_MAX_D] = e.second.second;
        ++i;
    }
    return n;
}

extern "C" void tt_tile_table_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}
