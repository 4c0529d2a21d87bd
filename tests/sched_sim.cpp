// Host simulator of the supernodal schedule's launches, for race and ordering checks (no GPU).
//
// Every launch of the refactorization sweep (per level: the panels of its supernodes, then the
// update tasks) and of the sparse L and U solves (per level: one launch) is replayed from the
// schedule records as the set of memory accesses its workgroups make: factor entries (by device
// position), solution rows and the scratch blocks where the units of a split supernode meet.  A
// unit's accesses follow its kernel: a panel unit reads its supernode's diagonal block and
// updates its slice of the rows below it, and the last unit to arrive writes the block back; an
// update item solves the suffix of its source present in the target column (reading L11 below
// the diagonal, updating the target's suffix slots) and then updates the target's rows of R
// through its row map (reading L21); a solve supernode pulls its entries outside the diagonal
// block (L: columns before it, U: columns after it), and the last of its units solves its
// triangle and writes its rows.
//
// Two modes.
//  exact: the launches run one unit at a time and every access is recorded.  A conflict is a
//    write, and a read or write of the same word, by two different units of one launch, other
//    than a split supernode's units against the unit that runs its last part.  Ordering: a panel
//    touches only its own columns, which no earlier launch finalised; an update touches its
//    target column, not yet finalised, and otherwise only reads columns finalised by an earlier
//    launch; a solve
//    reads only rows finalised by an earlier launch (or given: L rows without entries, the
//    dense block's rows in the U solve) and writes only its own, not yet finalised, rows; every
//    sparse column and row is finalised exactly once.  Every index is checked against its array.
//  threads: the same launches with their units spread over worker threads (unit u on thread
//    (u / stride) % P), built with -fsanitize=thread.  The units of a split supernode meet as
//    the kernels' do: each stores its part, counts its arrival, and the last to arrive runs the
//    rest.  The kernels order this with a release fence before a relaxed atomic increment and an
//    acquire fence after it; the C++ memory model gives that pattern the same ordering as an
//    increment with acquire-release semantics, which is what the simulator uses, since the
//    sanitizer does not track standalone fences.  Threads are joined at every launch boundary.
//
// usage: sched_sim <matrix file> <dense_tail_size> <solve_split_entries> <sweep_panel_rows>
//                  <exact|threads> [P stride [plant]]
// plant (a mistake put into the simulated launches, never into the library, to show that the
// checks see it): 1 runs the sweep's second level before its first, 2 merges the L solve's
// second and third levels into one launch, 3 (threads) lets a split supernode's unit p = P - 1
// run the last part without counting arrivals.
// The matrix file: int32 n, int64 nnz, int32 colptr[n+1], int32 rowind[nnz], float64 values[nnz].
// Prints "OK ..." and exits 0, or prints the first violation and exits 1.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace cktlu;

enum { AF = 0, AY = 1, AS = 2, NARR = 3 };   // factor entries, solution rows, scratch blocks

// one unit of a launch (a workgroup, wavefront or lane group of the kernel): its accesses, and
// for a split supernode the part that the last of its P units to arrive runs (counted on
// counter cnt)
struct Unit {
    std::function<void(int who)> body;
    std::function<void(int who)> tail;
    int cnt = -1, P = 1, tail_id = -1;
    int own_lo = 0, own_hi = 0;               // the columns (sweep) or rows (solve) it finalises
};

enum { PANEL, UPDATE, SOLVE };
struct Launch {
    std::string what;
    int kind = PANEL;
    std::vector<Unit> units;
    std::vector<int> tail_of;                 // unit id -> id of its supernode's last part
    // unit ids are positions in units; the last parts of the split supernodes take the ids after
    void finish() {
        int nt = 0;
        for (size_t u = 0; u < units.size(); u++)
            if (units[u].P > 1) {
                if (u == 0 || units[u - 1].P == 1 || units[u - 1].cnt != units[u].cnt) nt++;
                units[u].tail_id = (int)units.size() + nt - 1;
            }
        tail_of.assign(units.size() + nt, -1);
        for (size_t u = 0; u < units.size(); u++) tail_of[u] = units[u].tail_id;
    }
};

static const char *ARRNAME[NARR] = {"factor", "solution", "scratch"};

struct Sim {
    int n = 0, T = 0;
    int64_t size[NARR] = {0, 0, 0};
    std::vector<int> col_of;                  // factor position -> column (-1: padding)
    // exact mode
    std::vector<int> wstamp[NARR], wowner[NARR];
    std::vector<int> fin_col, fin_row;        // launch that finalised a column / row (-1: none)
    int clock = 0, pass = 0, cur_lo = 0, cur_hi = 0;
    const Launch *L = nullptr;
    bool failed = false;
    char msg[512] = {0};
    // threads mode
    std::vector<double> mem[NARR];
    std::vector<std::atomic<int>> cnt;
    int plant = 0;

    void fail(const char *why, int who, int arr, int64_t idx) {
        if (failed) return;
        failed = true;
        std::snprintf(msg, sizeof msg, "%s: unit %d, %s[%lld]: %s", L ? L->what.c_str() : "?", who,
                      ARRNAME[arr], (long long)idx, why);
    }
    bool allowed(int a, int b) const { return a == b || L->tail_of[a] == b || L->tail_of[b] == a; }

    // exact mode: the checks of one access (pass 0: writes and ordering, pass 1: reads)
    void access(int who, int arr, int64_t idx, bool wr) {
        if (failed) return;
        if (idx < 0 || idx >= size[arr]) return fail("index out of range", who, arr, idx);
        if (pass == 1) {
            if (!wr && wstamp[arr][idx] == clock && !allowed(wowner[arr][idx], who))
                fail("read while another unit of the launch writes it", who, arr, idx);
            return;
        }
        if (wr) {
            if (wstamp[arr][idx] == clock && !allowed(wowner[arr][idx], who))
                return fail("written by two units of one launch", who, arr, idx);
            wstamp[arr][idx] = clock;
            wowner[arr][idx] = who;
        }
        if (arr == AF) {
            const int c = col_of[idx];
            if (c < 0) return fail("padding, not an entry of a column", who, arr, idx);
            if (L->kind == PANEL) {
                if (c < cur_lo || c >= cur_hi) return fail("a panel touches another supernode's column", who, arr, idx);
                if (fin_col[c] >= 0) return fail("a column finalised twice", who, arr, idx);
            } else if (L->kind == UPDATE) {
                const bool own = c >= cur_lo && c < cur_hi;     // the task's target column
                if (own && c < T && fin_col[c] >= 0) return fail("an update touches a finalised column", who, arr, idx);
                if (!own && wr) return fail("an update writes a column other than its target", who, arr, idx);
                if (!own && (c >= T || fin_col[c] < 0 || fin_col[c] >= clock))
                    return fail("an update reads a column not yet finalised", who, arr, idx);
            } else if (wr) {
                return fail("a solve writes the factor", who, arr, idx);
            }
        } else if (arr == AY) {
            const bool own = idx >= cur_lo && idx < cur_hi;
            if (wr && !own) return fail("writes another supernode's row", who, arr, idx);
            if (wr && fin_row[idx] >= 0) return fail("writes a row already final", who, arr, idx);
            if (!wr && !own && (fin_row[idx] < 0 || fin_row[idx] >= clock))
                return fail("reads a row not yet final", who, arr, idx);
        }
    }

    int run_exact(const std::vector<Launch> &launches) {
        for (const Launch &La : launches) {
            L = &La;
            clock++;
            for (pass = 0; pass < 2 && !failed; pass++)
                for (size_t u = 0; u < La.units.size() && !failed; u++) {
                    const Unit &U = La.units[u];
                    cur_lo = U.own_lo;
                    cur_hi = U.own_hi;
                    U.body((int)u);
                    // a split supernode's last part, after its last unit
                    if (U.P > 1 && (u + 1 == La.units.size() || La.units[u + 1].tail_id != U.tail_id)) U.tail(U.tail_id);
                }
            if (failed) return 1;
            if (La.kind != UPDATE)
                for (const Unit &U : La.units)
                    for (int c = U.own_lo; c < U.own_hi; c++) (La.kind == SOLVE ? fin_row : fin_col)[c] = clock;
        }
        return 0;
    }

    int run_threads(const std::vector<Launch> &launches, int P, int stride) {
        for (const Launch &La : launches) {
            std::vector<std::thread> th;
            for (int p = 0; p < P; p++)
                th.emplace_back([&La, p, P, stride, this] {
                    for (size_t u = 0; u < La.units.size(); u++) {
                        if ((int)((u / stride) % P) != p) continue;
                        const Unit &U = La.units[u];
                        U.body((int)u);
                        if (plant == 3 && U.P > 1) {
                            if (u + 1 == La.units.size() || La.units[u + 1].tail_id != U.tail_id) U.tail(U.tail_id);
                            continue;
                        }
                        if (U.P > 1 && cnt[U.cnt].fetch_add(1, std::memory_order_acq_rel) == U.P - 1) {
                            cnt[U.cnt].store(0, std::memory_order_relaxed);
                            U.tail(U.tail_id);
                        }
                    }
                });
            for (auto &t : th) t.join();
            for (size_t i = 0; i < cnt.size(); i++)
                if (cnt[i].load() != 0) {
                    std::snprintf(msg, sizeof msg, "%s: counter %zu left at %d", La.what.c_str(), i, cnt[i].load());
                    return 1;
                }
        }
        return 0;
    }
};

static thread_local double sink = 0.0;        // where the threads mode's reads go

int main(int argc, char **argv) {
    if (argc < 6) {
        std::printf("usage: %s matrix dense_tail_size solve_split_entries sweep_panel_rows exact|threads [P stride]\n",
                    argv[0]);
        return 2;
    }
    FILE *fp = std::fopen(argv[1], "rb");
    if (!fp) return 2;
    int n = 0;
    int64_t nnz = 0;
    if (std::fread(&n, 4, 1, fp) != 1 || std::fread(&nnz, 8, 1, fp) != 1) return 2;
    std::vector<int> cp(n + 1), ri(nnz);
    std::vector<double> v(nnz);
    if (std::fread(cp.data(), 4, n + 1, fp) != (size_t)n + 1 || std::fread(ri.data(), 4, nnz, fp) != (size_t)nnz ||
        std::fread(v.data(), 8, nnz, fp) != (size_t)nnz)
        return 2;
    std::fclose(fp);
    const bool threads = std::strcmp(argv[5], "threads") == 0;
    const int P = argc > 6 ? std::atoi(argv[6]) : 8, stride = argc > 7 ? std::atoi(argv[7]) : 1;
    const int plant = argc > 8 ? std::atoi(argv[8]) : 0;
    Analysis an;
    run_analysis(an, n, cp.data(), ri.data(), CKTLU_ORDER_AUTO, 1);
    std::vector<int> init(n);
    for (int k = 0; k < n; k++) init[k] = k;
    Factor F;
    int fcol = -1, ns = 0;
    if (host_gp_factor(an, v.data(), 1e-3, init, nullptr, nullptr, F, fcol, ns) != CKTLU_OK) {
        std::printf("factorization failed\n");
        return 2;
    }
    cktlu_options opt;
    cktlu_default_options(&opt);
    opt.dense_tail_size = std::atoi(argv[2]);
    opt.solve_split_entries = std::atoi(argv[3]);
    opt.sweep_panel_rows = std::atoi(argv[4]);
    Schedule s;
    build_schedule(an, F, opt, s, 0);

    Sim sim;
    const int T = s.tail0;
    sim.n = n;
    sim.T = T;
    sim.size[AF] = s.nnz_dev;
    sim.size[AY] = n;
    sim.size[AS] = std::max({s.sn_pnscr, s.snl_nscr, s.snu_nscr, 1});
    sim.col_of.assign(s.nnz_dev, -1);
    for (int k = 0; k < n; k++)
        for (int p = s.Dp[k]; p < s.Dp[k] + s.Dlen[k]; p++) sim.col_of[p] = k;
    sim.fin_col.assign(n, -1);
    sim.fin_row.assign(n, -1);
    for (int a = 0; a < NARR; a++) {
        if (threads) sim.mem[a].assign(sim.size[a], 0.0);
        else {
            sim.wstamp[a].assign(sim.size[a], -1);
            sim.wowner[a].assign(sim.size[a], -1);
        }
    }
    sim.cnt = std::vector<std::atomic<int>>(std::max({s.sn_seq.size(), s.snl_seq.size(), s.snu_seq.size(), (size_t)1}));

    // the access both modes share: exact mode checks it, threads mode makes it
    auto acc = [&sim, threads](int who, int arr, int64_t idx, bool wr) {
        if (!threads) return sim.access(who, arr, idx, wr);
        if (wr) sim.mem[arr][idx] += 1.0;
        else sink += sim.mem[arr][idx];
    };
    const int *cb = s.sn_cb.data();

    // ---- the sweep: per level the singletons, the small panels, the wide panels (three
    // launches), then the update tasks (one launch)
    std::vector<Launch> sweep;
    for (int l = 0; l < s.sn_levels; l++) {
        Launch sg;
        sg.what = "sweep level " + std::to_string(l) + " singletons";
        for (int q = s.sn_lvl[l]; q < s.sn_lvl_single[l]; q++) {
            const int j = s.sn_rec[4 * s.sn_seq[q]];
            Unit U;
            U.own_lo = j;
            U.own_hi = j + 1;
            U.body = [&, j](int who) {                  // pivot, then the column below it
                acc(who, AF, cb[j], false);
                for (int p = cb[j] + 1; p < s.Dp[j] + s.Dlen[j]; p++) {
                    acc(who, AF, p, false);
                    acc(who, AF, p, true);
                }
            };
            sg.units.push_back(std::move(U));
        }
        sg.finish();
        sweep.push_back(std::move(sg));
        for (int wide = 0; wide < 2; wide++) {
            const std::vector<int> &unit = wide ? s.sn_punit : s.sn_sunit;
            const std::vector<int> &ulvl = wide ? s.sn_pulvl : s.sn_sulvl;
            Launch pl;
            pl.what = "sweep level " + std::to_string(l) + (wide ? " wide panels" : " small panels");
            for (int u = ulvl[l]; u < ulvl[l + 1]; u++) {
                const int q = unit[4 * (size_t)u], p = unit[4 * (size_t)u + 1], Pu = unit[4 * (size_t)u + 2];
                const int blk = unit[4 * (size_t)u + 3];
                const int S = s.sn_seq[q], s0 = s.sn_rec[4 * S], w = s.sn_rec[4 * S + 1], m = s.sn_rec[4 * S + 2];
                const int rb = (int)((int64_t)m * p / Pu), re = (int)((int64_t)m * (p + 1) / Pu);
                auto block = [&acc, cb, s0, w](int who, bool wr) {
                    for (int c = 0; c < w; c++)
                        for (int r = 0; r < w; r++) acc(who, AF, cb[s0 + c] + r, wr);
                };
                Unit U;
                U.own_lo = s0;
                U.own_hi = s0 + w;
                U.P = Pu;
                U.cnt = q;
                U.body = [&acc, cb, s0, w, rb, re, Pu, blk, p, block](int who) {
                    block(who, false);                  // the block, factored in registers / LDS
                    if (Pu == 1) block(who, true);
                    for (int c = 0; c < w; c++)         // this unit's rows of R
                        for (int r = rb; r < re; r++) {
                            acc(who, AF, cb[s0 + c] + w + r, false);
                            acc(who, AF, cb[s0 + c] + w + r, true);
                        }
                    if (Pu > 1) acc(who, AS, blk + p, true);   // its column maxima
                };
                if (Pu > 1)
                    U.tail = [&acc, Pu, blk, block](int who) {
                        for (int pp = 0; pp < Pu; pp++) acc(who, AS, blk + pp, false);
                        block(who, true);
                    };
                pl.units.push_back(std::move(U));
            }
            pl.finish();
            sweep.push_back(std::move(pl));
        }
        Launch ul;
        ul.what = "sweep level " + std::to_string(l) + " updates";
        ul.kind = UPDATE;
        for (int t = s.sn_task_lvl[l]; t < s.sn_task_lvl[l + 1]; t++) {
            const int k = s.sn_task[4 * (size_t)t], i0 = s.sn_task[4 * (size_t)t + 2], i1 = s.sn_task[4 * (size_t)t + 3];
            Unit U;
            U.own_lo = k;                               // its target
            U.own_hi = k + 1;
            U.body = [&, k, i0, i1](int who) {
                for (int it = i0; it < i1; it++) {
                    const int S = s.sn_item[4 * (size_t)it], slot0 = s.sn_item[4 * (size_t)it + 1];
                    const int len = s.sn_item[4 * (size_t)it + 2], mcnt = s.sn_item[4 * (size_t)it + 3];
                    const int s0 = s.sn_rec[4 * S], w = s.sn_rec[4 * S + 1], off = w - len;
                    const int64_t moff = s.sn_moff[it];
                    for (int c = 0; c < len; c++) {     // U(S, k) on the suffix, by L11
                        for (int c2 = 0; c2 < c; c2++) acc(who, AF, cb[s0 + off + c2] + off + c, false);
                        acc(who, AF, s.Dp[k] + slot0 + c, false);
                        acc(who, AF, s.Dp[k] + slot0 + c, true);
                    }
                    for (int r = 0; r < mcnt; r++) {    // x_k(R) -= L21 U(S, k)
                        const int64_t tgt = s.Dp[k] + (int64_t)s.sn_map[moff + r];
                        for (int c = 0; c < len; c++) acc(who, AF, cb[s0 + off + c] + w + r, false);
                        acc(who, AF, tgt, false);
                        acc(who, AF, tgt, true);
                    }
                }
            };
            ul.units.push_back(std::move(U));
        }
        ul.finish();
        sweep.push_back(std::move(ul));
    }

    // ---- the sparse solves of the rows [0, T): one launch per level
    std::vector<Launch> solve[2];
    for (int up = 0; up < 2; up++) {
        const int nl = up ? s.snu_levels : s.snl_levels;
        const std::vector<int> &first = up ? s.snu_first : s.snl_first, &single = up ? s.snu_single : s.snl_single;
        const std::vector<int> &seq = up ? s.snu_seq : s.snl_seq;
        const std::vector<int> &unit = up ? s.snu_unit : s.snl_unit, &ur = up ? s.snu_urange : s.snl_urange;
        const std::vector<int> &runs = up ? s.snu_runs : s.snl_runs, &ulvl = up ? s.snu_ulvl : s.snl_ulvl;
        const std::vector<int> &rp = up ? s.Urp : s.Lrp, &rj = up ? s.Urj : s.Lrj, &rsrc = up ? s.Ursrc : s.Lrsrc;
        // the triangle of [s0, s0 + w): its diagonal block (L: below the diagonal; U: on and
        // above it), then its rows
        auto triangle = [&acc, cb, up](int who, int s0, int w) {
            for (int c = 0; c < w; c++)
                for (int r = 0; r < w; r++)
                    if (up ? r >= c : r > c) acc(who, AF, up ? cb[s0 + r] + c : cb[s0 + c] + r, false);
            for (int c = 0; c < w; c++) {
                acc(who, AY, s0 + c, false);
                acc(who, AY, s0 + c, true);
            }
        };
        for (int l = 0; l < nl; l++) {
            Launch sl;
            sl.what = std::string(up ? "U" : "L") + " solve level " + std::to_string(l);
            sl.kind = SOLVE;
            for (int q = first[l]; q < single[l]; q++) {      // tiny rows and wavefront supernodes
                const int s0 = s.sn_rec[4 * seq[q]], w = s.sn_rec[4 * seq[q] + 1];
                Unit U;
                U.own_lo = s0;
                U.own_hi = s0 + w;
                U.body = [&, s0, w, up, triangle](int who) {
                    for (int c = 0; c < w; c++) {
                        const int i = s0 + c;
                        const int beg = up ? rp[i] + (w - 1 - c) : rp[i], end = up ? rp[i + 1] : rp[i + 1] - c;
                        for (int p = beg; p < end; p++) {
                            acc(who, AY, rj[p], false);
                            acc(who, AF, rsrc[p], false);
                        }
                    }
                    triangle(who, s0, w);
                };
                sl.units.push_back(std::move(U));
            }
            for (int u = ulvl[l]; u < ulvl[l + 1]; u++) {     // workgroup units: runs
                const int q = unit[4 * (size_t)u], p = unit[4 * (size_t)u + 1], Pu = unit[4 * (size_t)u + 2];
                const int blk = unit[4 * (size_t)u + 3];
                const int r0 = ur[4 * (size_t)u], r1 = ur[4 * (size_t)u + 1], s0 = ur[4 * (size_t)u + 2];
                const int w = ur[4 * (size_t)u + 3];
                Unit U;
                U.own_lo = s0;
                U.own_hi = s0 + w;
                U.P = Pu;
                U.cnt = q;
                U.body = [&, r0, r1, Pu, blk, p, s0, w, triangle](int who) {
                    for (int r = r0; r < r1; r++) {
                        const int j = runs[4 * (size_t)r], pos = runs[4 * (size_t)r + 1], c = runs[4 * (size_t)r + 3];
                        acc(who, AY, j, false);
                        for (int e = 0; e < c; e++) acc(who, AF, pos + e, false);
                    }
                    if (Pu > 1) acc(who, AS, blk + p, true);     // its partial sums
                    else triangle(who, s0, w);
                };
                if (Pu > 1)
                    U.tail = [&acc, Pu, blk, s0, w, triangle](int who) {
                        for (int pp = 0; pp < Pu; pp++) acc(who, AS, blk + pp, false);
                        triangle(who, s0, w);
                    };
                sl.units.push_back(std::move(U));
            }
            sl.finish();
            solve[up].push_back(std::move(sl));
        }
    }

    sim.plant = plant;
    if (plant == 1 && s.sn_levels >= 2)      // level 1's four launches before level 0's
        std::rotate(sweep.begin(), sweep.begin() + 4, sweep.begin() + 8);
    if (plant == 2 && solve[0].size() >= 3) {
        Launch &a = solve[0][1], &b = solve[0][2];
        for (Unit &U : b.units) a.units.push_back(std::move(U));
        a.finish();
        solve[0].erase(solve[0].begin() + 2);
    }
    int64_t nunits = 0;
    for (const Launch &La : sweep) nunits += (int64_t)La.units.size();
    for (int up = 0; up < 2; up++)
        for (const Launch &La : solve[up]) nunits += (int64_t)La.units.size();
    int rc = 0;
    if (threads) {
        rc = sim.run_threads(sweep, P, stride);
        for (int up = 0; up < 2 && !rc; up++) rc = sim.run_threads(solve[up], P, stride);
    } else {
        rc = sim.run_exact(sweep);
        for (int c = 0; c < T && !rc; c++)
            if (sim.fin_col[c] < 0) {
                std::snprintf(sim.msg, sizeof sim.msg, "sparse column %d never finalised", c);
                rc = 1;
            }
        for (int up = 0; up < 2 && !rc; up++) {
            // rows final before the solve's first launch: L rows with nothing to pull (left out
            // of the launches); U: the dense block's rows, solved before it
            const int given = ++sim.clock;
            const int nl = up ? s.snu_levels : s.snl_levels;
            const std::vector<int> &lvl = up ? s.snu_lvl : s.snl_lvl, &first = up ? s.snu_first : s.snl_first;
            const std::vector<int> &seq = up ? s.snu_seq : s.snl_seq;
            std::fill(sim.fin_row.begin(), sim.fin_row.end(), -1);
            for (int l = 0; l < nl; l++)
                for (int q = lvl[l]; q < first[l]; q++) sim.fin_row[s.sn_rec[4 * seq[q]]] = given;
            for (int i = T; i < n; i++) sim.fin_row[i] = up ? given : -1;
            rc = sim.run_exact(solve[up]);
            for (int i = 0; i < T && !rc; i++)
                if (sim.fin_row[i] < 0) {
                    std::snprintf(sim.msg, sizeof sim.msg, "%s solve: row %d never final", up ? "U" : "L", i);
                    rc = 1;
                }
        }
    }
    if (rc) {
        std::printf("FAIL %s\n", sim.msg);
        return 1;
    }
    std::printf("OK n=%d T=%d launches=%zu units=%lld\n", n, T, sweep.size() + solve[0].size() + solve[1].size(),
                (long long)nunits);
    return 0;
}
