// Host-side check of the supernodal schedule's device records (the structures the sweep and
// solve kernels index without bounds checks).  Built by tests/test_schedule_invariants.py
// against the in-tree library; reads a matrix file (int32 n, int64 nnz, int32 colptr[n+1],
// int32 rowind[nnz], float64 values[nnz]), runs the library's analysis, host factorization and
// schedule builder, and checks every record against the factor it was built from.
// usage: schedule_check <matrix file> <dense_tail_size> <solve_split_entries> <sweep_panel_rows>
// Prints "OK" and exits 0, or prints the failed condition and exits 1.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <iterator>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace cktlu;

#define REQ(c)                                                   \
    do {                                                         \
        if (!(c)) {                                              \
            std::printf("FAIL %s (line %d)\n", #c, __LINE__);    \
            return 1;                                            \
        }                                                        \
    } while (0)

// what the checks covered (printed with OK, so that a caller can tell they were not vacuous)
static long n_groups, n_split_panels, n_tiny_items, n_dense_items, n_split_solves, n_runs, n_lskip;

static int check(const Schedule &s) {
    const int nsn = s.sn_count, T = s.tail0;
    // ---- panels: levels hold singletons, then small, then wide panels; units cover them
    for (int l = 0; l < s.sn_levels; l++) {
        REQ(s.sn_lvl[l] <= s.sn_lvl_single[l] && s.sn_lvl_single[l] <= s.sn_lvl_small[l] &&
            s.sn_lvl_small[l] <= s.sn_lvl[l + 1]);
        for (int q = s.sn_lvl[l]; q < s.sn_lvl[l + 1]; q++) {
            const int w = s.sn_rec[4 * s.sn_seq[q] + 1];
            if (q < s.sn_lvl_single[l]) REQ(w == 1);
            else if (q < s.sn_lvl_small[l]) REQ(w >= 2 && w <= cktlu_dev::kSnSmallW);
            else REQ(w > cktlu_dev::kSnSmallW && w <= 64);
        }
        for (int pass = 0; pass < 2; pass++) {
            const std::vector<int> &unit = pass ? s.sn_punit : s.sn_sunit;
            const std::vector<int> &u2 = pass ? s.sn_pu2 : s.sn_su2;
            const std::vector<int> &ulvl = pass ? s.sn_pulvl : s.sn_sulvl;
            const int q0 = pass ? s.sn_lvl_small[l] : s.sn_lvl_single[l], q1 = pass ? s.sn_lvl[l + 1] : s.sn_lvl_small[l];
            int covered = 0;
            for (int u = ulvl[l]; u < ulvl[l + 1]; u++) {
                const int *U = &unit[4 * (size_t)u];
                REQ(U[0] >= q0 && U[0] < q1 && U[1] >= 0 && U[1] < U[2]);
                if (U[2] > 1) REQ(U[3] >= 0 && U[3] + U[2] <= s.sn_pnscr);
                else REQ(U[3] == -1);
                if (U[1] > 0) REQ(unit[4 * (size_t)(u - 1)] == U[0] && unit[4 * (size_t)(u - 1) + 1] == U[1] - 1);
                else covered++;
                if (U[1] == 1) n_split_panels++;
                const int S = s.sn_seq[U[0]];
                REQ(u2[4 * (size_t)u] == s.sn_rec[4 * S] && u2[4 * (size_t)u + 1] == s.sn_rec[4 * S + 1] &&
                    u2[4 * (size_t)u + 2] == s.sn_rec[4 * S + 2]);
            }
            REQ(covered == q1 - q0);
        }
        // ---- update tasks: heavy, light, tiny; every item's suffix and slots
        REQ(s.sn_task_lvl[l] <= s.sn_task_heavy[l] && s.sn_task_heavy[l] <= s.sn_task_tiny[l] &&
            s.sn_task_tiny[l] <= s.sn_task_lvl[l + 1]);
        for (int t = s.sn_task_lvl[l]; t < s.sn_task_lvl[l + 1]; t++) {
            const int k = s.sn_task[4 * (size_t)t];
            REQ(s.sn_task[4 * (size_t)t + 1] == s.Dp[k]);
            for (int it = s.sn_task[4 * (size_t)t + 2]; it < s.sn_task[4 * (size_t)t + 3]; it++) {
                const int S = s.sn_item[4 * (size_t)it], slot0 = s.sn_item[4 * (size_t)it + 1];
                const int len = s.sn_item[4 * (size_t)it + 2], mcnt = s.sn_item[4 * (size_t)it + 3];
                const int s0 = s.sn_rec[4 * S], w = s.sn_rec[4 * S + 1], off = w - len;
                REQ(len >= 1 && len <= w && mcnt >= 0);
                if (t >= s.sn_task_tiny[l]) {
                    REQ(len <= cktlu_dev::kTinyRows && mcnt <= cktlu_dev::kTinyRowsR);
                    n_tiny_items++;
                }
                if (k >= T) n_dense_items++;
                // the suffix: rows s0 + off .. s0 + w - 1 at consecutive slots of column k
                REQ(slot0 >= 0 && slot0 + len <= s.Dlen[k]);
                for (int c = 0; c < len; c++) REQ(s.Fi_dev[s.Dp[k] + slot0 + c] == s0 + off + c);
                // the second record
                REQ(s.sn_item2[4 * (size_t)it] == s0 + off && s.sn_item2[4 * (size_t)it + 1] == w);
                const int64_t moff = (int64_t)(((uint64_t)(uint32_t)s.sn_item2[4 * (size_t)it + 3] << 32) |
                                               (uint32_t)s.sn_item2[4 * (size_t)it + 2]);
                REQ(moff == s.sn_moff[it]);
                // R's rows updated land on the same rows of column k (rows < T for a dense target)
                const int jl = s0 + w - 1;
                for (int r = 0; r < mcnt; r++) {
                    const int slot = s.sn_map[moff + r];
                    REQ(slot >= 0 && slot < s.Dlen[k]);
                    REQ(s.Fi_dev[s.Dp[k] + slot] == s.Fi_dev[s.sn_cb[jl] + w + r]);
                    if (k >= T) REQ(s.Fi_dev[s.Dp[k] + slot] < T);
                }
            }
        }
        // ---- within a task (one target column, one level): the suffix slots of its items are
        // pairwise distinct and none is a slot of any item's rows of R (a source's suffix solve
        // reads no slot another source of the level updates, so the suffix solves may go
        // first), and one item's rows of R land on distinct slots (a pass may load its target
        // values before its sums).  Rows of R of different items may meet: those updates
        // accumulate, one source after another
        for (int t = s.sn_task_lvl[l]; t < s.sn_task_lvl[l + 1]; t++) {
            std::vector<int> suffix, rrows;
            for (int it = s.sn_task[4 * (size_t)t + 2]; it < s.sn_task[4 * (size_t)t + 3]; it++) {
                const int slot0 = s.sn_item[4 * (size_t)it + 1], len = s.sn_item[4 * (size_t)it + 2];
                const int mcnt = s.sn_item[4 * (size_t)it + 3];
                for (int c = 0; c < len; c++) suffix.push_back(slot0 + c);
                std::vector<int> mine(s.sn_map.begin() + s.sn_moff[it], s.sn_map.begin() + s.sn_moff[it] + mcnt);
                std::sort(mine.begin(), mine.end());
                REQ(std::adjacent_find(mine.begin(), mine.end()) == mine.end());
                rrows.insert(rrows.end(), mine.begin(), mine.end());
            }
            std::sort(suffix.begin(), suffix.end());
            std::sort(rrows.begin(), rrows.end());
            REQ(std::adjacent_find(suffix.begin(), suffix.end()) == suffix.end());
            std::vector<int> both;
            std::set_intersection(suffix.begin(), suffix.end(), rrows.begin(), rrows.end(), std::back_inserter(both));
            REQ(both.empty());
        }
        // ---- heavy groups: consecutive heavy tasks of one target supernode (or all dense);
        // every item exactly once; a source's entries update the same rows of R
        int tnext = s.sn_task_lvl[l];
        for (int g = s.sn_grp_lvl[l]; g < s.sn_grp_lvl[l + 1]; g++) {
            const int *G = &s.sn_grp[4 * (size_t)g];
            REQ(G[0] == tnext && G[1] >= 1 && G[1] <= cktlu_dev::kGroupTargets);
            n_groups++;
            tnext += G[1];
            std::vector<int> items;
            int prevS = -1;
            for (int r = G[2]; r < G[3]; r++) {
                const int *R = &s.sn_gsrc[4 * (size_t)r];
                REQ(R[0] > prevS && R[2] >= 1 && R[2] <= G[1]);
                prevS = R[0];
                if (r > G[2]) REQ(R[1] == s.sn_gsrc[4 * (size_t)(r - 1) + 1] + s.sn_gsrc[4 * (size_t)(r - 1) + 2]);
                int prevj = -1;
                for (int e = R[1]; e < R[1] + R[2]; e++) {
                    const int j = s.sn_gent[2 * (size_t)e], it = s.sn_gent[2 * (size_t)e + 1];
                    REQ(j > prevj && j < G[1]);
                    prevj = j;
                    const int t = G[0] + j;
                    REQ(it >= s.sn_task[4 * (size_t)t + 2] && it < s.sn_task[4 * (size_t)t + 3]);
                    REQ(s.sn_item[4 * (size_t)it] == R[0] && s.sn_item[4 * (size_t)it + 3] == R[3]);
                    items.push_back(it);
                }
            }
            int nit = 0;
            for (int t = G[0]; t < G[0] + G[1]; t++) nit += s.sn_task[4 * (size_t)t + 3] - s.sn_task[4 * (size_t)t + 2];
            std::sort(items.begin(), items.end());
            REQ((int)items.size() == nit && std::unique(items.begin(), items.end()) == items.end());
        }
        REQ(tnext == s.sn_task_heavy[l]);
    }
    // ---- solves
    for (int up = 0; up < 2; up++) {
        const int nl = up ? s.snu_levels : s.snl_levels;
        const std::vector<int> &lvl = up ? s.snu_lvl : s.snl_lvl, &first = up ? s.snu_first : s.snl_first;
        const std::vector<int> &tiny = up ? s.snu_tiny : s.snl_tiny, &single = up ? s.snu_single : s.snl_single;
        const std::vector<int> &seq = up ? s.snu_seq : s.snl_seq, &sw = up ? s.snu_sw : s.snl_sw;
        const std::vector<int> &unit = up ? s.snu_unit : s.snl_unit, &ur = up ? s.snu_urange : s.snl_urange;
        const std::vector<int> &runs = up ? s.snu_runs : s.snl_runs, &ulvl = up ? s.snu_ulvl : s.snl_ulvl;
        const std::vector<int> &rp = up ? s.Urp : s.Lrp, &rj = up ? s.Urj : s.Lrj, &rsrc = up ? s.Ursrc : s.Lrsrc;
        REQ((int)seq.size() == nsn && sw.size() == 2 * seq.size() && ur.size() == unit.size());
        for (size_t q = 0; q < seq.size(); q++)
            REQ(sw[2 * q] == s.sn_rec[4 * seq[q]] && sw[2 * q + 1] == s.sn_rec[4 * seq[q] + 1]);
        for (int l = 0; l < nl; l++) {
            REQ(lvl[l] <= first[l] && first[l] <= tiny[l] && tiny[l] <= single[l] && single[l] <= lvl[l + 1]);
            if (up) REQ(first[l] == lvl[l]);
            for (int q = lvl[l]; q < first[l]; q++) {     // left out of the L launches: nothing to pull
                const int i = s.sn_rec[4 * seq[q]];
                REQ(s.sn_rec[4 * seq[q] + 1] == 1 && rp[i + 1] == rp[i]);
                n_lskip++;
            }
            // the runs of every workgroup supernode hold exactly its entries outside the block
            for (int u = ulvl[l]; u < ulvl[l + 1]; u++) {
                const int *U = &unit[4 * (size_t)u];
                REQ(U[0] >= single[l] && U[0] < lvl[l + 1] && U[1] >= 0 && U[1] < U[2]);
                REQ(ur[4 * (size_t)u + 2] == s.sn_rec[4 * seq[U[0]]] && ur[4 * (size_t)u + 3] == s.sn_rec[4 * seq[U[0]] + 1]);
                if (U[1] > 0) REQ(ur[4 * (size_t)u] == ur[4 * (size_t)(u - 1) + 1]);
                if (U[1] == 1) n_split_solves++;
                if (U[1] != U[2] - 1) continue;
                const int s0 = ur[4 * (size_t)u + 2], w = ur[4 * (size_t)u + 3];
                const int rb = ur[4 * (size_t)(u - U[1])], re = ur[4 * (size_t)u + 1];
                std::vector<std::tuple<int, int, int>> want, got;   // {row c, column j, position}
                for (int c = 0; c < w; c++) {
                    const int i = s0 + c;
                    const int beg = up ? rp[i] + (w - 1 - c) : rp[i], end = up ? rp[i + 1] : rp[i + 1] - c;
                    for (int p = beg; p < end; p++) want.emplace_back(c, rj[p], rsrc[p]);
                }
                for (int r = rb; r < re; r++) {
                    const int *R = &runs[4 * (size_t)r];
                    REQ(R[2] >= 0 && R[3] >= 1 && R[2] + R[3] <= w);
                    for (int e = 0; e < R[3]; e++) {
                        got.emplace_back(R[2] + e, R[0], R[1] + e);
                        if (e == 0) n_runs++;
                        REQ(s.Fi_dev[R[1] + e] == s0 + R[2] + e);   // the position holds that row
                    }
                }
                std::sort(want.begin(), want.end());
                std::sort(got.begin(), got.end());
                REQ(want == got);
            }
        }
    }
    // ---- Schur items (dense block)
    for (size_t i = 0; i < s.schur_sn_items.size(); i += 4) {
        const int S = s.schur_sn_items[i], c0 = s.schur_sn_items[i + 1], g = s.schur_sn_items[i + 2];
        REQ(S >= 0 && S < nsn && c0 >= 0 && g >= 1 && c0 + g <= s.sn_rec[4 * S + 1]);
    }
    return 0;
}

int main(int argc, char **argv) {
    if (argc < 5) {
        std::printf("usage: %s matrix dense_tail_size solve_split_entries sweep_panel_rows\n", argv[0]);
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
    Analysis an;
    run_analysis(an, n, cp.data(), ri.data(), CKTLU_ORDER_AUTO, 1);
    std::vector<int> init(n);
    for (int k = 0; k < n; k++) init[k] = k;
    Factor F;
    int fail = 0, ns = 0;
    host_gp_factor(an, v.data(), 1e-3, init, nullptr, nullptr, F, fail, ns);
    if (fail >= 0) {
        std::printf("factorization failed at column %d\n", fail);
        return 2;
    }
    cktlu_options opt;
    cktlu_default_options(&opt);
    opt.dense_tail_size = std::atoi(argv[2]);
    opt.solve_split_entries = std::atoi(argv[3]);
    opt.sweep_panel_rows = std::atoi(argv[4]);
    Schedule s;
    build_schedule(an, F, opt, s, 0);
    if (check(s)) return 1;
    std::printf("OK n=%d supernodes=%d levels=%d T=%d groups=%ld split_panels=%ld tiny_items=%ld "
                "dense_items=%ld split_solves=%ld runs=%ld lskip=%ld\n",
                n, s.sn_count, s.sn_levels, s.tail0, n_groups, n_split_panels, n_tiny_items, n_dense_items,
                n_split_solves, n_runs, n_lskip);
    return 0;
}
