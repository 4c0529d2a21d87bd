// Schedule construction for a fixed factor pattern (Section II-B, Section
// IV-B, Section V-C): dependency levels of the columns (the "guessed"
// elimination graph), the column sequence ordered by level, the scatter map
// of the matrix values into the factor storage, the row-wise structures
// of L and U used by the triangular solves, the dense trailing block, and (by
// default) the supernodes with their sweep levels, panel units, update tasks,
// slot maps, Schur items and solve levels.
#include <algorithm>
#include <array>
#include <climits>
#include <thread>
#include <new>
#include <numeric>

#include <hip/hip_runtime.h>

#include "internal.h"

namespace cktlu {

// Order D of the trailing block factored densely (Section V-A).  Forced by a
// positive option value, never with -1; otherwise the largest multiple of the
// panel width (at least 256, at most 8192) whose block of L+U has a fill density
// of at least dense_tail_density.  An entry (i,k) lies in the trailing block of
// order D exactly when min(i,k) >= n - D.
static int choose_tail(const Factor &f, const cktlu_options &opt) {
    const int n = f.n;
    if (opt.dense_tail_size < 0 || n == 0) return 0;
    if (opt.dense_tail_size > 0) return std::min(opt.dense_tail_size, n);
    const int nb = cktlu_dev::kDenseBlock, dmax = std::min(n, 8192) / nb * nb;
    if (dmax < 256) return 0;
    std::vector<double> cnt(dmax + 1, 0.0);
    for (int k = n - dmax; k < n; k++)
        for (int64_t q = f.Fp[k]; q < f.Fp[k + 1]; q++) {
            const int m = std::min(f.Fi[q], k);
            if (m >= n - dmax) cnt[n - m] += 1.0;
        }
    for (int d = 1; d <= dmax; d++) cnt[d] += cnt[d - 1];
    for (int d = dmax; d >= 256; d -= nb)
        if (cnt[d] >= opt.dense_tail_density * (double)d * (double)d) return d;
    return 0;
}

// update tasks of at least this many multiply-adds get a workgroup (four wavefronts)
constexpr double kHeavyTask = 16384.0;
constexpr int kHeavyRows = 384;          // a task with an item of this many rows of R is heavy too
// supernodal solves: a singleton whose row pulls at least kSolveLongRow entries gets a
// workgroup; a supernode's pull, as runs of rows present in one column, is split into units of
// kSolvePullChunk / 64 to kSolvePullChunk / 16 runs (the default of options.solve_split_entries;
// at most kSolveMaxSplit units), one workgroup each
constexpr int64_t kSolveLongRow = 1024;
constexpr int64_t kSolveTinyRow = 32;      // singletons with this many entries at most: 16 lanes
constexpr int64_t kSolvePullChunk = 8192;
constexpr int64_t kSolveMaxSplit = 1024;
// rows of R per unit of a wide panel (two passes of its eight wavefronts; the default of
// options.sweep_panel_rows), half of it for a small one (two passes of its wavefront)
constexpr int kPanelRows = 256;

// Supernodal sweep schedule of the sparse columns [0, T) (see Schedule).  Needs the device
// layout (Dp, Dlen, Fi_dev) and the row lists of L (Lrp, Lrj).
static void build_supernodal(const Factor &f, Schedule &s, int T, int wmax, int panel_rows, int64_t pull_chunk) {
    const int n = f.n;
    auto lbeg = [&](int j) { return f.Fp[j] + f.nU[j]; };
    // ---- supernodes: j joins the supernode of j-1 when L(:,j-1) = {j} u L(:,j) and U(s0..j-1, j)
    // are all present (the diagonal block is dense), up to wmax columns
    std::vector<int> s0v;
    std::vector<int> snof(T);
    for (int j = 0; j < T; j++) {
        bool join = false;
        if (j > 0) {
            const int p = j - 1, st = s0v.back();
            const int64_t lp = f.Fp[p + 1] - lbeg(p), lj = f.Fp[j + 1] - lbeg(j);
            join = j - st < wmax && lp == lj + 1 && f.Fi[lbeg(p)] == j &&
                   std::equal(f.Fi.begin() + lbeg(p) + 1, f.Fi.begin() + f.Fp[p + 1], f.Fi.begin() + lbeg(j));
            if (join) {
                const int nuj = f.nU[j] - 1;   // U rows of column j above its diagonal; the last j - st are s0..j-1
                join = nuj >= j - st && f.Fi[f.Fp[j] + nuj - (j - st)] == st;
            }
        }
        if (!join) s0v.push_back(j);
        snof[j] = (int)s0v.size() - 1;
    }
    const int nsn = (int)s0v.size();
    s0v.push_back(T);
    s.sn_count = nsn;
    s.sn_rec.assign(4 * (size_t)nsn, 0);
    s.sn_cb.assign(T, 0);
    for (int S = 0; S < nsn; S++) {
        const int a = s0v[S], w = s0v[S + 1] - a;
        s.sn_rec[4 * (size_t)S + 0] = a;
        s.sn_rec[4 * (size_t)S + 1] = w;
        s.sn_rec[4 * (size_t)S + 2] = (int)(f.Fp[a + w] - lbeg(a + w - 1));   // |R| = |L(:, s1-1)|
        {
            const int *rb = f.Fi.data() + lbeg(a + w - 1), *re = f.Fi.data() + f.Fp[a + w];
            s.sn_rec[4 * (size_t)S + 3] = (int)(std::lower_bound(rb, re, T) - rb);   // rows of R below T
        }
        for (int j = a; j < a + w; j++) s.sn_cb[j] = s.Dp[j] + f.nU[j] - 1 - (j - a);
    }
    // ---- levels
    std::vector<int> lev(nsn, 0);
    int nl = nsn ? 1 : 0;
    for (int S = 0; S < nsn; S++) {
        int l = 0;
        const int a = s0v[S];
        for (int k = a; k < s0v[S + 1]; k++) {
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1; q++) {
                const int j = f.Fi[q];
                if (j < a) l = std::max(l, lev[snof[j]] + 1);
            }
            for (int q = s.Lrp[k]; q < s.Lrp[k + 1]; q++) {
                const int j = s.Lrj[q];
                if (j < a) l = std::max(l, lev[snof[j]] + 1);
            }
        }
        lev[S] = l;
        nl = std::max(nl, l + 1);
    }
    s.sn_levels = nl;
    // supernodes by level: singletons, then small panels, then the wider ones; ascending ids
    // inside each group
    std::vector<int> cnt(nl + 1, 0), cnt1(nl, 0), cnt2(nl, 0);
    for (int S = 0; S < nsn; S++) {
        const int w = s0v[S + 1] - s0v[S];
        cnt[lev[S] + 1]++;
        if (w == 1) cnt1[lev[S]]++;
        else if (w <= cktlu_dev::kSnSmallW) cnt2[lev[S]]++;
    }
    for (int l = 0; l < nl; l++) cnt[l + 1] += cnt[l];
    s.sn_lvl.assign(cnt.begin(), cnt.end());
    s.sn_lvl_single.resize(nl);
    s.sn_lvl_small.resize(nl);
    std::vector<int> fill1(nl), fill2(nl), fill3(nl);
    for (int l = 0; l < nl; l++) {
        s.sn_lvl_single[l] = cnt[l] + cnt1[l];
        s.sn_lvl_small[l] = cnt[l] + cnt1[l] + cnt2[l];
        fill1[l] = cnt[l];
        fill2[l] = s.sn_lvl_single[l];
        fill3[l] = s.sn_lvl_small[l];
    }
    s.sn_seq.resize(nsn);
    for (int S = 0; S < nsn; S++) {
        const int w = s0v[S + 1] - s0v[S];
        if (w == 1) s.sn_seq[fill1[lev[S]]++] = S;
        else if (w <= cktlu_dev::kSnSmallW) s.sn_seq[fill2[lev[S]]++] = S;
        else s.sn_seq[fill3[lev[S]]++] = S;
    }
    // panels as units, each taking a slice of R's rows: small panels (a wavefront each)
    // P = ceil(m / (panel_rows / 2)), wide ones (a workgroup each) P = ceil(m / panel_rows).
    // Scratch blocks are numbered per launch
    s.sn_punit.clear();
    s.sn_sunit.clear();
    s.sn_pulvl.assign(nl + 1, 0);
    s.sn_sulvl.assign(nl + 1, 0);
    s.sn_pnscr = 0;
    s.sn_pu2.clear();
    s.sn_su2.clear();
    auto units = [&](int q0, int q1, int rows, std::vector<int> &u, std::vector<int> &u2) {
        int blocks = 0;
        for (int q = q0; q < q1; q++) {
            const int S = s.sn_seq[q];
            const int m = s.sn_rec[4 * (size_t)S + 2];
            const int P = std::max(1, (m + rows - 1) / rows);
            for (int p = 0; p < P; p++) {
                u.insert(u.end(), {q, p, P, P > 1 ? blocks : -1});
                u2.insert(u2.end(), {s.sn_rec[4 * (size_t)S], s.sn_rec[4 * (size_t)S + 1], m, 0});
            }
            if (P > 1) blocks += P;
        }
        s.sn_pnscr = std::max(s.sn_pnscr, blocks);
    };
    for (int l = 0; l < nl; l++) {
        units(s.sn_lvl_single[l], s.sn_lvl_small[l], std::max(1, panel_rows / 2), s.sn_sunit, s.sn_su2);
        units(s.sn_lvl_small[l], s.sn_lvl[l + 1], panel_rows, s.sn_punit, s.sn_pu2);
        s.sn_sulvl[l + 1] = (int)(s.sn_sunit.size() / 4);
        s.sn_pulvl[l + 1] = (int)(s.sn_punit.size() / 4);
    }
    // ---- update tasks: the pairs (S, k), k outside S with U(s1-1, k) != 0 (then U(S, k) is a
    // suffix of S's rows: a row of S present in k fills every later row of S in k), grouped
    // by (level of S, k), items ascending in S
    std::vector<int64_t> bucket(nl + 1, 0);
    for (int k = 0; k < n; k++)
        for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1 && f.Fi[q] < T; q++) {
            const int j = f.Fi[q], S = snof[j];
            if (j == s0v[S + 1] - 1 && k >= s0v[S + 1]) bucket[lev[S] + 1]++;
        }
    for (int l = 0; l < nl; l++) bucket[l + 1] += bucket[l];
    const int64_t nitems = bucket[nl];
    std::vector<int> it_k(nitems), it_S(nitems), it_slot0(nitems), it_len(nitems);
    {
        std::vector<int64_t> fp(bucket.begin(), bucket.end() - 1);
        for (int k = 0; k < n; k++)
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1 && f.Fi[q] < T; q++) {
                const int j = f.Fi[q], S = snof[j];
                if (j != s0v[S + 1] - 1 || k < s0v[S + 1]) continue;
                int len = 1;
                while (len < s0v[S + 1] - s0v[S] && q - len >= f.Fp[k] && f.Fi[q - len] == j - len) len++;
                const int64_t o = fp[lev[S]]++;
                it_k[o] = k;
                it_S[o] = S;
                it_slot0[o] = (int)(q - (len - 1) - f.Fp[k]);
                it_len[o] = len;
            }
    }
    s.sn_items = nitems;
    s.sn_item.resize(4 * (size_t)nitems);
    s.sn_moff.resize(nitems + 1);
    s.sn_task.clear();
    s.sn_task_lvl.assign(nl + 1, 0);
    int64_t moff = 0;
    double macs = 0;
    int l = 0;
    for (int64_t i = 0; i < nitems; i++) {
        while (i >= bucket[l + 1]) l++;
        const int k = it_k[i], S = it_S[i];
        const int a = s0v[S], s1 = s0v[S + 1];
        // rows of R updated: all of them for a sparse target, those < T for a dense one
        const int *rb = f.Fi.data() + lbeg(s1 - 1), *re = f.Fi.data() + f.Fp[s1];
        const int mcnt = k < T ? (int)(re - rb) : (int)(std::lower_bound(rb, re, T) - rb);
        if (i == bucket[l] || k != it_k[i - 1]) {
            if (!s.sn_task.empty()) s.sn_task[s.sn_task.size() - 1] = (int)i;
            s.sn_task.insert(s.sn_task.end(), {k, s.Dp[k], (int)i, 0});
            s.sn_task_lvl[l + 1]++;
        }
        int *it = s.sn_item.data() + 4 * (size_t)i;
        it[0] = S;
        it[1] = it_slot0[i];
        it[2] = it_len[i];
        it[3] = mcnt;
        s.sn_moff[i] = moff;
        moff += mcnt;
        macs += (double)mcnt * it_len[i] + 0.5 * (double)it_len[i] * (it_len[i] - 1);
        (void)a;
    }
    if (!s.sn_task.empty()) s.sn_task[s.sn_task.size() - 1] = (int)nitems;
    s.sn_moff[nitems] = moff;
    s.sn_item2.resize(4 * (size_t)nitems);
    for (int64_t i = 0; i < nitems; i++) {
        const int S = s.sn_item[4 * i], len = s.sn_item[4 * i + 2];
        const int w = s.sn_rec[4 * (size_t)S + 1];
        s.sn_item2[4 * i] = s.sn_rec[4 * (size_t)S] + (w - len);
        s.sn_item2[4 * i + 1] = w;
        s.sn_item2[4 * i + 2] = (int)(uint32_t)(uint64_t)s.sn_moff[i];
        s.sn_item2[4 * i + 3] = (int)(uint32_t)((uint64_t)s.sn_moff[i] >> 32);
    }
    for (int q = 0; q < nl; q++) s.sn_task_lvl[q + 1] += s.sn_task_lvl[q];
    // inside each level: heavy tasks (rows of R times suffix rows at least kHeavyTask, or an
    // item with at least kHeavyRows rows of R: its rows split over four wavefronts) first, a
    // workgroup each; then light tasks, a wavefront each; then tiny tasks (every item at most
    // kTinyRows suffix rows and kTinyRowsR rows of R), sixteen lanes each.  The order of tasks does not
    // change results
    s.sn_task_heavy.assign(nl, 0);
    s.sn_task_tiny.assign(nl, 0);
    {
        std::vector<int> tmp;
        for (int q = 0; q < nl; q++) {
            const int t0 = s.sn_task_lvl[q], t1 = s.sn_task_lvl[q + 1];
            std::vector<int> heavy, light, tiny;
            for (int t = t0; t < t1; t++) {
                double cost = 0;
                bool small = true;
                int rows = 0;
                for (int it2 = s.sn_task[4 * (size_t)t + 2]; it2 < s.sn_task[4 * (size_t)t + 3]; it2++) {
                    cost += (double)s.sn_item[4 * (size_t)it2 + 3] * s.sn_item[4 * (size_t)it2 + 2];
                    rows = std::max(rows, s.sn_item[4 * (size_t)it2 + 3]);
                    small = small && s.sn_item[4 * (size_t)it2 + 2] <= cktlu_dev::kTinyRows &&
                            s.sn_item[4 * (size_t)it2 + 3] <= cktlu_dev::kTinyRowsR;
                }
                (cost >= kHeavyTask || rows >= kHeavyRows ? heavy : small ? tiny : light).push_back(t);
            }
            s.sn_task_heavy[q] = t0 + (int)heavy.size();
            s.sn_task_tiny[q] = t0 + (int)(heavy.size() + light.size());
            for (const std::vector<int> *g : {&heavy, &light, &tiny})
                for (int t : *g) tmp.insert(tmp.end(), s.sn_task.begin() + 4 * (size_t)t, s.sn_task.begin() + 4 * (size_t)t + 4);
        }
        s.sn_task.swap(tmp);
    }
    // heavy tasks in groups of up to kGroupTargets consecutive targets that lie in one sparse
    // supernode or are all dense-block columns: such targets share most of their sources, and
    // a group reads each source's rows of R once for all its targets.  Source records {S,
    // first entry, entries, rows of R updated} ascend in S; entries {target index in the
    // group, item}.
    s.sn_grp.clear();
    s.sn_gsrc.clear();
    s.sn_gent.clear();
    s.sn_grp_lvl.assign(nl + 1, 0);
    for (int q = 0; q < nl; q++) {
        const int t0 = s.sn_task_lvl[q], t1 = s.sn_task_heavy[q];
        for (int ga = t0; ga < t1;) {
            const int ka = s.sn_task[4 * (size_t)ga];
            const int key = ka < T ? snof[ka] : -1;
            int gb = ga + 1;
            while (gb < t1 && gb - ga < cktlu_dev::kGroupTargets) {
                const int kb = s.sn_task[4 * (size_t)gb];
                if ((kb < T ? snof[kb] : -1) != key) break;
                gb++;
            }
            std::vector<std::array<int, 3>> ent;    // {S, target index, item}
            auto collect = [&]() {
                ent.clear();
                for (int t = ga; t < gb; t++)
                    for (int it = s.sn_task[4 * (size_t)t + 2]; it < s.sn_task[4 * (size_t)t + 3]; it++)
                        ent.push_back({s.sn_item[4 * (size_t)it], t - ga, it});
                std::sort(ent.begin(), ent.end());
                // a source's entries must update the same rows of R (they do: targets in one
                // sparse supernode take all of R, dense-block targets its rows < T)
                for (size_t e = 1; e < ent.size(); e++)
                    if (ent[e][0] == ent[e - 1][0] &&
                        s.sn_item[4 * (size_t)ent[e][2] + 3] != s.sn_item[4 * (size_t)ent[e - 1][2] + 3])
                        return false;
                return true;
            };
            if (!collect()) {
                gb = ga + 1;                        // a group of one: one entry per source
                collect();
            }
            const int src0 = (int)(s.sn_gsrc.size() / 4);
            for (size_t e = 0; e < ent.size();) {
                size_t f = e;
                while (f < ent.size() && ent[f][0] == ent[e][0]) f++;
                s.sn_gsrc.insert(s.sn_gsrc.end(), {ent[e][0], (int)(s.sn_gent.size() / 2), (int)(f - e),
                                                   s.sn_item[4 * (size_t)ent[e][2] + 3]});
                for (size_t h = e; h < f; h++) s.sn_gent.insert(s.sn_gent.end(), {ent[h][1], ent[h][2]});
                e = f;
            }
            s.sn_grp.insert(s.sn_grp.end(), {ga, gb - ga, src0, (int)(s.sn_gsrc.size() / 4)});
            ga = gb;
        }
        s.sn_grp_lvl[q + 1] = (int)(s.sn_grp.size() / 4);
    }
    // panels: the diagonal block's LU and L21 = A21 U11^-1
    for (int S = 0; S < nsn; S++) {
        const double w = s0v[S + 1] - s0v[S], m = s.sn_rec[4 * (size_t)S + 2];
        macs += w * w * w / 3.0 + m * w * w / 2.0;
    }
    s.sn_macs = macs;
    // ---- Schur update of the dense block by supernodes: a dense column k's rows < T (U entries)
    // that belong to one supernode are consecutive columns of it, so S(:, k) -= L21_hi U(those, k)
    // is one product per (supernode, k), L21_hi being the supernode's rows >= T.  Items {S, first
    // column of S, columns, position of the first row in k}; each column's items are cut into
    // parts of similar cost (one round trip per item plus one per 128 rows times columns / 8),
    // part 0 in place and later parts in scratch columns added in part order.
    s.schur_sn_items.clear();
    s.schur_parts.clear();
    s.schur_add.clear();
    s.schur_nscr = 0;
    if (T < n) {
        const int Dn = n - T;
        std::vector<std::vector<int>> citems(Dn);
        std::vector<double> ccost(Dn, 0.0);
        double tot = 0.0;
        for (int c = 0; c < Dn; c++) {
            const int k = T + c;
            const int64_t b = f.Fp[k], e = f.Fp[k] + f.nU[k] - 1;
            int64_t q = b;
            while (q < e && f.Fi[q] < T) {
                const int j = f.Fi[q], S = snof[j];
                int g = 1;
                while (q + g < e && f.Fi[q + g] == j + g && j + g < s0v[S + 1]) g++;
                const int mhi = s.sn_rec[4 * (size_t)S + 2] - s.sn_rec[4 * (size_t)S + 3];
                if (mhi > 0) {
                    citems[c].insert(citems[c].end(), {S, j - s0v[S], g, (int)(q - b)});
                    const double cost = 1.0 + (double)mhi * g / 1024.0;
                    ccost[c] += cost;
                    tot += cost;
                }
                q += g;
            }
        }
        const double budget = std::max(1.0, 1.5 * tot / Dn);
        for (int c = 0; c < Dn; c++) {
            const int ni = (int)citems[c].size() / 4;
            const int scr0 = s.schur_nscr;
            for (int i0 = 0, part = 0; i0 < ni; part++) {
                double acc = 0.0;
                int i1 = i0;
                while (i1 < ni) {
                    const int *it = citems[c].data() + 4 * i1;
                    const double cost = 1.0 + (double)(s.sn_rec[4 * (size_t)it[0] + 2] - s.sn_rec[4 * (size_t)it[0] + 3]) *
                                                  it[2] / 1024.0;
                    if (i1 > i0 && acc + cost > budget) break;
                    acc += cost;
                    i1++;
                }
                const int first = (int)(s.schur_sn_items.size() / 4);
                s.schur_sn_items.insert(s.schur_sn_items.end(), citems[c].begin() + 4 * i0, citems[c].begin() + 4 * i1);
                const int scr = part == 0 ? -1 : s.schur_nscr++;
                s.schur_parts.insert(s.schur_parts.end(), {c, first, first + (i1 - i0), scr});
                i0 = i1;
            }
            if (s.schur_nscr > scr0) s.schur_add.insert(s.schur_add.end(), {c, scr0, s.schur_nscr - scr0, 0});
        }
    }
    // ---- solve levels over the supernodes.  L: the rows of S reach column j < s0 through
    // L(i, j); U: the rows of S reach column k >= s1 through U(i, k) (k < T: dense columns are
    // solved before the sparse U rows)
    std::vector<int> lastc(n, -2), lastpos(n, -2), recidx(n, 0);
    auto solve_levels = [&](bool upper, int &nlev, std::vector<int> &lvl, std::vector<int> &tiny,
                            std::vector<int> &single, std::vector<int> &first, std::vector<int> &seq, std::vector<int> &unit,
                            std::vector<int> &urange, std::vector<int> &runs, std::vector<int> &ulvl, int &nscr) {
        std::vector<int> lv(nsn, 0);
        std::vector<int64_t> pull(nsn, 0);            // entries outside the diagonal block
        nlev = nsn ? 1 : 0;
        for (int q = 0; q < nsn; q++) {
            const int S = upper ? nsn - 1 - q : q;
            const int a = s0v[S], e = s0v[S + 1];
            int v = 0;
            for (int i = a; i < e; i++) {
                if (!upper) {
                    for (int p = s.Lrp[i]; p < s.Lrp[i + 1] - (i - a); p++) v = std::max(v, lv[snof[s.Lrj[p]]] + 1);
                    pull[S] += s.Lrp[i + 1] - (i - a) - s.Lrp[i];
                } else {
                    for (int p = s.Urp[i] + (e - 1 - i); p < s.Urp[i + 1]; p++)
                        if (s.Urj[p] < T) v = std::max(v, lv[snof[s.Urj[p]]] + 1);
                    pull[S] += s.Urp[i + 1] - (s.Urp[i] + (e - 1 - i));
                }
            }
            lv[S] = v;
            nlev = std::max(nlev, v + 1);
        }
        // sixteen lanes per singleton with at most kSolveTinyRow entries; a wavefront per other
        // supernode of at most kSnSmallW rows with a short pull; a workgroup per unit of every
        // other supernode
        // (L only: a singleton that pulls nothing has y_i = b_i already: nothing to launch; it
        // is placed first in its level, before first[l])
        auto kind = [&](int S) {
            const int w = s0v[S + 1] - s0v[S];
            if (!upper && w == 1 && pull[S] == 0) return 0;
            if (w == 1 && pull[S] <= kSolveTinyRow) return 1;
            return w <= cktlu_dev::kSnSmallW && pull[S] < kSolveLongRow ? 2 : 3;
        };
        std::vector<int> c(nlev + 1, 0), cn(nlev, 0), c0(nlev, 0), c1(nlev, 0);
        for (int S = 0; S < nsn; S++) {
            c[lv[S] + 1]++;
            const int k = kind(S);
            if (k == 0) cn[lv[S]]++;
            else if (k == 1) c0[lv[S]]++;
            else if (k == 2) c1[lv[S]]++;
        }
        for (int l2 = 0; l2 < nlev; l2++) c[l2 + 1] += c[l2];
        lvl.assign(c.begin(), c.end());
        first.resize(nlev);
        tiny.resize(nlev);
        single.resize(nlev);
        std::vector<int> f[4] = {std::vector<int>(nlev), std::vector<int>(nlev), std::vector<int>(nlev),
                                 std::vector<int>(nlev)};
        for (int l2 = 0; l2 < nlev; l2++) {
            first[l2] = c[l2] + cn[l2];
            tiny[l2] = first[l2] + c0[l2];
            single[l2] = tiny[l2] + c1[l2];
            f[0][l2] = c[l2];
            f[1][l2] = first[l2];
            f[2][l2] = tiny[l2];
            f[3][l2] = single[l2];
        }
        seq.resize(nsn);
        for (int S = 0; S < nsn; S++) seq[f[kind(S)][lv[S]]++] = S;
        // the pull of a workgroup supernode S as runs {column j, position of its first entry,
        // first row c_a, rows}: rows s0 + c_a .. s0 + c_a + rows - 1 of S all present in column
        // j (their entries are consecutive in j's storage, rows being sorted); a run per column
        // unless its rows of S have a gap.  The runs are cut into P units; P > 1 units' partial
        // sums meet in scratch blocks (P per supernode, numbered within the level) and the last
        // unit to finish solves the triangle.  Units hold up to pull_chunk / 16 runs, fewer (down
        // to pull_chunk / 64) on a level with few runs, whose time is its units' chain, not
        // their number: the level's runs / 128, clamped to that range
        const int64_t unit_max = std::max<int64_t>(1, pull_chunk / 16);
        const int64_t unit_min = std::max<int64_t>(1, pull_chunk / 64);
        unit.clear();
        urange.clear();
        runs.clear();
        ulvl.assign(nlev + 1, 0);
        nscr = 0;
        std::vector<int> touched;
        std::vector<int64_t> rbeg;
        for (int l2 = 0; l2 < nlev; l2++) {
            int blocks = 0;
            rbeg.clear();
            for (int q = single[l2]; q < lvl[l2 + 1]; q++) {
                const int S = seq[q];
                const int a = s0v[S], w = s0v[S + 1] - a;
                rbeg.push_back((int64_t)runs.size() / 4);
                touched.clear();
                for (int c = 0; c < w; c++) {
                    const int i = a + c;
                    const int beg = upper ? s.Urp[i] + (w - 1 - c) : s.Lrp[i];
                    const int end = upper ? s.Urp[i + 1] : s.Lrp[i + 1] - c;
                    for (int p = beg; p < end; p++) {
                        const int j = upper ? s.Urj[p] : s.Lrj[p], pos = upper ? s.Ursrc[p] : s.Lrsrc[p];
                        if (lastc[j] == c - 1 && lastpos[j] == pos - 1) {
                            runs[4 * (size_t)recidx[j] + 3]++;
                        } else {
                            if (lastc[j] < 0) touched.push_back(j);
                            recidx[j] = (int)(runs.size() / 4);
                            runs.insert(runs.end(), {j, pos, c, 1});
                        }
                        lastc[j] = c;
                        lastpos[j] = pos;
                    }
                }
                for (int j : touched) lastc[j] = lastpos[j] = -2;
            }
            rbeg.push_back((int64_t)runs.size() / 4);
            const int64_t per_unit = std::min(unit_max, std::max(unit_min, (rbeg.back() - rbeg.front() + 127) / 128));
            for (int q = single[l2]; q < lvl[l2 + 1]; q++) {
                const int64_t r0 = rbeg[q - single[l2]], nr = rbeg[q - single[l2] + 1] - r0;
                const int P = (int)std::min<int64_t>(kSolveMaxSplit, std::max<int64_t>(1, (nr + per_unit - 1) / per_unit));
                for (int p = 0; p < P; p++) {
                    unit.insert(unit.end(), {q, p, P, P > 1 ? blocks : -1});
                    urange.insert(urange.end(), {(int)(r0 + nr * p / P), (int)(r0 + nr * (p + 1) / P),
                                                 s0v[seq[q]], s0v[seq[q] + 1] - s0v[seq[q]]});
                }
                if (P > 1) blocks += P;
            }
            ulvl[l2 + 1] = (int)(unit.size() / 4);
            nscr = std::max(nscr, blocks);
        }
    };
    solve_levels(false, s.snl_levels, s.snl_lvl, s.snl_tiny, s.snl_single, s.snl_first, s.snl_seq, s.snl_unit,
                 s.snl_urange, s.snl_runs, s.snl_ulvl, s.snl_nscr);
    solve_levels(true, s.snu_levels, s.snu_lvl, s.snu_tiny, s.snu_single, s.snu_first, s.snu_seq, s.snu_unit,
                 s.snu_urange, s.snu_runs, s.snu_ulvl, s.snu_nscr);
    for (int up = 0; up < 2; up++) {
        const std::vector<int> &seq = up ? s.snu_seq : s.snl_seq;
        std::vector<int> &sw = up ? s.snu_sw : s.snl_sw;
        sw.resize(2 * seq.size());
        for (size_t q = 0; q < seq.size(); q++) {
            sw[2 * q] = s0v[seq[q]];
            sw[2 * q + 1] = s0v[seq[q] + 1] - s0v[seq[q]];
        }
    }
    // (runs never outnumber the entries, which the int row pointers index)
    // ---- slot map: where each row of R lands in the target column (struct R is inside it)
    s.sn_map.resize((size_t)moff);
    auto fill = [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; i++) {
            const int k = it_k[i], S = it_S[i];
            const int s1 = s0v[S + 1];
            const int *rk = s.Fi_dev.data() + s.Dp[k];
            const int *rb = f.Fi.data() + lbeg(s1 - 1);
            const int mcnt = s.sn_item[4 * (size_t)i + 3];
            int pos = it_slot0[i] + it_len[i];          // R's rows lie below s1 - 1 in column k
            int *dst = s.sn_map.data() + s.sn_moff[i];
            for (int r = 0; r < mcnt; r++) {
                pos = (int)(std::lower_bound(rk + pos, rk + s.Dlen[k], rb[r]) - rk);
                dst[r] = pos;
            }
        }
    };
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (hw == 1 || moff < (1 << 20)) fill(0, nitems);
    else {
        std::vector<std::thread> th;
        int64_t i0 = 0;
        for (unsigned t = 1; t <= hw; t++) {
            const int64_t goal = moff * (int64_t)t / hw;
            int64_t i1 = std::lower_bound(s.sn_moff.begin(), s.sn_moff.end() - 1, goal) - s.sn_moff.begin();
            i1 = std::min(std::max(i1, i0), nitems);
            if (t == hw) i1 = nitems;
            if (i1 > i0) {
                try {
                    th.emplace_back(fill, i0, i1);
                } catch (...) {
                    fill(i0, i1);
                }
            }
            i0 = i1;
        }
        for (auto &x : th) x.join();
    }
}

void build_schedule(const Analysis &an, const Factor &f, const cktlu_options &opt, Schedule &s, int64_t map_cap) {
    const int n = an.n;
    s = Schedule();
    s.n = n;
    const int T = n - choose_tail(f, opt);
    s.tail0 = T;
    // ---- device layout: columns padded to whole cache lines
    const int al = cktlu_dev::kColAlign;
    s.Dp.assign(n + 1, 0);
    s.Dlen.resize(n);
    for (int k = 0; k < n; k++) {
        const int len = (int)(f.Fp[k + 1] - f.Fp[k]);
        s.Dlen[k] = len;
        s.Dp[k + 1] = s.Dp[k] + (len + al - 1) / al * al;
    }
    s.nnz_dev = s.Dp[n];
    s.Fi_dev.assign(s.nnz_dev, INT_MAX);
    for (int k = 0; k < n; k++)
        std::copy(f.Fi.begin() + f.Fp[k], f.Fi.begin() + f.Fp[k + 1], s.Fi_dev.begin() + s.Dp[k]);
    auto dpos = [&](int k, int64_t q) { return (int)(s.Dp[k] + (q - f.Fp[k])); };
    // ---- levels: column k depends on every j with U(j,k) != 0, j < k
    s.level.assign(n, 0);
    int maxlev = -1;
    for (int k = 0; k < n; k++) {
        int lev = 0;
        for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1; q++) lev = std::max(lev, s.level[f.Fi[q]] + 1);
        s.level[k] = lev;
        maxlev = std::max(maxlev, lev);
        s.max_col = std::max(s.max_col, (int)(f.Fp[k + 1] - f.Fp[k]));
    }
    s.nlevels = maxlev + 1;
    std::vector<int> cnt(s.nlevels + 1, 0);
    for (int k = 0; k < n; k++) cnt[s.level[k] + 1]++;
    for (int l = 0; l < s.nlevels; l++) {
        s.max_width = std::max(s.max_width, cnt[l + 1]);
        cnt[l + 1] += cnt[l];
    }
    // ---- value map: user nonzero p -> slot offset inside its factor column
    s.amap.resize(an.nnz);
    for (int c = 0; c < n; c++) {
        const int k = an.colinv[c];
        const int *beg = f.Fi.data() + f.Fp[k], *end = f.Fi.data() + f.Fp[k + 1];
        for (int p = an.Ap[c]; p < an.Ap[c + 1]; p++) {
            const int pos = f.posof[an.rowinv_pre[an.Ai[p]]];
            const int *it = std::lower_bound(beg, end, pos);
            s.amap[p] = (int)(it - beg);   // always found: struct(A) is inside struct(L+U)
        }
    }
    // ---- MAC count (Section VI arithmetic density)
    double macs = 0;
    for (int k = 0; k < n; k++)
        for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1; q++) {
            const int j = f.Fi[q];
            macs += (double)(f.Fp[j + 1] - f.Fp[j] - f.nU[j]);
        }
    s.macs = macs;
    s.flops = 2.0 * macs + (double)f.nnz_l();
    // ---- row-wise L (strictly lower) and U (strictly upper) for the solves
    s.Lrp.assign(n + 1, 0);
    s.Urp.assign(n + 1, 0);
    s.udiag.resize(n);
    for (int k = 0; k < n; k++) {
        const int64_t b = f.Fp[k], d = f.Fp[k] + f.nU[k] - 1, e = f.Fp[k + 1];
        for (int64_t q = b; q < d; q++) s.Urp[f.Fi[q] + 1]++;
        for (int64_t q = d + 1; q < e; q++) s.Lrp[f.Fi[q] + 1]++;
        s.udiag[k] = dpos(k, d);
    }
    for (int i = 0; i < n; i++) { s.Lrp[i + 1] += s.Lrp[i]; s.Urp[i + 1] += s.Urp[i]; }
    s.Lrj.resize(s.Lrp[n]); s.Lrsrc.resize(s.Lrp[n]);
    s.Urj.resize(s.Urp[n]); s.Ursrc.resize(s.Urp[n]);
    {
        std::vector<int> lf(s.Lrp.begin(), s.Lrp.end() - 1), uf(s.Urp.begin(), s.Urp.end() - 1);
        for (int k = 0; k < n; k++) {   // ascending k -> ascending column index inside each row
            const int64_t b = f.Fp[k], d = f.Fp[k] + f.nU[k] - 1, e = f.Fp[k + 1];
            for (int64_t q = b; q < d; q++) { int i = f.Fi[q]; s.Urj[uf[i]] = k; s.Ursrc[uf[i]++] = dpos(k, q); }
            for (int64_t q = d + 1; q < e; q++) { int i = f.Fi[q]; s.Lrj[lf[i]] = k; s.Lrsrc[lf[i]++] = dpos(k, q); }
        }
    }
    // ---- right-looking schedule of the sparse columns [0, T).  Column k must follow
    // every j with U(j,k) != 0 (its updates) and every j with L(k,j) != 0 (so that the
    // multiplier U(k,m) that row k holds in any target m is final when k updates m).
    // rlevel = longest path.  Columns [T, n) are update targets only (dense block).
    // With supernodes (the default) the sweep runs on the supernodal schedule built below
    // instead, and this column schedule is not built.
    const bool snodal = opt.sweep_supernodes >= 0;
    {
        // L entries of each sparse column in rows < T (they come first: rows ascend)
        std::vector<int> lo_cnt(T, 0);
        for (int j = 0; j < T; j++) {
            const int *b = f.Fi.data() + f.Fp[j] + f.nU[j], *e = f.Fi.data() + f.Fp[j + 1];
            lo_cnt[j] = (int)(std::lower_bound(b, e, T) - b);
        }
        if (!snodal) {
        std::vector<int> rlev(n, 0);
        int nl = T ? 1 : 0;
        for (int k = 0; k < T; k++) {
            int v = 0;
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1; q++) v = std::max(v, rlev[f.Fi[q]] + 1);
            for (int q = s.Lrp[k]; q < s.Lrp[k + 1]; q++) v = std::max(v, rlev[s.Lrj[q]] + 1);
            rlev[k] = v;
            nl = std::max(nl, v + 1);
        }
        s.n_rlevels = nl;
        std::vector<int> c(nl + 1, 0);
        for (int k = 0; k < T; k++) c[rlev[k] + 1]++;
        for (int l = 0; l < nl; l++) c[l + 1] += c[l];
        s.lvl_ptr.assign(c.begin(), c.end());
        s.seq.resize(T);
        for (int k = 0; k < T; k++) s.seq[c[rlev[k]]++] = k;
        // an item (j -> k) of a dense-block target updates only its rows < T (the rest is the
        // Schur update of the dense block, applied after the sweep); it exists if there are any
        auto keep = [&](int j, int k) { return k < T || lo_cnt[j] > 0; };
        // update tasks: items (j -> k) for U(j,k) != 0, j < min(k, T), in (rlevel(j), k, j)
        // order by a stable counting sort over the level (k and j ascend in column order)
        std::vector<int64_t> bucket(nl + 1, 0);
        for (int k = 0; k < n; k++)
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1 && f.Fi[q] < T; q++)
                if (keep(f.Fi[q], k)) bucket[rlev[f.Fi[q]] + 1]++;
        for (int l = 0; l < nl; l++) bucket[l + 1] += bucket[l];
        const int64_t nitems = bucket[nl];
        std::vector<int> it_k(nitems), it_j(nitems), it_slot(nitems);
        std::vector<int64_t> fillp(bucket.begin(), bucket.end() - 1);
        for (int k = 0; k < n; k++)
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1 && f.Fi[q] < T; q++) {
                const int j = f.Fi[q];
                if (!keep(j, k)) continue;
                const int64_t o = fillp[rlev[j]]++;
                it_k[o] = k;
                it_j[o] = j;
                it_slot[o] = (int)(q - f.Fp[k]);
            }
        s.task_ptr.assign(nl + 1, 0);
        s.task_tgt.clear();
        s.src_ptr.assign(1, 0);
        s.src_col.swap(it_j);
        s.src_slot.swap(it_slot);
        int l = 0;
        for (int64_t i = 0; i < nitems; i++) {
            while (i >= bucket[l + 1]) l++;
            if (i == bucket[l] || it_k[i] != it_k[i - 1]) {
                if (i > 0) s.src_ptr.push_back((int)i);
                s.task_tgt.push_back(it_k[i]);
                s.task_ptr[l + 1]++;
            }
        }
        if (nitems > 0) s.src_ptr.push_back((int)nitems);
        for (int q = 0; q < nl; q++) s.task_ptr[q + 1] += s.task_ptr[q];
        // packed device records.  colrec[i] = {Dp, nU, Dlen, column} of column seq[i].  Task t
        // is two int4s: {target k, Dp[k], length of the part of column k that is searched for
        // rows (all of it for k < T, its rows < T otherwise), first extra item} and its first
        // item; a sentinel task after the last one holds the end of the extra items.  An item
        // is {position of the pivot of its source j, begin and end of L(:,j), offset of row j
        // in the target column (where the multiplier U(j,k) lives)}; a task's items after the
        // first are item4[first extra item .. next task's first extra item).
        s.colrec.resize(4 * (size_t)T);
        for (int i = 0; i < T; i++) {
            const int j = s.seq[i];
            s.colrec[4 * (size_t)i + 0] = s.Dp[j];
            s.colrec[4 * (size_t)i + 1] = f.nU[j];
            s.colrec[4 * (size_t)i + 2] = s.Dlen[j];
            s.colrec[4 * (size_t)i + 3] = j;
        }
        auto item_of = [&](int64_t i, int k, int *dst) {
            const int j = s.src_col[i];
            dst[0] = s.Dp[j] + f.nU[j] - 1;
            dst[1] = s.Dp[j] + f.nU[j];
            dst[2] = k < T ? s.Dp[j] + s.Dlen[j] : s.Dp[j] + f.nU[j] + lo_cnt[j];
            dst[3] = s.src_slot[i];
        };
        const int ntasks = (int)s.task_tgt.size();
        s.task8.assign(8 * (size_t)(ntasks + 1), 0);
        s.item4.clear();
        for (int t = 0; t < ntasks; t++) {
            const int k = s.task_tgt[t];
            int slen = s.Dlen[k];
            if (k >= T) {
                const int *b = f.Fi.data() + f.Fp[k], *e = f.Fi.data() + f.Fp[k + 1];
                slen = (int)(std::lower_bound(b, e, T) - b);
            }
            int *rec = s.task8.data() + 8 * (size_t)t;
            rec[0] = k;
            rec[1] = s.Dp[k];
            rec[2] = slen;
            rec[3] = (int)(s.item4.size() / 4);
            item_of(s.src_ptr[t], k, rec + 4);
            for (int i = s.src_ptr[t] + 1; i < s.src_ptr[t + 1]; i++) {
                int it[4];
                item_of(i, k, it);
                s.item4.insert(s.item4.end(), it, it + 4);
            }
        }
        s.task8[8 * (size_t)ntasks + 3] = (int)(s.item4.size() / 4);
        // slot map: the slot in column k of every entry of every item, so that the device
        // loads it instead of searching column k's rows; items in the order the task
        // applies them, entries in L order; built in parallel over tasks
        s.smap.clear();
        s.tmoff.clear();
        if (map_cap < 0 && opt.sweep_slot_map == 0) {
            size_t fr = 0, tot = 0;
            map_cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)(0.25 * (double)fr / sizeof(int)) : 0;
        }
        if (opt.sweep_slot_map == 0 && ntasks > 0 && map_cap > 0) {
            std::vector<int64_t> off(ntasks + 1, 0);
            for (int t = 0; t < ntasks; t++) {
                int64_t len = 0;
                for (int i = s.src_ptr[t]; i < s.src_ptr[t + 1]; i++) {
                    int it[4];
                    item_of(i, s.task_tgt[t], it);
                    len += it[2] - it[1];
                }
                off[t + 1] = off[t] + len;
            }
            bool fits = off[ntasks] <= map_cap;
            if (fits) {
                try {                                  // host memory for the map: none, no map
                    s.tmoff.assign(off.begin(), off.end());
                    s.smap.resize((size_t)off[ntasks]);
                } catch (const std::bad_alloc &) {
                    std::vector<int>().swap(s.smap);
                    std::vector<int64_t>().swap(s.tmoff);
                    fits = false;
                }
            }
            if (fits) {
                auto fill = [&](int t0, int t1) {
                    for (int t = t0; t < t1; t++) {
                        const int k = s.task_tgt[t];
                        const int *rk = s.Fi_dev.data() + s.Dp[k];
                        const int slen = s.task8[8 * (size_t)t + 2];
                        int64_t o = off[t];
                        for (int i = s.src_ptr[t]; i < s.src_ptr[t + 1]; i++) {
                            int it[4];
                            item_of(i, k, it);
                            int pos = it[3] + 1;               // rows of L(:,j) lie below row j in column k
                            for (int q = it[1]; q < it[2]; q++) {
                                pos = (int)(std::lower_bound(rk + pos, rk + slen, s.Fi_dev[q]) - rk);
                                s.smap[(size_t)o++] = pos;   // struct(L(:,j)) is inside struct(column k)
                            }
                        }
                    }
                };
                const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
                if (hw == 1 || off[ntasks] < (1 << 20)) fill(0, ntasks);
                else {
                    // split by map entries so that the threads get similar work; a range whose
                    // thread cannot be started is filled here
                    std::vector<std::thread> th;
                    int t0 = 0;
                    for (unsigned w = 1; w <= hw; w++) {
                        const int64_t goal = off[ntasks] * (int64_t)w / hw;
                        int t1 = (int)(std::lower_bound(off.begin(), off.end(), goal) - off.begin());
                        t1 = std::min(std::max(t1, t0), ntasks);
                        if (w == hw) t1 = ntasks;
                        if (t1 > t0) {
                            try {
                                th.emplace_back(fill, t0, t1);
                            } catch (...) {
                                fill(t0, t1);
                            }
                        }
                        t0 = t1;
                    }
                    for (auto &x : th) x.join();
                }
            }
        }
        }  // !snodal
        // multiply-adds of the sweep: every source j < T of every column k, over L(:,j)
        // (a dense-block target only in its rows < T)
        s.macs_sweep = 0;
        for (int k = 0; k < n; k++)
            for (int64_t q = f.Fp[k]; q < f.Fp[k] + f.nU[k] - 1 && f.Fi[q] < T; q++) {
                const int j = f.Fi[q];
                s.macs_sweep += (double)(k < T ? s.Dlen[j] - f.nU[j] : lo_cnt[j]);
            }
        // Schur update of the dense block: per dense column, its U rows < T (the bridge) and,
        // per sparse column, the range of its L entries in rows >= T
        s.tail_nb.assign(n - T, 0);
        s.l21.assign(2 * (size_t)T, 0);
        s.macs_schur = 0;
        for (int j = 0; j < T; j++) {
            s.l21[2 * (size_t)j] = s.Dp[j] + f.nU[j] + lo_cnt[j];
            s.l21[2 * (size_t)j + 1] = s.Dp[j] + s.Dlen[j];
        }
        for (int k = T; k < n; k++) {
            const int *b = f.Fi.data() + f.Fp[k], *e = f.Fi.data() + f.Fp[k + 1];
            const int nb = (int)(std::lower_bound(b, e, T) - b);
            s.tail_nb[k - T] = nb;
            for (int q = 0; q < nb; q++) {
                const int j = b[q];
                s.macs_schur += (double)(s.Dlen[j] - f.nU[j] - lo_cnt[j]);
            }
        }
        // Schur parts: each dense column's bridge sources, in order, cut into parts of
        // similar cost (a source costs one round trip plus one per 64 entries), so that no
        // column's chain sets the kernel's time alone; part 0 updates S in place, each later
        // part a zeroed scratch column that the add pass folds into S in part order
        {
            const int Dn = n - T;
            std::vector<double> ccost(Dn, 0.0);
            auto scost = [&](int j) { return 1.0 + (double)(s.Dlen[j] - f.nU[j] - lo_cnt[j]) / 64.0; };
            double tot = 0.0;
            for (int c = 0; c < Dn; c++) {
                const int *b = f.Fi.data() + f.Fp[T + c];
                for (int q = 0; q < s.tail_nb[c]; q++) ccost[c] += scost(b[q]);
                tot += ccost[c];
            }
            const double budget = Dn > 0 ? std::max(1.0, 1.5 * tot / Dn) : 1.0;
            s.schur_parts.clear();
            s.schur_add.clear();
            s.schur_nscr = 0;
            for (int c = 0; c < Dn; c++) {
                const int *b = f.Fi.data() + f.Fp[T + c];
                const int nb = s.tail_nb[c];
                const int scr0 = s.schur_nscr;
                for (int q0 = 0, part = 0; q0 < nb; part++) {   // no part for a column without bridge
                    double acc = 0.0;
                    int q1 = q0;
                    while (q1 < nb && (q1 == q0 || acc + scost(b[q1]) <= budget)) acc += scost(b[q1++]);
                    const int scr = part == 0 ? -1 : s.schur_nscr++;
                    s.schur_parts.insert(s.schur_parts.end(), {c, q0, q1, scr});
                    q0 = q1;
                }
                if (s.schur_nscr > scr0) s.schur_add.insert(s.schur_add.end(), {c, scr0, s.schur_nscr - scr0, 0});
            }
        }
        s.lnz_front = 0;
        for (int k = 0; k < T; k++) s.lnz_front += (double)(s.Dlen[k] - f.nU[k]);
        // the method's own work and entries per phase (the compulsory bytes of the roofline)
        s.entries_sweep = 0;
        for (int k = 0; k < T; k++) s.entries_sweep += (double)s.Dlen[k];
        s.entries_dense = 0;
        s.macs_dense = 0;
        for (int k = T; k < n; k++) {
            s.entries_sweep += (double)s.tail_nb[k - T];
            s.entries_dense += (double)(s.Dlen[k] - s.tail_nb[k - T]);
            for (int64_t q = f.Fp[k] + s.tail_nb[k - T]; q < f.Fp[k] + f.nU[k] - 1; q++) {
                const int j = f.Fi[q];
                s.macs_dense += (double)(s.Dlen[j] - f.nU[j]);
            }
        }
    }
    if (snodal)
        build_supernodal(f, s, T, opt.sweep_supernodes > 0 ? std::min(opt.sweep_supernodes, 64) : 64,
                         opt.sweep_panel_rows > 0 ? opt.sweep_panel_rows : kPanelRows,
                         opt.solve_split_entries > 0 ? opt.solve_split_entries : kSolvePullChunk);
    // ---- solve levels of the sparse rows [0, T): row i of L waits for every j with
    // L(i,j) != 0, row i of U for every j > i with U(i,j) != 0 (rows >= T of U are
    // solved densely before any sparse U row).  The L sequence ends with one more
    // level holding the rows [T, n), which take only their entries in columns < T.
    auto order_by_level = [T](const std::vector<int> &lev, int nl, std::vector<int> &seq,
                              std::vector<int> &ptr) {
        std::vector<int> c(nl + 1, 0);
        for (int i = 0; i < T; i++) c[lev[i] + 1]++;
        for (int l = 0; l < nl; l++) c[l + 1] += c[l];
        ptr.assign(c.begin(), c.end());
        seq.resize(T);
        for (int i = 0; i < T; i++) seq[c[lev[i]]++] = i;
    };
    {
        std::vector<int> lev(n, 0);
        int nl = T ? 1 : 0;
        for (int i = 0; i < T; i++) {
            int v = 0;
            for (int q = s.Lrp[i]; q < s.Lrp[i + 1]; q++) v = std::max(v, lev[s.Lrj[q]] + 1);
            lev[i] = v;
            nl = std::max(nl, v + 1);
        }
        order_by_level(lev, nl, s.lseq, s.lsptr);
        if (T < n) {
            for (int i = T; i < n; i++) s.lseq.push_back(i);
            s.lsptr.push_back(n);
        }
        std::fill(lev.begin(), lev.end(), 0);
        nl = T ? 1 : 0;
        for (int i = T - 1; i >= 0; i--) {
            int v = 0;
            for (int q = s.Urp[i]; q < s.Urp[i + 1]; q++)
                if (s.Urj[q] < T) v = std::max(v, lev[s.Urj[q]] + 1);
            lev[i] = v;
            nl = std::max(nl, v + 1);
        }
        order_by_level(lev, nl, s.useq, s.usptr);
        s.tail_rend.resize(n - T);
        for (int i = T; i < n; i++) {
            int q = s.Lrp[i];
            while (q < s.Lrp[i + 1] && s.Lrj[q] < T) q++;
            s.tail_rend[i - T] = q;
        }
        // packed device records: per solve position {row, first entry, end, position of the
        // diagonal}; per entry {column, position of the value}
        s.lrec.resize(4 * s.lseq.size());
        for (size_t q = 0; q < s.lseq.size(); q++) {
            const int i = s.lseq[q];
            s.lrec[4 * q + 0] = i;
            s.lrec[4 * q + 1] = s.Lrp[i];
            s.lrec[4 * q + 2] = i >= T ? s.tail_rend[i - T] : s.Lrp[i + 1];
            s.lrec[4 * q + 3] = s.udiag[i];
        }
        s.urec.resize(4 * s.useq.size());
        for (size_t q = 0; q < s.useq.size(); q++) {
            const int i = s.useq[q];
            s.urec[4 * q + 0] = i;
            s.urec[4 * q + 1] = s.Urp[i];
            s.urec[4 * q + 2] = s.Urp[i + 1];
            s.urec[4 * q + 3] = s.udiag[i];
        }
        s.Lrjs.resize(2 * s.Lrj.size());
        for (size_t q = 0; q < s.Lrj.size(); q++) { s.Lrjs[2 * q] = s.Lrj[q]; s.Lrjs[2 * q + 1] = s.Lrsrc[q]; }
        s.Urjs.resize(2 * s.Urj.size());
        for (size_t q = 0; q < s.Urj.size(); q++) { s.Urjs[2 * q] = s.Urj[q]; s.Urjs[2 * q + 1] = s.Ursrc[q]; }
        // launch segments {first level, end level, kind}: kind 2 = a level with a row longer
        // than kSolveLongRow entries (a workgroup per row); kind 1 = a run of two or more
        // consecutive narrow levels of short rows (one chained launch, a workgroup per
        // instance stepping through them); kind 0 = one level, a wavefront per row
        const int cw = opt.solve_chain_width == 0 ? -1 : opt.solve_chain_width;
        auto segments = [cw](const std::vector<int> &ptr, const std::vector<int> &rec, std::vector<int> &seg) {
            seg.clear();
            const int nl = (int)ptr.size() - 1;
            auto long_rows = [&](int l) {
                for (int q = ptr[l]; q < ptr[l + 1]; q++)
                    if (rec[4 * q + 2] - rec[4 * q + 1] > cktlu_dev::kSolveLongRow) return true;
                return false;
            };
            for (int l = 0; l < nl;) {
                if (long_rows(l)) {
                    seg.insert(seg.end(), {l, l + 1, 2});
                    l++;
                    continue;
                }
                int e = l;
                while (cw > 0 && e < nl && ptr[e + 1] - ptr[e] <= cw && !long_rows(e)) e++;
                if (e - l >= 2) {
                    seg.insert(seg.end(), {l, e, 1});
                    l = e;
                } else {
                    seg.insert(seg.end(), {l, l + 1, 0});
                    l++;
                }
            }
        };
        segments(s.lsptr, s.lrec, s.lseg);
        segments(s.usptr, s.urec, s.useg);
    }
    s.rowperm_final.resize(n);
    for (int k = 0; k < n; k++) s.rowperm_final[k] = an.rowperm_pre[f.pivrow[k]];
    // ---- user-space CSR of A for residuals
    s.Acp.assign(n + 1, 0);
    for (int64_t p = 0; p < an.nnz; p++) s.Acp[an.Ai[p] + 1]++;
    for (int i = 0; i < n; i++) s.Acp[i + 1] += s.Acp[i];
    s.Acj.resize(an.nnz);
    s.Acsrc.resize(an.nnz);
    {
        std::vector<int> fill(s.Acp.begin(), s.Acp.end() - 1);
        for (int c = 0; c < n; c++)
            for (int p = an.Ap[c]; p < an.Ap[c + 1]; p++) {
                int r = an.Ai[p];
                s.Acj[fill[r]] = c;
                s.Acsrc[fill[r]++] = p;
            }
    }
}

}  // namespace cktlu
