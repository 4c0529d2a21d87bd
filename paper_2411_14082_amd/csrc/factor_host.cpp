// Host factorization with threshold pivoting (Section II-A, Algorithm 1 on
// the transpose) and the tail re-factorization used by the pivot-check
// fallback (Sections IV-C and IV-D).
//
// Rows are tracked by their A_hat index while the factorization runs because
// a later exchange can still move a not-yet-pivotal row to another position;
// the result is renumbered into final positions at the end.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace cktlu {

void restart_closure(const std::vector<int> &parent, const std::vector<char> &unfinished,
                     std::vector<char> &in_set) {
    const int n = (int)parent.size();
    in_set.assign(n, 0);
    // parent[j] > j, so one ascending sweep propagates membership to ancestors
    for (int j = 0; j < n; j++) {
        if (unfinished[j]) in_set[j] = 1;
        if (in_set[j] && parent[j] >= 0) in_set[parent[j]] = 1;
    }
}

namespace {

struct ColStore {
    // per finished column, in A_hat-row space: L rows/values and U columns/values
    std::vector<int64_t> lptr{0}, uptr{0};
    std::vector<int> lrow, ucol;
    std::vector<double> lval, uval;
    std::vector<double> diag;
};

}  // namespace

int host_gp_factor(const Analysis &an, const double *values, double eps,
                   const std::vector<int> &init_pivrow, const Factor *prev,
                   const std::vector<char> *keep, Factor &out, int &fail_col, int &nswaps,
                   const DenseSource *dsrc) {
    const int n = an.n;
    fail_col = -1;
    nswaps = 0;
    std::vector<int> pivrow(init_pivrow), posof(n);
    for (int k = 0; k < n; k++) posof[pivrow[k]] = k;
    // dense source: final positions of every row after the block's exchanges
    std::vector<int> fpos;
    if (dsrc) {
        if (!prev || dsrc->T + dsrc->D != n) return CKTLU_E_STATE;
        std::vector<int> fr(pivrow);
        for (int c = 0; c < dsrc->D; c++) std::swap(fr[dsrc->T + c], fr[dsrc->T + dsrc->swap[c]]);
        fpos.resize(n);
        for (int q = 0; q < n; q++) fpos[fr[q]] = q;
    }
    std::vector<int> pivcol(n, -1);          // A_hat row -> column it is pivot of
    std::vector<int> stamp(n, -1), reach, deps, queue;
    std::vector<double> x(n, 0.0);
    ColStore cs;
    cs.diag.resize(n);
    reach.reserve(1024);

    for (int k = 0; k < n; k++) {
        if (keep && prev && (*keep)[k]) {
            // column kept from the previous factorization (its pivot is unchanged)
            const int64_t b = prev->Fp[k], e = prev->Fp[k + 1];
            const int nu = prev->nU[k];
            if (pivrow[k] != prev->pivrow[k]) return CKTLU_E_STATE;
            for (int64_t q = b; q < b + nu - 1; q++) {
                cs.ucol.push_back(prev->Fi[q]);
                cs.uval.push_back(prev->Fx[q]);
            }
            cs.diag[k] = prev->Fx[b + nu - 1];
            for (int64_t q = b + nu; q < e; q++) {
                cs.lrow.push_back(prev->pivrow[prev->Fi[q]]);
                cs.lval.push_back(prev->Fx[q]);
            }
            pivcol[pivrow[k]] = k;
            cs.lptr.push_back((int64_t)cs.lrow.size());
            cs.uptr.push_back((int64_t)cs.ucol.size());
            continue;
        }
        // symbolic: rows reachable from struct(A_hat(:,k)) (breadth-first)
        reach.clear();
        for (int p = an.Hp[k]; p < an.Hp[k + 1]; p++) {
            int r = an.Hi[p];
            if (stamp[r] != k) { stamp[r] = k; reach.push_back(r); }
        }
        for (size_t h = 0; h < reach.size(); h++) {
            int j = pivcol[reach[h]];
            if (j < 0) continue;
            for (int64_t q = cs.lptr[j]; q < cs.lptr[j + 1]; q++) {
                int s = cs.lrow[q];
                if (stamp[s] != k) { stamp[s] = k; reach.push_back(s); }
            }
        }
        // dependencies in ascending column order (a topological order)
        deps.clear();
        for (int r : reach) {
            x[r] = 0.0;
            if (pivcol[r] >= 0) deps.push_back(pivcol[r]);
        }
        std::sort(deps.begin(), deps.end());
        if (dsrc && k >= dsrc->T) {
            // pivot and values from the dense source: the exchange it made at this step,
            // U entries in rows < T from prev, the rest from the block in final positions
            const int T = dsrc->T, D = dsrc->D;
            const double *Sk = dsrc->S + (size_t)(k - T) * D;
            const int d = pivrow[k], piv = pivrow[T + dsrc->swap[k - T]];
            if (pivcol[piv] >= 0 || stamp[piv] != k) return CKTLU_E_STATE;   // not a candidate
            if (piv != d) {
                const int q = posof[piv];
                pivrow[q] = d;  posof[d] = q;
                pivrow[k] = piv; posof[piv] = k;
                nswaps++;
            }
            const int64_t pb = prev->Fp[k];
            const int pnu = prev->nU[k];
            for (int j : deps) {
                double v;
                if (j < T) {
                    const int *b = prev->Fi.data() + pb, *e = b + pnu - 1;
                    const int *f = std::lower_bound(b, e, j);
                    if (f == e || *f != j) return CKTLU_E_STATE;
                    v = prev->Fx[pb + (f - b)];
                } else {
                    v = Sk[j - T];
                }
                cs.ucol.push_back(j);
                cs.uval.push_back(v);
            }
            cs.diag[k] = Sk[k - T];
            for (int r : reach)
                if (pivcol[r] < 0 && r != piv) {
                    cs.lrow.push_back(r);
                    cs.lval.push_back(Sk[fpos[r] - T]);
                }
            pivcol[piv] = k;
            cs.lptr.push_back((int64_t)cs.lrow.size());
            cs.uptr.push_back((int64_t)cs.ucol.size());
            continue;
        }
        for (int p = an.Hp[k]; p < an.Hp[k + 1]; p++) x[an.Hi[p]] = values[an.Hsrc[p]];
        for (int j : deps) {
            const double xj = x[pivrow[j]];
            for (int64_t q = cs.lptr[j]; q < cs.lptr[j + 1]; q++) x[cs.lrow[q]] -= cs.lval[q] * xj;
        }
        // threshold pivot among the candidates (reached rows not yet pivotal)
        const int d = pivrow[k];
        bool have_d = false, bad = false;
        int best = -1;
        double best_abs = -1.0, others = 0.0;
        for (int r : reach) {
            if (pivcol[r] >= 0) continue;
            const double v = x[r], a = std::fabs(v);
            if (!std::isfinite(v)) bad = true;
            if (r == d) have_d = true;
            else others = std::max(others, a);
            if (a > best_abs || (a == best_abs && posof[r] < posof[best])) { best_abs = a; best = r; }
        }
        if (best < 0) { fail_col = k; return CKTLU_E_STRUCT_SINGULAR; }
        if (bad) { fail_col = k; return CKTLU_E_NUM_SINGULAR; }
        int piv = d;
        if (!(have_d && x[d] != 0.0 && std::fabs(x[d]) >= eps * others)) {
            piv = best;
            if (x[piv] == 0.0) { fail_col = k; return CKTLU_E_NUM_SINGULAR; }
            if (piv != d) {
                const int q = posof[piv];
                pivrow[q] = d;  posof[d] = q;
                pivrow[k] = piv; posof[piv] = k;
                nswaps++;
            }
        }
        const double xp = x[piv];
        for (int j : deps) {
            cs.ucol.push_back(j);
            cs.uval.push_back(x[pivrow[j]]);
        }
        cs.diag[k] = xp;
        for (int r : reach)
            if (pivcol[r] < 0 && r != piv) {
                cs.lrow.push_back(r);
                cs.lval.push_back(x[r] / xp);
            }
        pivcol[piv] = k;
        cs.lptr.push_back((int64_t)cs.lrow.size());
        cs.uptr.push_back((int64_t)cs.ucol.size());
    }

    // ---- final positions, combined column storage
    out = Factor();
    out.n = n;
    out.pivrow = pivrow;
    out.posof = posof;
    out.Fp.assign(n + 1, 0);
    out.nU.resize(n);
    for (int k = 0; k < n; k++) {
        out.nU[k] = (int)(cs.uptr[k + 1] - cs.uptr[k]) + 1;
        out.Fp[k + 1] = out.Fp[k] + out.nU[k] + (cs.lptr[k + 1] - cs.lptr[k]);
    }
    out.Fi.resize(out.Fp[n]);
    out.Fx.resize(out.Fp[n]);
    std::vector<std::pair<int, double>> tmp;
    for (int k = 0; k < n; k++) {
        int64_t o = out.Fp[k];
        tmp.clear();
        for (int64_t q = cs.uptr[k]; q < cs.uptr[k + 1]; q++) tmp.emplace_back(cs.ucol[q], cs.uval[q]);
        std::sort(tmp.begin(), tmp.end(),
                  [](const std::pair<int, double> &a, const std::pair<int, double> &b) { return a.first < b.first; });
        for (auto &t : tmp) { out.Fi[o] = t.first; out.Fx[o] = t.second; o++; }
        out.Fi[o] = k; out.Fx[o] = cs.diag[k]; o++;
        tmp.clear();
        for (int64_t q = cs.lptr[k]; q < cs.lptr[k + 1]; q++) tmp.emplace_back(posof[cs.lrow[q]], cs.lval[q]);
        std::sort(tmp.begin(), tmp.end(),
                  [](const std::pair<int, double> &a, const std::pair<int, double> &b) { return a.first < b.first; });
        for (auto &t : tmp) { out.Fi[o] = t.first; out.Fx[o] = t.second; o++; }
    }
    return CKTLU_OK;
}

}  // namespace cktlu
