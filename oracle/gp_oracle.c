/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded FP64 reference for the sparse LU hot path.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code; the product library never calls it and shares no code,
 * header or table with it.
 *
 * Orientation.  The paper stores matrices by rows and runs the up-looking form
 * of the Gilbert-Peierls algorithm (Section II-A, Algorithm 1).  This file
 * runs the same algorithm on the transpose: matrices are CSC and factored
 * column by column (left-looking).  Row k of the paper is column k here; the
 * pivot search that the paper runs along a row of U runs here down the
 * not-yet-pivotal part of a column, and pivoting exchanges rows.
 *
 * Notation.  A-hat(i,j) = A(rowperm[i], colperm[j]) is the pre-processed
 * matrix (Section III-A: static pivoting and fill-reducing ordering, taken as
 * given here).  pivrow[k] is the A-hat row that sits in position k; the result
 * satisfies A-hat(pivrow, :) = L * U with unit-diagonal L.
 *
 * Readings of points the paper leaves open (each documented in the design
 * notes next to the tests):
 *   - the threshold test keeps the preferred row d when x(d) is finite and
 *     nonzero and |x(d)| >= eps * max{|x(c)| : c candidate, c != d};
 *   - the preferred row of column k is the row currently in position k
 *     (pivrow[k]), which is the identity for a first factorization and the
 *     previous pivot sequence for a re-factorization (Section II-A: the
 *     re-factorization reuses the previous pivoting order);
 *   - "exchange" swaps positions k and pos(p) (LAPACK-style);
 *   - ties in the arg-max go to the smallest current position;
 *   - every structurally reached entry is stored, exact zeros included;
 *   - any non-finite candidate value makes the column numerically singular.
 *
 * Parity status: the LU, the solves, the levels, the column elimination tree
 * and the restart closure are all pinned by independent checks in the tests
 * (dense brute force, LAPACK pivots, closed forms, exact integer systems).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_STRUCT_SINGULAR (-1)
#define OR_NUM_SINGULAR (-2)
#define OR_NOMEM (-3)
#define OR_BADARG (-4)

typedef struct {
    int n;
    int status;     /* OR_* code */
    int fail_col;   /* column that failed, or -1 */
    int nswaps;     /* number of exchanges that the threshold rule made */
    int *pivrow;    /* [n] position -> A-hat row */
    int *Lp, *Li;   /* CSC of strictly lower L, rows are final positions, sorted */
    double *Lx;
    int *Up, *Ui;   /* CSC of U, rows are positions <= k, sorted (diagonal last) */
    double *Ux;
} or_lu;

/* growable arrays ------------------------------------------------------ */
typedef struct { int *i; double *x; long len, cap; } vec_id;

static int vec_push(vec_id *v, int i, double x) {
    if (v->len == v->cap) {
        long nc = v->cap ? 2 * v->cap : 1024;
        int *ni = (int *)realloc(v->i, nc * sizeof(int));
        if (!ni) return 0;
        v->i = ni;
        double *nx = (double *)realloc(v->x, nc * sizeof(double));
        if (!nx) return 0;
        v->x = nx;
        v->cap = nc;
    }
    v->i[v->len] = i;
    v->x[v->len] = x;
    v->len++;
    return 1;
}

static void sort_pairs(int *idx, double *val, long m) {
    /* insertion sort: columns are short and this is the oracle */
    for (long a = 1; a < m; a++) {
        int ki = idx[a];
        double kv = val[a];
        long b = a - 1;
        while (b >= 0 && idx[b] > ki) {
            idx[b + 1] = idx[b];
            val[b + 1] = val[b];
            b--;
        }
        idx[b + 1] = ki;
        val[b + 1] = kv;
    }
}

void or_lu_free(or_lu *f) {
    if (!f) return;
    free(f->pivrow); free(f->Lp); free(f->Li); free(f->Lx);
    free(f->Up); free(f->Ui); free(f->Ux);
    memset(f, 0, sizeof(*f));
}

/*
 * Gilbert-Peierls left-looking LU with threshold partial pivoting
 * (Section II-A, Algorithm 1, transposed to columns).
 *
 * For each column k:
 *   1. symbolic prediction: the rows reachable from struct(A-hat(:,k)) in the
 *      graph whose edges lead from the pivot row of each finished column j to
 *      the rows of L(:,j); ordered topologically by depth-first postorder;
 *   2. numerical update: x = A-hat(:,k), then for each reached pivot row in
 *      topological order, x(rows of L(:,j)) -= L(:,j) * x(pivot row of j);
 *   3. pivoting: threshold test of the preferred row against the largest
 *      candidate, exchange on failure;
 *   4. store U(:,k) (pivotal rows and the pivot) and L(:,k) = x / pivot.
 */
int or_gp_lu(int n, const int *Ap, const int *Ai, const double *Ax,
             const int *rowperm, const int *colperm, double eps,
             const int *init_pivrow, or_lu *out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    out->fail_col = -1;
    if (n < 0) return out->status = OR_BADARG;

    int *rowinv = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *pivrow = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *posof = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *pivotal = (int *)malloc((size_t)(n + 1) * sizeof(int)); /* -1 or the column */
    int *visited = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *stack = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *child = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *post = (int *)malloc((size_t)(n + 1) * sizeof(int));
    double *x = (double *)malloc((size_t)(n + 1) * sizeof(double));
    long *lptr = (long *)malloc((size_t)(n + 2) * sizeof(long));
    long *uptr = (long *)malloc((size_t)(n + 2) * sizeof(long));
    vec_id Lc = {0}, Uc = {0};
    int status = OR_OK;
    if (!rowinv || !pivrow || !posof || !pivotal || !visited || !stack || !child ||
        !post || !x || !lptr || !uptr) {
        status = OR_NOMEM;
        goto done;
    }
    for (int i = 0; i < n; i++) rowinv[rowperm[i]] = i;
    for (int k = 0; k < n; k++) {
        pivrow[k] = init_pivrow ? init_pivrow[k] : k;
        posof[pivrow[k]] = k;
        pivotal[k] = -1;
        visited[k] = -1;
    }
    lptr[0] = 0;
    uptr[0] = 0;

    for (int k = 0; k < n; k++) {
        int c = colperm[k];
        /* 1. symbolic prediction by depth-first search */
        int npost = 0;
        for (int p = Ap[c]; p < Ap[c + 1]; p++) {
            int r0 = rowinv[Ai[p]];
            if (visited[r0] == k) continue;
            int top = 0;
            stack[0] = r0;
            visited[r0] = k;
            child[0] = 0;
            while (top >= 0) {
                int r = stack[top];
                int j = pivotal[r];
                int pushed = 0;
                if (j >= 0) {
                    long beg = lptr[j], end = lptr[j + 1];
                    while (beg + child[top] < end) {
                        int s = Lc.i[beg + child[top]];
                        child[top]++;
                        if (visited[s] != k) {
                            visited[s] = k;
                            top++;
                            stack[top] = s;
                            child[top] = 0;
                            pushed = 1;
                            break;
                        }
                    }
                }
                if (!pushed) {
                    post[npost++] = r;
                    top--;
                }
            }
        }
        /* 2. numerical update in topological order (reverse postorder) */
        for (int t = 0; t < npost; t++) x[post[t]] = 0.0;
        for (int p = Ap[c]; p < Ap[c + 1]; p++) x[rowinv[Ai[p]]] = Ax[p];
        for (int t = npost - 1; t >= 0; t--) {
            int r = post[t];
            int j = pivotal[r];
            if (j < 0) continue;
            double xr = x[r];
            for (long q = lptr[j]; q < lptr[j + 1]; q++) x[Lc.i[q]] -= Lc.x[q] * xr;
        }
        /* 3. threshold pivoting over the candidates (non-pivotal reached rows) */
        int d = pivrow[k];
        int d_is_cand = 0, best = -1, nonfinite = 0;
        double best_abs = -1.0, m_other = 0.0;
        for (int t = 0; t < npost; t++) {
            int r = post[t];
            if (pivotal[r] >= 0) continue;
            double a = fabs(x[r]);
            if (!isfinite(x[r])) nonfinite = 1;
            if (r == d) d_is_cand = 1; else if (a > m_other) m_other = a;
            if (a > best_abs || (a == best_abs && posof[r] < posof[best])) {
                best_abs = a;
                best = r;
            }
        }
        if (best < 0) {                 /* no candidate row: structurally singular */
            status = OR_STRUCT_SINGULAR;
            out->fail_col = k;
            goto done;
        }
        if (nonfinite) {
            status = OR_NUM_SINGULAR;
            out->fail_col = k;
            goto done;
        }
        int piv = d;
        if (!(d_is_cand && x[d] != 0.0 && fabs(x[d]) >= eps * m_other)) {
            piv = best;
            if (x[piv] == 0.0) {
                status = OR_NUM_SINGULAR;
                out->fail_col = k;
                goto done;
            }
            if (piv != d) {             /* exchange positions k and pos(piv) */
                int q = posof[piv];
                pivrow[k] = piv; posof[piv] = k;
                pivrow[q] = d;   posof[d] = q;
                out->nswaps++;
            }
        }
        /* 4. store U(:,k) and L(:,k) */
        double xp = x[piv];
        for (int t = 0; t < npost; t++) {
            int r = post[t];
            if (pivotal[r] >= 0) {
                if (!vec_push(&Uc, pivotal[r], x[r])) { status = OR_NOMEM; goto done; }
            }
        }
        sort_pairs(Uc.i + uptr[k], Uc.x + uptr[k], Uc.len - uptr[k]);
        if (!vec_push(&Uc, k, xp)) { status = OR_NOMEM; goto done; }
        for (int t = 0; t < npost; t++) {
            int r = post[t];
            if (pivotal[r] < 0 && r != piv) {
                if (!vec_push(&Lc, r, x[r] / xp)) { status = OR_NOMEM; goto done; }
            }
        }
        pivotal[piv] = k;
        lptr[k + 1] = Lc.len;
        uptr[k + 1] = Uc.len;
    }

    /* renumber L rows from A-hat rows to final positions, sort each column */
    for (long q = 0; q < Lc.len; q++) Lc.i[q] = posof[Lc.i[q]];
    for (int k = 0; k < n; k++) sort_pairs(Lc.i + lptr[k], Lc.x + lptr[k], lptr[k + 1] - lptr[k]);

    out->pivrow = pivrow; pivrow = NULL;
    out->Lp = (int *)malloc((size_t)(n + 1) * sizeof(int));
    out->Up = (int *)malloc((size_t)(n + 1) * sizeof(int));
    if (!out->Lp || !out->Up) { status = OR_NOMEM; goto done; }
    for (int k = 0; k <= n; k++) { out->Lp[k] = (int)lptr[k]; out->Up[k] = (int)uptr[k]; }
    out->Li = Lc.i; out->Lx = Lc.x; Lc.i = NULL; Lc.x = NULL;
    out->Ui = Uc.i; out->Ux = Uc.x; Uc.i = NULL; Uc.x = NULL;
    if (!out->Li) { out->Li = (int *)malloc(sizeof(int)); out->Lx = (double *)malloc(sizeof(double)); }

done:
    free(rowinv); free(pivrow); free(posof); free(pivotal); free(visited);
    free(stack); free(child); free(post); free(x); free(lptr); free(uptr);
    free(Lc.i); free(Lc.x); free(Uc.i); free(Uc.x);
    out->status = status;
    return status;
}

/* Forward substitution with unit-diagonal L in CSC (Section II-C, Algorithm 2,
 * column-oriented form).  b and y may alias. */
void or_lsolve(int n, const int *Lp, const int *Li, const double *Lx,
               const double *b, double *y) {
    if (y != b) memcpy(y, b, (size_t)n * sizeof(double));
    for (int j = 0; j < n; j++) {
        double yj = y[j];
        for (int p = Lp[j]; p < Lp[j + 1]; p++) y[Li[p]] -= Lx[p] * yj;
    }
}

/* Back substitution with U in CSC, diagonal stored last in each column
 * (Section II-C: the upper solve traverses the rows in reverse order). */
void or_usolve(int n, const int *Up, const int *Ui, const double *Ux,
               const double *y, double *x) {
    if (x != y) memcpy(x, y, (size_t)n * sizeof(double));
    for (int j = n - 1; j >= 0; j--) {
        int dpos = Up[j + 1] - 1;
        x[j] /= Ux[dpos];
        double xj = x[j];
        for (int p = Up[j]; p < dpos; p++) x[Ui[p]] -= Ux[p] * xj;
    }
}

/* Level of every column of the dependency graph given by the U pattern
 * (Section II-B: the level is the longest path from a source; column k depends
 * on column j iff U(j,k) != 0, j < k).  Sources are level 0. */
void or_levels(int n, const int *Up, const int *Ui, int *level) {
    for (int k = 0; k < n; k++) {
        int lev = 0;
        for (int p = Up[k]; p < Up[k + 1]; p++) {
            int j = Ui[p];
            if (j < k && level[j] + 1 > lev) lev = level[j] + 1;
        }
        level[k] = lev;
    }
}

/*
 * Column elimination tree by brute force (Section II-B): form the pattern of
 * M = A-hat' * A-hat explicitly, run a symbolic Cholesky on it, and take
 * parent(j) = smallest row index i > j with Lc(i,j) != 0 (-1 for a root).
 * Symbolic Cholesky: struct(Lc(:,j)) = {i > j : M(i,j) != 0} united with
 * struct(Lc(:,c)) minus {j} for every column c whose parent is j.
 * Quadratic memory in the worst case; meant for test-sized inputs.
 */
int or_coletree(int n, const int *Hp, const int *Hi, int *parent) {
    /* row lists of A-hat */
    int nnz = Hp[n];
    int *rp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *ri = (int *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
    char *dense = NULL;
    int **cols = (int **)calloc((size_t)n, sizeof(int *));
    int *clen = (int *)calloc((size_t)n, sizeof(int));
    int *mark = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
    int *buf = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
    int rc = OR_OK;
    (void)dense;
    if (!rp || !ri || !cols || !clen || !mark || !buf) { rc = OR_NOMEM; goto out; }
    for (int p = 0; p < nnz; p++) rp[Hi[p] + 1]++;
    for (int i = 0; i < n; i++) rp[i + 1] += rp[i];
    {
        int *fill = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
        if (!fill) { rc = OR_NOMEM; goto out; }
        memcpy(fill, rp, (size_t)n * sizeof(int));
        for (int j = 0; j < n; j++)
            for (int p = Hp[j]; p < Hp[j + 1]; p++) ri[fill[Hi[p]]++] = j;
        free(fill);
    }
    for (int i = 0; i < n; i++) mark[i] = -1;
    for (int j = 0; j < n; j++) {
        int m = 0;
        /* lower part of column j of M: columns i > j sharing a row with j */
        for (int p = Hp[j]; p < Hp[j + 1]; p++) {
            int row = Hi[p];
            for (int q = rp[row]; q < rp[row + 1]; q++) {
                int i = ri[q];
                if (i > j && mark[i] != j) { mark[i] = j; buf[m++] = i; }
            }
        }
        /* children's structures */
        for (int c = 0; c < j; c++) {
            if (parent[c] != j) continue;
            for (int t = 0; t < clen[c]; t++) {
                int i = cols[c][t];
                if (i > j && mark[i] != j) { mark[i] = j; buf[m++] = i; }
            }
            free(cols[c]); cols[c] = NULL; clen[c] = 0;
        }
        int par = -1;
        for (int t = 0; t < m; t++) if (par < 0 || buf[t] < par) par = buf[t];
        parent[j] = par;
        cols[j] = (int *)malloc((size_t)(m ? m : 1) * sizeof(int));
        if (!cols[j]) { rc = OR_NOMEM; goto out; }
        memcpy(cols[j], buf, (size_t)m * sizeof(int));
        clen[j] = m;
    }
out:
    if (cols) for (int j = 0; j < n; j++) free(cols[j]);
    free(cols); free(clen); free(rp); free(ri); free(mark); free(buf);
    return rc;
}

/* Restart set (Section IV-C): every unfinished column plus everything
 * reachable from it along elimination-tree parent pointers. */
void or_restart_set(int n, const int *parent, const int *unfinished, int *in_set) {
    int *queue = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
    int head = 0, tail = 0;
    for (int k = 0; k < n; k++) {
        in_set[k] = 0;
    }
    for (int k = 0; k < n; k++)
        if (unfinished[k] && !in_set[k]) { in_set[k] = 1; queue[tail++] = k; }
    while (head < tail) {
        int k = queue[head++];
        int p = parent[k];
        if (p >= 0 && !in_set[p]) { in_set[p] = 1; queue[tail++] = p; }
    }
    free(queue);
}

/* Count of multiply-add operations in a left-looking factorization with the
 * given patterns (used for the arithmetic density of Section VI). */
double or_mac_count(int n, const int *Lp, const int *Up, const int *Ui) {
    double macs = 0.0;
    for (int k = 0; k < n; k++)
        for (int p = Up[k]; p < Up[k + 1] - 1; p++) {
            int j = Ui[p];
            macs += (double)(Lp[j + 1] - Lp[j]);
        }
    return macs;
}

/* Transposed solves, used only by the condition estimate of the tests
 * (Section II-C's two substitutions applied to U' and L').
 * or_utsolve: U' z = c with U in CSC (diagonal last in each column): U' is
 * lower triangular and column j of U is row j of U', so z(j) is
 * (c(j) - sum_{i<j} U(i,j) z(i)) / U(j,j), j ascending.  c and z may alias. */
void or_utsolve(int n, const int *Up, const int *Ui, const double *Ux,
                const double *c, double *z) {
    if (z != c) memcpy(z, c, (size_t)n * sizeof(double));
    for (int j = 0; j < n; j++) {
        int dpos = Up[j + 1] - 1;
        double s = z[j];
        for (int p = Up[j]; p < dpos; p++) s -= Ux[p] * z[Ui[p]];
        z[j] = s / Ux[dpos];
    }
}

/* or_ltsolve: L' w = z with unit-diagonal L in CSC: L' is unit upper
 * triangular and column j of L is row j of L', so w(j) is
 * z(j) - sum_{i>j} L(i,j) w(i), j descending.  z and w may alias. */
void or_ltsolve(int n, const int *Lp, const int *Li, const double *Lx,
                const double *z, double *w) {
    if (w != z) memcpy(w, z, (size_t)n * sizeof(double));
    for (int j = n - 1; j >= 0; j--) {
        double s = w[j];
        for (int p = Lp[j]; p < Lp[j + 1]; p++) s -= Lx[p] * w[Li[p]];
        w[j] = s;
    }
}

/*
 * First-order bound on the rounding error of every factor entry (running error
 * analysis of the column update of Section II-A, done on absolute values).  The
 * tests compare two factorizations computed in different orders (the library's
 * and this oracle's) against the sum of their bounds.
 *
 * Column k is rebuilt from the given factors in the update order: for each source
 * j (U(j,k) != 0, ascending), U(j,k) is final, and its error is what it inherited
 * plus the rounding of its own sum, at most gamma_{g(m+1)} times the sum of the
 * absolute values of its terms (m terms were subtracted; |A(j,k)| is bounded by
 * |U(j,k)| plus the subtracted magnitudes, hence |U(j,k)| + 2 s).  The update
 * x(r) -= L(r,j) U(j,k) passes |L(r,j)| e_U(j,k) + e_L(r,j) |U(j,k)| on to x(r).
 * The pivot is rounded likewise; L(r,k) = x(r) / U(k,k) adds the pivot's error
 * times |L(r,k)| / |U(k,k)| and one rounding of the division.  g is the number
 * of roundings per product (1 for this oracle, more for an implementation that
 * forms a product in several steps).  Inputs: the oracle's CSC factors (rows
 * sorted, U's diagonal last).  Outputs eL[nnz(L)], eU[nnz(U)] in the same order.
 */
static double or_gamma(double m) {
    const double u = 1.1102230246251565e-16;   /* 2^-53 */
    return m * u / (1.0 - m * u);
}

int or_lu_errbound(int n, const int *Lp, const int *Li, const double *Lx,
                   const int *Up, const int *Ui, const double *Ux, double g,
                   double *eL, double *eU) {
    double *e = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    double *s = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    int *cnt = (int *)calloc((size_t)(n ? n : 1), sizeof(int));
    if (!e || !s || !cnt) { free(e); free(s); free(cnt); return OR_NOMEM; }
    for (int k = 0; k < n; k++) {
        for (int p = Up[k]; p < Up[k + 1]; p++) { int r = Ui[p]; e[r] = 0.0; s[r] = 0.0; cnt[r] = 0; }
        for (int p = Lp[k]; p < Lp[k + 1]; p++) { int r = Li[p]; e[r] = 0.0; s[r] = 0.0; cnt[r] = 0; }
        int pd = Up[k + 1] - 1;
        for (int p = Up[k]; p < pd; p++) {
            int j = Ui[p];
            double u = fabs(Ux[p]);
            eU[p] = e[j] + or_gamma(g * (cnt[j] + 1)) * (u + 2.0 * s[j]);
            for (int q = Lp[j]; q < Lp[j + 1]; q++) {
                int r = Li[q];
                double l = fabs(Lx[q]);
                e[r] += l * eU[p] + eL[q] * u;
                s[r] += l * u;
                cnt[r]++;
            }
        }
        double d = fabs(Ux[pd]);
        eU[pd] = e[k] + or_gamma(g * (cnt[k] + 1)) * (d + 2.0 * s[k]);
        for (int q = Lp[k]; q < Lp[k + 1]; q++) {
            int r = Li[q];
            double l = fabs(Lx[q]);
            double ex = e[r] + or_gamma(g * (cnt[r] + 1)) * (l * d + 2.0 * s[r]);
            eL[q] = (ex + l * eU[pd]) / d + 1.1102230246251565e-16 * l;
        }
    }
    free(e); free(s); free(cnt);
    return OR_OK;
}
