// Internal declarations of the cktlu library (host analysis, host
// factorization with pivoting, schedule construction, device launchers).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cktlu.h"

namespace cktlu {

// ---------------------------------------------------------------- analysis
struct Analysis {
    int n = 0;
    int64_t nnz = 0;
    std::vector<int> Ap, Ai;               // copy of the user pattern (CSC)
    std::vector<int> rowperm_pre, colperm; // A_hat(i,j) = A(rowperm_pre[i], colperm[j])
    std::vector<int> rowinv_pre, colinv;
    std::vector<int> Hp, Hi, Hsrc;         // A_hat pattern (CSC, sorted) and source nonzero index
    std::vector<int> parent;               // column elimination tree of A_hat
    int etree_height = 0;
    int ordering_used = 0;                 // CKTLU_ORDER_* that produced colperm
    int64_t fill_amd = -1, fill_amf = -1, fill_nd = -1;  // nnz of the symbolic Cholesky of B + B' under each
    int64_t fill_ndc = -1;                 // ... under ND + constrained AMD
    int static_pivoting_used = 0;          // 0 structural transversal, 1 max-product matching, 2 and scaling
    std::vector<double> rscale, cscale;    // static scaling of A's rows and columns (empty: none)
};

int validate_csc(int n, const int32_t *colptr, const int32_t *rowind);
bool max_transversal(int n, const std::vector<int> &Ap, const std::vector<int> &Ai,
                     std::vector<int> &match_of_col);
// group != nullptr: constrained minimum degree, the nodes eliminated in ascending group
void amd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si,
               std::vector<int> &perm, bool amf = false, const std::vector<int> *group = nullptr);
// nested dissection with AMD on parts of at most `leaf` nodes; with groups, the leaves are not
// ordered and every node receives the number of its part in the dissection's order instead
constexpr int kNdLeaf = 4096;
void nd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si, std::vector<int> &perm,
              int leaf, std::vector<int> *groups = nullptr);
// nested dissection to parts of at most `leaf` nodes, then constrained AMD over the parts
void nd_camd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si, std::vector<int> &perm,
                   int leaf);
// nnz (diagonal included) of the Cholesky factor of the symmetric pattern (Sp, Si)
// eliminated in the order perm: elimination tree, then one row subtree per row
int64_t symbolic_cholesky_nnz(int n, const std::vector<int> &Sp, const std::vector<int> &Si,
                              const std::vector<int> &perm);
void column_etree(int n, const std::vector<int> &Hp, const std::vector<int> &Hi,
                  std::vector<int> &parent);
// values (may be null) and static_pivoting (0, 1 matching, 2 matching and scaling) select the
// value-based static pivoting of Section III-A instead of the structural transversal
bool max_product_matching(int n, const std::vector<int> &Ap, const std::vector<int> &Ai, const double *Ax,
                          std::vector<int> &match_of_col, std::vector<double> &lnr, std::vector<double> &lnc);
int run_analysis(Analysis &an, int n, const int32_t *colptr, const int32_t *rowind,
                 int ordering, int transversal, const double *values = nullptr, int static_pivoting = 0);

// ------------------------------------------------------------------ factor
// Factors in position space.  Column k of the combined storage F holds the
// U entries (rows < k ascending, then the diagonal k) followed by the L
// entries (rows > k ascending), so Fi is ascending inside every column.
struct Factor {
    int n = 0;
    std::vector<int> pivrow, posof;   // position -> A_hat row, and inverse
    std::vector<int64_t> Fp;          // [n+1]
    std::vector<int> Fi, nU;          // rows; |U(:,k)| incl. diagonal
    std::vector<double> Fx;           // FP64 values
    int64_t nnz_l() const { return (int64_t)Fi.size() - nnz_u(); }
    int64_t nnz_u() const { int64_t s = 0; for (int v : nU) s += v; return s; }
};

// The trailing columns [T, n) factored elsewhere (the device's pivoted dense LU):
// the position exchanged with each position at its step (swap[c] >= c, local to the
// block) and the factors in final row positions (D x D, column-major, unit L below
// the diagonal, U on and above).  Their rows < T (U entries) come from `prev`.
struct DenseSource {
    int T = 0, D = 0;
    const int *swap = nullptr;
    const double *S = nullptr;
};

// Host left-looking LU with threshold pivoting.  Columns with keep[k] != 0
// are copied from `prev` (pattern and values) instead of being recomputed;
// the others are factored with pivoting, the preferred row of column k being
// the row in position k of init_pivrow.  With dsrc, the columns >= dsrc->T that
// are not kept take their pivots and values from dsrc (only their pattern is
// computed here).  Returns CKTLU_OK or an error code.
int host_gp_factor(const Analysis &an, const double *values, double eps,
                   const std::vector<int> &init_pivrow, const Factor *prev,
                   const std::vector<char> *keep, Factor &out, int &fail_col, int &nswaps,
                   const DenseSource *dsrc = nullptr);

// Restart set: unfinished columns and their elimination-tree ancestors.
void restart_closure(const std::vector<int> &parent, const std::vector<char> &unfinished,
                     std::vector<char> &in_set);

// ---------------------------------------------------------------- schedule
struct Schedule {
    int n = 0;
    // elimination graph (column k depends on j when U(j,k) != 0): level of each column
    std::vector<int> level;
    int nlevels = 0, max_width = 0;
    // right-looking schedule: columns by (rlevel, index) and the rlevel boundaries
    std::vector<int> seq, lvl_ptr;
    int n_rlevels = 0;
    // right-looking update tasks: level l owns tasks [task_ptr[l], task_ptr[l+1]); task t
    // updates target column task_tgt[t] with the sources src_col[src_ptr[t] .. src_ptr[t+1])
    // (columns of level l, ascending); src_slot is the offset of the source's row in the
    // target column (where the multiplier U(j,k) lives)
    std::vector<int> task_ptr, task_tgt, src_ptr, src_col, src_slot;
    std::vector<int> colrec, task8, item4;    // the same schedule packed for the device
    // slot map: for task t, the slots in its target column of the entries of its items
    // (first item, then the extra ones, each its L range in order) from smap[tmoff[t]]
    std::vector<int> smap;
    std::vector<int64_t> tmoff;
    std::vector<int> amap;                    // user nonzero -> slot offset inside its column
    // device layout of the factor storage: column k occupies [Dp[k], Dp[k] + Dlen[k]);
    // every column starts on a kColAlign-entry boundary
    std::vector<int> Dp, Dlen, Fi_dev;        // Fi_dev: rows at device positions, padding = INT_MAX
    int64_t nnz_dev = 0;
    // CSR of strictly-lower L and strictly-upper U (position space) for the solves
    std::vector<int> Lrp, Lrj, Lrsrc, Urp, Urj, Ursrc, udiag;
    // solve dependency graphs: rows by level (L: ascending dependencies, U: descending)
    std::vector<int> lseq, lsptr, useq, usptr;
    std::vector<int> lseg, useg;              // launch segments {first level, end level, kind}
    std::vector<int> rowperm_final;           // position k <- user row
    // user-space CSR of A (for the FP64 residual of iterative refinement)
    std::vector<int> Acp, Acj, Acsrc;
    int max_col = 0;                          // longest column of F
    double macs = 0, flops = 0;
    double macs_sweep = 0, lnz_front = 0;     // MACs of the update tasks; L entries of sparse columns
    double macs_schur = 0;                    // MACs of the dense block's Schur update (S -= L21 U12)
    double macs_dense = 0;                    // MACs of the dense block's own LU (dense sources and targets)
    double entries_sweep = 0;                 // factor entries the sweep finalises (sparse columns, bridge rows)
    double entries_dense = 0;                 // factor entries of the dense columns in rows >= tail0
    std::vector<int> tail_nb;                 // per dense column: its U entries in rows < T (the bridge)
    // Schur update parts {dense column, first and end bridge source, scratch column or -1}
    // and the add pass {dense column, first scratch column, count, 0}
    std::vector<int> schur_parts, schur_add;
    int schur_nscr = 0;
    std::vector<int> l21;                     // per sparse column: device range of its L rows >= T
    int tail0 = 0;                            // first column of the densely factored tail (n = none)
    std::vector<int> tail_rend;               // rows i >= tail0: L entries of columns < tail0 end here
    std::vector<int> lrec, urec, Lrjs, Urjs;  // the solve levels packed for the device
    // ---- supernodal sweep (options.sweep_supernodes >= 0).  A supernode is a run of sparse
    // columns [s0, s0 + w) (w <= 64) whose diagonal block is dense and whose L columns share the
    // rows R below it (L(:,j) = {j+1} u L(:,j+1)).  Level = longest path over the supernodes
    // whose columns update its columns (U entries) or whose rows feed its rows (L entries).
    // Level l runs two launches: the panels of its supernodes (dense LU of the diagonal block,
    // L21 = A21 U11^-1, the pivot test), then update tasks: a task owns one target column k and
    // applies every supernode S of level l with U(S, k) != 0 in ascending order: U(S, k) =
    // L11^-1 x_k(S) on the suffix of S's rows present in k, then x_k(R) -= L21 U(S, k).
    int sn_count = 0, sn_levels = 0;
    std::vector<int> sn_rec;                  // int4 per supernode {s0, w, m = |R|, rows of R below tail0}
    // Schur update by supernodes (with sn_count > 0, schur_parts index these items instead of
    // bridge rows): {supernode, first column in it, columns, position of the first row in k}
    std::vector<int> schur_sn_items;
    std::vector<int> sn_cb;                   // per sparse column j: device offset of row s0(j) in column j
    std::vector<int> sn_lvl;                  // [sn_levels+1] supernodes of level l: sn_seq[sn_lvl[l] ..]
    std::vector<int> sn_seq;                  // supernode ids by level: singletons, small panels, panels
    std::vector<int> sn_lvl_single;           // [sn_levels] singletons of level l: sn_seq[sn_lvl[l] ..
                                              // sn_lvl_single[l])
    std::vector<int> sn_lvl_small;            // [sn_levels] then panels at most kSnSmallW wide (a
                                              // wavefront each) up to sn_lvl_small[l], wider ones after
    std::vector<int> sn_punit;                // wide panels as units: int4 {position in sn_seq, slice p,
                                              // slices P, first scratch block (-1 when P = 1)}
    std::vector<int> sn_pulvl;                // [sn_levels+1] units of level l
    std::vector<int> sn_sunit, sn_sulvl;      // the same for the small panels
    std::vector<int> sn_pu2, sn_su2;          // per unit: int4 {s0, w, m, 0} of its supernode
    int sn_pnscr = 0;                         // scratch blocks a launch uses at most
    std::vector<int> sn_task_lvl;             // [sn_levels+1] tasks of level l
    std::vector<int> sn_task_heavy;           // [sn_levels] its heavy tasks (a workgroup each) end here
    std::vector<int> sn_task_tiny;            // [sn_levels] its tiny tasks (sixteen lanes each) start here
    // the heavy tasks of level l as groups sn_grp [sn_grp_lvl[l], sn_grp_lvl[l+1]): int4 {first task,
    // tasks, first source record, end source record}; source records sn_gsrc int4 {S, first
    // entry, entries, rows of R updated}, ascending in S; entries sn_gent int2 {task index in the
    // group, item}
    std::vector<int> sn_grp, sn_gsrc, sn_gent, sn_grp_lvl;
    std::vector<int> sn_task;                 // int4 per task {k, Dp[k], first item, end item}
    std::vector<int> sn_item;                 // int4 per item {supernode, slot of its first row in k, rows
                                              // of S present in k (the suffix), rows of R updated}
    std::vector<int64_t> sn_moff;             // per item: its slots of R's rows in column k in sn_map
    std::vector<int> sn_item2;                // per item: int4 {sn_cb index of the suffix's first column
                                              // (the source's first column + its rows not in k), the
                                              // source's width, sn_moff low and high 32 bits}
    std::vector<int> sn_map;
    int64_t sn_items = 0;
    double sn_macs = 0;                       // multiply-adds of the supernodal updates and panels
    // supernodal solves of the rows [0, T): a supernode's rows first pull their entries outside
    // its diagonal block (L: columns < s0; U: columns >= s0 + w), then its dense triangle is
    // solved.  Level = longest path over the supernodes those entries reach.  Per level of the
    // L (U) solve: its supernodes in snl_seq (snu_seq) [snl_lvl[l], snl_lvl[l+1]), singletons
    // first: singletons with a short row up to snl_tiny[l] (sixteen lanes each), then up to
    // snl_single[l] the others of at most kSnSmallW rows and a short pull (a wavefront each).
    // The workgroup units of level l: snl_unit [snl_ulvl[l], snl_ulvl[l+1]), int4 {position in
    // snl_seq, unit p, units P, first scratch block of the supernode (-1 when P = 1)}; a level
    // uses at most snl_nscr scratch blocks.  A workgroup supernode's pull is a list of runs
    // (snl_runs, int4 {column j, position of the first entry, first row c_a, rows}: rows
    // s0 + c_a ... of the supernode present in column j, at consecutive positions); unit u pulls
    // the runs [snl_urange[4u], snl_urange[4u+1]) of supernode [snl_urange[4u+2], + snl_urange[4u+3]).
    int snl_levels = 0, snu_levels = 0;
    std::vector<int> snl_lvl, snl_tiny, snl_single, snl_seq, snu_lvl, snu_tiny, snu_single, snu_seq;
    // first position of level l that a launch takes (L: singletons with no L entries come
    // first and need nothing; U: snu_lvl[l])
    std::vector<int> snl_first, snu_first;
    std::vector<int> snl_unit, snl_ulvl, snu_unit, snu_ulvl;
    std::vector<int> snl_urange, snl_runs, snu_urange, snu_runs;
    // the device copies of the sequences: int2 {first column, width} per position
    std::vector<int> snl_sw, snu_sw;
    int snl_nscr = 0, snu_nscr = 0;
};

// map_cap: most slot-map entries to build (-1: what a quarter of the device's free memory
// holds; none without a device)
void build_schedule(const Analysis &an, const Factor &f, const cktlu_options &opt, Schedule &s,
                    int64_t map_cap = -1);

// ------------------------------------------------------------------ device
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Device {
    bool uploaded = false;
    int batch_cap = 0;                 // instances the value buffers hold
    // pattern / schedule
    DevBuf seq, Dp, Dlen, Fi, nU, Ap, colperm, amap;
    DevBuf colrec, task8, item4, smap, tmoff, tail_nb, l21, schur_parts, schur_add, schur_scr;
    DevBuf lrec, urec, Lrjs, Urjs, lsptr, usptr, rowperm, colperm_sol;   // colperm_sol: user index -> position
    DevBuf Acp, Acj, Acsrc;
    DevBuf sn_rec, sn_cb, sn_seq, sn_task, sn_item, sn_moff, sn_map;   // supernodal sweep
    DevBuf sn_item2;
    DevBuf snl_seq, snu_seq, Lrp, Urp;                                 // supernodal solves ({s0, w} per position)
    DevBuf snl_unit, snu_unit, sn_part, sn_cnt;                        // their split units
    DevBuf snl_urange, snl_runs, snu_urange, snu_runs;                 // the units' runs
    DevBuf sn_punit, sn_sunit, sn_pu2, sn_su2;                         // split panels
    DevBuf sn_grp, sn_gsrc, sn_gent;                                   // grouped heavy tasks
    DevBuf ascale, gscale, sscale;     // static scaling: per nonzero of A, per solve row, per solve column
    DevBuf schur_sn_items;             // supernodal Schur update items
    // values and status words
    DevBuf Fx64, Fx32;                 // factor values (FP64 always; FP32 in FP32_IR mode)
    DevBuf Aval;                       // copy of the last values (FP64) for residuals
    DevBuf done, ctrl;                 // per-column completion epochs, status words
    DevBuf vec;                        // solve work vectors
    DevBuf S;                          // dense trailing block, batch x D x D (8-byte slots)
    DevBuf Dg;                         // batch x 64 x 64 (8-byte slots): a panel's diagonal block
    DevBuf Dinv;                       // batch x nblk x 2 x 64 x 64 FP64: diagonal blocks' inverses
    size_t vec_cap = 0;
    unsigned epoch = 0;
    int S_prec = -1;                   // what S holds: -1 stale, 0 FP64 factors, 1 FP32 factors
};

}  // namespace cktlu

// -------------------------------------------------------------- launchers
// Implemented in kernels.hip.  All return a hipError_t as int.
namespace cktlu_dev {

constexpr int kColAlign = 32;   // factor column alignment in entries (>= one 128-byte line)
constexpr int YS = 16;          // doubles per solve-vector row at most (rows hold solve_slots(nrhs) doubles)
constexpr int kSolveRowWG = 256; // threads of the workgroup that solves one long row
constexpr int kSolveLongRow = 64; // levels holding a longer row get a workgroup per row (64, 128 and
                                  // 256 measured: 64 best on the RC mesh and the power grid)
// right-hand-side slots the solve kernels carry per row: nrhs rounded up to 1, 2, 4 or 8
inline int solve_slots(int nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8; }

struct RefactorArgs {
    int n, batch;
    const int *seq, *Dp, *Dlen, *Fi, *nU, *Ap, *colperm, *amap;
    const int *colrec;         // {Dp, nU, Dlen, column} per position of seq
    const int *task8, *item4;  // right-looking update tasks (two int4s each) and their extra items
    const int *smap;           // slot map (target slot of every source entry), or nullptr: the tasks
    const int64_t *tmoff;      // search the target rows; its offset per task
    const double *Aval;        // batch x nnzA
    int64_t nnzA, nnzF;
    void *Fx;                  // batch x nnzF (double or float)
    int T, D;                  // columns [T, n) form the dense block: their rows >= T live in S
    void *S;                   // batch x D x D (factor type), column-major
    int *done;                 // batch x n: epoch of the last successful computation of each column
    int *ctrl;                 // [1, 1+batch) interrupt words (1 + the level whose check failed, any
                               // nonzero value after the dense block's test), [1+batch, 1+2 batch) first
                               // failing column
    double eps;
    unsigned epoch;
    int force_fail_col;
    int fp32, check;
    // supernodal sweep (see Schedule): supernode records, per-column offset of the supernode's
    // first row, supernodes by level, update tasks, their items and the rows' slots
    const int *sn_rec, *sn_cb, *sn_seq, *sn_task, *sn_item, *sn_map;
    const int64_t *sn_moff;
    const int *sn_item2;       // per item: {suffix's first sn_cb index, source width, map offset lo, hi}
    // wide panels split by rows of R: units int4 {position in sn_seq, slice, slices, first
    // scratch block}; column maxima of the slices (64 doubles per block and instance) and an
    // arrival counter per sn_seq position and instance (zero on entry and on exit)
    const int *sn_punit, *sn_sunit;
    const int *sn_pu2, *sn_su2;    // per unit: {s0, w, m, 0} (the supernode record, read with the unit)
    const int *sn_grp, *sn_gsrc, *sn_gent;   // grouped heavy update tasks (see Schedule)
    double *sn_pmax;
    int *sn_pcnt;
    const double *ascale;      // static scaling per nonzero of A (row scale x column scale), or null
};

// Zero every factor column and scatter the matrix values into it.
int launch_refactor_init(const RefactorArgs &a, void *stream);
// FP64, one instance: S = the dense columns' matrix values in rows >= T (their rows < T untouched).
int launch_dense_reinit(const RefactorArgs &a, void *stream);
// One right-looking level `lev`: pivot check of columns seq[cbeg, cend), normalisation of
// the previous level seq[pbeg, pend) (L = x / pivot), and update tasks [tbeg, tend).
int launch_refactor_level(const RefactorArgs &a, int cbeg, int cend, int pbeg, int pend, int tbeg,
                          int tend, int lev, void *stream);
// Supernodal sweep, level `lev` (dense.hip): the singleton supernodes sn_seq[sbeg, s1) (pivot test
// and L = x / pivot, sixteen lanes each), the small panels as units sn_sunit[sub, sue) (a
// wavefront each) and the wider panels as units sn_punit[ubeg, uend) (a workgroup each): dense
// LU of the diagonal block, L21 = A21 U11^-1, pivot test; then the level's update tasks: the
// heavy ones as groups
// sn_grp [gbeg, gend) (a workgroup each), [theavy, ttiny) a wavefront each, [ttiny, tend)
// sixteen lanes each.
int launch_sn_panels(const RefactorArgs &a, int lev, int sbeg, int s1, int sub, int sue, int ubeg, int uend,
                     void *stream);
int launch_sn_updates(const RefactorArgs &a, int lev, int gbeg, int gend, int theavy, int ttiny, int tend,
                      void *stream);
int launch_reset_ctrl(int *ctrl, int nwords, int value, void *stream);
// status[i] = firstfail[i] == INT_MAX ? -1 : firstfail[i]
int launch_status_out(const int *firstfail, int *status, int batch, void *stream);

struct SolveArgs {
    int n, nrhs, batch;
    const int *lrec, *urec;    // per solve position: {row, first entry, end, position of U(i,i)}
    const int *Lrjs, *Urjs;    // per entry: {column, position of the value}
    const void *Fx;            // factor values (double or float), batch x nnzF
    int64_t nnzF;
    int fp32;
    double *y;                 // batch x n rows of solve_slots(nrhs) doubles, rhs r in slot r
    const int *skip;           // per-instance status (-1 = solve), may be null
    // supernodal solves: supernode records and first-row offsets (as RefactorArgs), and the row
    // pointers of the strictly lower L and strictly upper U (entries in Lrjs / Urjs)
    const int *sn_rec, *sn_cb, *Lrp, *Urp;
    double *sn_part;           // partial sums of split supernodes: 512 doubles per block and instance
};

// One level of the supernodal L (U) solve: sixteen lanes per singleton seq[sbeg, stiny), a
// wavefront per supernode seq[stiny, smid) and a workgroup per unit units[ubeg, uend) (int4
// {position in seq, slice, slices, first scratch block}); cnt: an arrival counter per seq
// position and instance, zero on entry and on exit.
int launch_sn_lsolve(const SolveArgs &a, const int *sw, const int *units, const int *urange, const int *runs, int sbeg,
                     int stiny, int smid, int ubeg, int uend, int *cnt, void *stream);
int launch_sn_usolve(const SolveArgs &a, const int *sw, const int *units, const int *urange, const int *runs, int sbeg,
                     int stiny, int smid, int ubeg, int uend, int *cnt, void *stream);

// Solve positions [lbeg, lend) of lrec / urec (one level of the solve graph).
int launch_lsolve_level(const SolveArgs &a, int lbeg, int lend, void *stream);
int launch_usolve_level(const SolveArgs &a, int lbeg, int lend, void *stream);
// Solve positions [lbeg, lend) with one workgroup of kSolveRowWG threads per (row, instance).
int launch_lsolve_level_wg(const SolveArgs &a, int lbeg, int lend, void *stream);
int launch_usolve_level_wg(const SolveArgs &a, int lbeg, int lend, void *stream);
// Levels [l0, l1) of the L / U solve graph in one launch: one workgroup per instance,
// a barrier between levels; lvptr = level boundaries in solve positions (device).
int launch_lsolve_chain(const SolveArgs &a, const int *lvptr, int l0, int l1, void *stream);
int launch_usolve_chain(const SolveArgs &a, const int *lvptr, int l0, int l1, void *stream);
// y[((i*n + k)*ns + r] = b[(i*nrhs + r)*ldb + perm[k]] for r < nrhs, 0 for r < ns = solve_slots(nrhs)
int launch_gather_rhs(int n, int nrhs, int batch, const double *b, int64_t ldb, const int *perm,
                      double *y, void *stream, const double *scale = nullptr);
// x[(i*nrhs + r)*ldx + j] (+)= y[(i*n + inv[j])*solve_slots(nrhs) + r]; inv: user index -> solve position
int launch_scatter_sol(int n, int nrhs, int batch, const double *z, const int *inv, double *x,
                       int64_t ldx, int accumulate, const int *skip, void *stream, const double *scale = nullptr);
// r = b - A x (user space, FP64), per rhs; also writes |r|_inf, |x|_inf, |b|_inf maxima.  Nothing
// when skip is given and *skip != -1.
int launch_residual(int n, int nrhs, const int *Acp, const int *Acj, const int *Acsrc,
                    const double *Aval, const double *x, int64_t ldx, const double *b,
                    int64_t ldb, double *r, int64_t ldr, double *norms, void *stream, const int *skip = nullptr);
int launch_anorm(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out,
                 void *stream);
int launch_copy_f64(const double *src, double *dst, int64_t count, void *stream);
int launch_copy_i32(const int *src, int *dst, int64_t count, void *stream);
int launch_fill_f64(double *dst, int64_t count, double value, void *stream);
// batched refinement: per-instance residuals and their norms, |A|_inf per instance,
// and the convergence test that takes converged instances out of skip
int launch_residual_batched(int n, int nrhs, int batch, int64_t nnzA, const int *Acp, const int *Acj,
                            const int *Acsrc, const double *Aval, const double *x, const double *b, double *r,
                            double *norms, const int *skip, void *stream);
int launch_anorm_batched(int n, int batch, int64_t nnzA, const int *Acp, const int *Acsrc, const double *Aval,
                         double *out, void *stream);
int launch_ir_check(int batch, int nrhs, const double *norms, const double *anorm, double tol, int *skip,
                    double *eta, void *stream);
int launch_f64_to_f32(const double *src, float *dst, int64_t count, void *stream);
int launch_fill_i32(int *dst, int64_t count, int value, void *stream);
// Work rows of the allocation-free solve: a file-scope device array of kNoAllocRows rows of YS
// doubles (64 MiB), one per GPU for the life of the process.  *out receives its device address on
// the current device (looked up once per device).  Returns a hipError_t as int.
constexpr int kNoAllocRows = 1 << 19;
int noalloc_scratch(double **out);

// Dense trailing block (dense.hip): columns and rows [T, n) of the factors,
// D = n - T, held per instance as a column-major D x D matrix S.
constexpr int kDenseBlock = 64;  // panel width of the blocked LU and of the block solves
constexpr int kSnSmallW = 16;    // supernodes up to this wide are factored by one wavefront
constexpr int kGroupTargets = 4; // heavy update tasks with shared sources grouped this many at a time
constexpr int kTinyRows = 16;    // update tasks whose items have at most this many suffix rows and
constexpr int kTinyRowsR = 64;   // at most this many rows of R: 16 lanes each
struct DenseArgs {
    int n, T, D, batch;
    const int *Dp, *Dlen, *Fi;
    void *Fx;                  // factor values (double or float), batch x nnzF
    int64_t nnzF;
    void *S;                   // batch x D x D values of the factor type
    void *Dg;                  // batch x NB x NB: factored diagonal block of the current panel
    double *Dinv;              // batch x nblk x 2 x NB x NB: inverses of the diagonal blocks' L and U
    int *ctrl, *done;          // status words and completion epochs (as RefactorArgs)
    double eps;
    unsigned epoch;
    int force_fail_col;
    int fp32, check;
    int W;                     // columns factored between two updates of the whole trailing block
    void *scr;                 // batch x nscr x D Schur scratch columns (factor type, 8-byte slots)
    int nscr;
};
// S <- rows >= T of the tail columns of Fx (zeros elsewhere)
int launch_dense_gather(const DenseArgs &a, void *stream);
// S -= L21 U12: the sparse columns' contributions to the dense block, after the sweep, in
// nparts parts (int4 {dense column, first and end bridge source, scratch column or -1}),
// then the scratch columns added into S (nadd records {column, first scratch, count, 0})
int launch_schur(const DenseArgs &a, const int *parts, int nparts, const int *add, int nadd, const int *l21,
                 void *stream);
// The same update by supernodes: parts index the items sn_items ({supernode, first column,
// columns, position of the first row in the dense column}); sn_rec and sn_cb as in RefactorArgs.
int launch_schur_sn(const DenseArgs &a, const int *parts, int nparts, const int *add, int nadd, const int *sn_items,
                    const int *sn_rec, const int *sn_cb, void *stream);
// Look-ahead resources of the dense LU: a second stream (default priority) on which the
// panels of group g+1 run while the trailing update of group g runs on the main stream,
// and events that order the two (2 per group boundary).  side == nullptr: one stream.
struct DenseStreams {
    void *side;
    void *const *ev;
    int nev;
};
// (gather if asked), blocked LU with the pivot test, scatter back into Fx
int launch_dense_refactor(const DenseArgs &a, bool gather, const DenseStreams *la, void *stream);
// events the look-ahead needs for this dense block (0: it runs on one stream)
int dense_lookahead_events(const DenseArgs &a);
// FP64, one instance: LU of S with the threshold pivot rule (Section II-A): at column c
// the row in position c stays unless its value is zero, not finite or below eps times
// the largest other candidate; then the largest candidate (smallest position on ties)
// is exchanged into position c.  Rows are exchanged across the whole block, so on
// return S holds unit L below the diagonal and U on and above it in final row
// positions; swap[c] (device, D ints) is the position exchanged with c at step c.
// info (device int, zeroed here) receives 1 + the first column with no usable pivot.
int launch_dense_pivoted_lu(const DenseArgs &a, int *swap, int *info, void *stream);
// Dinv <- inverses of the unit-lower and upper triangles of S's 64 x 64 diagonal blocks
int launch_dense_inverses(const DenseArgs &a, void *stream);
// y rows [T, n): lower (unit) or upper triangular solve with the block in S and Dinv
int launch_dense_solve(const DenseArgs &a, double *y, int nrhs, const int *skip, bool upper, void *stream);

}  // namespace cktlu_dev
