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
};

int validate_csc(int n, const int32_t *colptr, const int32_t *rowind);
bool max_transversal(int n, const std::vector<int> &Ap, const std::vector<int> &Ai,
                     std::vector<int> &match_of_col);
void amd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si,
               std::vector<int> &perm);
void column_etree(int n, const std::vector<int> &Hp, const std::vector<int> &Hi,
                  std::vector<int> &parent);
int run_analysis(Analysis &an, int n, const int32_t *colptr, const int32_t *rowind,
                 int ordering, int transversal);

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

// Host left-looking LU with threshold pivoting.  Columns with keep[k] != 0
// are copied from `prev` (pattern and values) instead of being recomputed;
// the others are factored with pivoting, the preferred row of column k being
// the row in position k of init_pivrow.  Returns CKTLU_OK or an error code.
int host_gp_factor(const Analysis &an, const double *values, double eps,
                   const std::vector<int> &init_pivrow, const Factor *prev,
                   const std::vector<char> *keep, Factor &out, int &fail_col, int &nswaps);

// Restart set: unfinished columns and their elimination-tree ancestors.
void restart_closure(const std::vector<int> &parent, const std::vector<char> &unfinished,
                     std::vector<char> &in_set);

// ---------------------------------------------------------------- schedule
struct Schedule {
    int n = 0;
    std::vector<int> level, seq;              // level of each column; columns by (level, index)
    int nlevels = 0, max_width = 0;
    std::vector<int> amap;                    // user nonzero -> slot offset inside its column
    // device layout of the factor storage: column k occupies [Dp[k], Dp[k] + Dlen[k]);
    // every column starts on a kColAlign-entry boundary so that no cache line holds
    // entries of two columns
    std::vector<int> Dp, Dlen, Fi_dev;        // Fi_dev: rows at device positions, padding = INT_MAX
    int64_t nnz_dev = 0;
    // CSR of strictly-lower L and strictly-upper U (position space) for the solves
    std::vector<int> Lrp, Lrj, Lrsrc, Urp, Urj, Ursrc, udiag;
    std::vector<int> rowperm_final;           // position k <- user row
    // user-space CSR of A (for the FP64 residual of iterative refinement)
    std::vector<int> Acp, Acj, Acsrc;
    int max_col = 0;                          // longest column of F
    double macs = 0, flops = 0;
    // dense trailing block [tail0, n)
    int tail0 = 0;
};

void build_schedule(const Analysis &an, const Factor &f, const cktlu_options &opt, Schedule &s);

// ------------------------------------------------------------------ device
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Device {
    bool uploaded = false;
    int prec = CKTLU_FP64;
    int batch_cap = 0;                 // instances the value buffers hold
    // pattern / schedule
    DevBuf seq, Dp, Dlen, Fi, nU, Ap, colperm, amap;
    DevBuf Lrp, Lrj, Lrsrc, Urp, Urj, Ursrc, udiag, rowperm, colperm_sol;
    DevBuf Acp, Acj, Acsrc;
    // values and sync words
    DevBuf Fx64, Fx32;                 // factor values (FP64 always; FP32 in FP32_IR mode)
    DevBuf Aval;                       // copy of the last values (FP64) for residuals
    DevBuf ready, sready, ctrl;        // per-column flags, per-row solve flags, control words
    DevBuf scratch;                    // per-wave overflow work vectors
    DevBuf vec;                        // solve work vectors
    size_t vec_cap = 0;
    unsigned epoch = 0, sepoch = 0;
    int grid_refactor = 0, grid_solve = 0;
};

}  // namespace cktlu

// -------------------------------------------------------------- launchers
// Implemented in kernels.hip.  All return a hipError_t as int.
namespace cktlu_dev {

constexpr int kColAlign = 32;   // factor column alignment in entries (>= one 128-byte line)
constexpr int YS = 16;          // doubles per solve-vector row (one 128-byte line); nrhs <= 8

struct RefactorArgs {
    int n, batch;
    const int *seq, *Dp, *Dlen, *Fi, *nU, *Ap, *colperm, *amap;
    const double *Aval;        // batch x nnzA
    int64_t nnzA, nnzF;
    void *Fx;                  // batch x nnzF (double or float)
    int *ready;                // batch x n
    int *ctrl;                 // [0] ticket, [1..] per-instance interrupt, then first-fail
    double eps;
    unsigned epoch;
    int force_fail_col;
    void *scratch;             // per-wave work vectors of max_col entries
    int max_col;
    int fp32, check;
    int *err;                  // watchdog word: set when a wait exceeds spin_limit
    int spin_limit;
};

int launch_refactor(const RefactorArgs &a, int grid, void *stream);
int launch_reset_ctrl(int *ctrl, int nwords, int value, void *stream);
// status[i] = firstfail[i] == INT_MAX ? -1 : firstfail[i]
int launch_status_out(const int *firstfail, int *status, int batch, void *stream);

struct SolveArgs {
    int n, nrhs, batch;
    const int *Lrp, *Lrj, *Lrsrc, *Urp, *Urj, *Ursrc, *udiag;
    const void *Fx;            // factor values (double or float), batch x nnzF
    int64_t nnzF;
    int fp32;
    double *y;                 // batch x n x nrhs work (interleaved by rhs)
    int *ready;                // batch x n
    int *ctrl;                 // ticket words
    unsigned epoch;
    const int *skip;           // per-instance status (-1 = solve), may be null
    int *err;                  // watchdog word
    int spin_limit;
};

int launch_lsolve(const SolveArgs &a, int grid, void *stream);
int launch_usolve(const SolveArgs &a, int grid, void *stream);
// y[(i*n + k)*nrhs + r] = b[(i*nrhs + r)*ldb + perm[k]]  (ldb = n for batched)
int launch_gather_rhs(int n, int nrhs, int batch, const double *b, int64_t ldb, const int *perm,
                      double *y, void *stream);
// x[(i*nrhs + r)*ldx + perm[k]] (+)= z[(i*n + k)*nrhs + r]
int launch_scatter_sol(int n, int nrhs, int batch, const double *z, const int *perm, double *x,
                       int64_t ldx, int accumulate, const int *skip, void *stream);
// r = b - A x (user space, FP64), per rhs; also writes |r|_inf, |x|_inf, |b|_inf maxima
int launch_residual(int n, int nrhs, const int *Acp, const int *Acj, const int *Acsrc,
                    const double *Aval, const double *x, int64_t ldx, const double *b,
                    int64_t ldb, double *r, int64_t ldr, double *norms, void *stream);
int launch_anorm(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out,
                 void *stream);
int launch_copy_f64(const double *src, double *dst, int64_t count, void *stream);
int launch_f64_to_f32(const double *src, float *dst, int64_t count, void *stream);
int occupancy_grid(int kind, int *grid);

}  // namespace cktlu_dev
