// Device kernels of the cktlu hot path (gfx950).
//
// Refactorization (fast factorization with pivot check, Section IV-B) runs as
// right-looking sweeps over dependency levels, one launch per level:
//   refactor_init_kernel   zeroes every factor column and scatters the matrix
//                          values into it (one wavefront per column);
//   refactor_level_kernel  for level l: (a) tests the pivot of every column of
//                          level l against eps times the largest entry of its L
//                          part (its values are final: every update came from an
//                          earlier level); (b) divides the L part of every column
//                          of level l-1 by its pivot; (c) runs the update tasks of
//                          level l: a task owns one target column k and applies
//                          x_k -= L(:,j) * U(j,k) for every source j of level l
//                          with U(j,k) != 0, in ascending j, so no two wavefronts
//                          write the same column and results are bit-reproducible.
// This is the paper's cluster mode (Algorithm 3) with the left-looking column
// update of the paper turned around: a column's updates are spread over the
// levels of its sources, so the critical path is the number of levels, not the
// length of a column's update list.  A failed test records the column (atomic
// minimum) and raises the instance's interrupt word; later levels of that
// instance return at once.
//
// Solves (Section II-C, Algorithm 2): trisolve_level_kernel, row ("pull") form,
// one launch per level of the solve dependency graph, one wavefront per row.
//
// All communication between wavefronts happens at kernel boundaries, where the
// runtime makes device memory coherent across the MI355X's eight XCDs.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"

namespace cktlu_dev {

constexpr int WAVE = 64;
constexpr int WG = 256;
constexpr int WAVES = WG / WAVE;
constexpr int kStageRows = 1024;   // target-column rows staged in LDS per wavefront

// Orders this wavefront's global-memory accesses across its lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------------ refactorize
// one wavefront per (column, instance).  Columns of the dense block keep their
// rows >= T in S (column k at S + (k - T) D), so those rows are zeroed there.
template <typename T>
__global__ __launch_bounds__(WG) void refactor_init_kernel(RefactorArgs a) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t w = (int64_t)blockIdx.x * WAVES + wv;
    if (w >= (int64_t)a.n * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int k = (int)(w / a.batch);
    T *x = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[k];
    const double *Av = a.Aval + (size_t)inst * a.nnzA;
    const int len = a.Dlen[k];
    const int c = a.colperm[k];
    if (k < a.T) {
        for (int i = lane; i < len; i += WAVE) x[i] = T(0);
        wave_sync();
        for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) x[a.amap[p]] = (T)Av[p];
        return;
    }
    T *Sk = reinterpret_cast<T *>(a.S) + (size_t)inst * a.D * a.D + (size_t)(k - a.T) * a.D;
    const int *rows = a.Fi + a.Dp[k];
    for (int i = lane; i < len; i += WAVE) x[i] = T(0);
    for (int i = lane; i < a.D; i += WAVE) Sk[i] = T(0);
    wave_sync();
    for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) {
        const int slot = a.amap[p];
        const int r = rows[slot];
        if (r >= a.T) Sk[r - a.T] = (T)Av[p];
        else x[slot] = (T)Av[p];
    }
}

// one wavefront per (task, instance); tasks: [checks | normalisations | updates]
template <typename T, bool CHECK>
__global__ __launch_bounds__(WG) void refactor_level_kernel(RefactorArgs a, int cbeg, int cend, int pbeg,
                                                             int pend, int tbeg, int tend) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t w = (int64_t)blockIdx.x * WAVES + wv;
    const int nchk = cend - cbeg, nnorm = pend - pbeg, nupd = tend - tbeg;
    if (w >= (int64_t)(nchk + nnorm + nupd) * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int idx = (int)(w / a.batch);
    int *interrupted = a.ctrl + 1;
    int *firstfail = a.ctrl + 1 + a.batch;
    if (CHECK && interrupted[inst]) return;          // an earlier level failed its check
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    if (idx < nchk) {
        // (a) pivot check of a column of this level
        if (!CHECK) return;
        const int j = a.seq[cbeg + idx];
        const T *x = Fx + a.Dp[j];
        const int nu = a.nU[j], len = a.Dlen[j];
        double m = 0.0;
        int bad = 0;
        for (int i = nu + lane; i < len; i += WAVE) {
            const double v = (double)x[i];
            if (!isfinite(v)) bad = 1;
            m = fmax(m, fabs(v));
        }
        m = wave_max(m);
        bad = __any(bad);
        const double d = (double)x[nu - 1];
        if (bad || !isfinite(d) || d == 0.0 || fabs(d) < a.eps * m || j == a.force_fail_col) {
            if (lane == 0) {
                atomicMin(&firstfail[inst], j);
                atomicExch(&interrupted[inst], 1);
            }
        }
        return;
    }
    if (idx < nchk + nnorm) {
        // (b) L(:,j) = x / pivot for a column of the previous level
        const int j = a.seq[pbeg + idx - nchk];
        T *x = Fx + a.Dp[j];
        const int nu = a.nU[j], len = a.Dlen[j];
        const T d = x[nu - 1];
        for (int i = nu + lane; i < len; i += WAVE) x[i] = x[i] / d;
        if (lane == 0) a.done[(size_t)inst * a.n + j] = (int)a.epoch;
        return;
    }
    // (c) update task: target column k, sources j of this level in ascending order.
    // Rows of the target are located by binary search in the searched part of column k,
    // staged in LDS when it fits; rows >= T of a dense-block target are addressed in S.
    const int4 tr = reinterpret_cast<const int4 *>(a.task4)[tbeg + idx - nchk - nnorm];
    const int iend = reinterpret_cast<const int4 *>(a.task4)[tbeg + idx - nchk - nnorm + 1].w;
    const int k = tr.x, bk = tr.y, slen = tr.z;
    T *xk = Fx + bk;
    const int *rowsk = a.Fi + bk;
    T *Sk = k >= a.T ? reinterpret_cast<T *>(a.S) + (size_t)inst * a.D * a.D + (size_t)(k - a.T) * a.D : nullptr;
    __shared__ int srows[WAVES][kStageRows];
    int *lrows = srows[wv];
    const bool staged = slen <= kStageRows;
    if (staged) {
        for (int i = lane; i < slen; i += WAVE) lrows[i] = rowsk[i];
    }
    const int4 *items = reinterpret_cast<const int4 *>(a.item4);
    for (int s0 = tr.w; s0 < iend; s0 += WAVE) {
        // lane u holds item s0 + u: its record, the pivot of its source and its multiplier
        int4 it = make_int4(0, 0, 0, 0);
        T inv = T(0), mult = T(0);
        if (s0 + lane < iend) {
            it = items[s0 + lane];
            inv = T(1) / Fx[it.x];                  // the pivot of j (not yet divided into L(:,j))
            mult = xk[it.w];                        // U(j,k): final, no source of this level updates it
        }
        wave_sync();                                // staged rows and earlier updates visible
        const int ns = min(WAVE, iend - s0);
        for (int u = 0; u < ns; ++u) {
            const int lb = __shfl(it.y, u), le = __shfl(it.z, u), lo0 = __shfl(it.w, u) + 1;
            const T iv = __shfl(inv, u), m = __shfl(mult, u);
            for (int q = lb + lane; q < le; q += WAVE) {
                const int r = a.Fi[q];
                const T l = Fx[q] * iv;
                if (Sk && r >= a.T) {
                    Sk[r - a.T] -= l * m;
                    continue;
                }
                int lo = lo0, hi = slen;            // rows of L(:,j) lie below row j in column k
                if (staged) {
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (lrows[mid] < r) lo = mid + 1; else hi = mid;
                    }
                } else {
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (rowsk[mid] < r) lo = mid + 1; else hi = mid;
                    }
                }
                if (lo < slen) xk[lo] -= l * m;     // always found: struct(L(:,j)) is inside struct(col k)
            }
            wave_sync();
        }
    }
}

__global__ void reset_ctrl_kernel(int *ctrl, int nwords, int value, int batch) {
    // ctrl[0] unused; ctrl[1..batch] = 0 (interrupt); the rest = value (first failing column)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        ctrl[i] = (i == 0 || i <= batch) ? 0 : value;
}

int launch_reset_ctrl(int *ctrl, int nwords, int value, void *stream) {
    const int batch = (nwords - 1) / 2;
    hipLaunchKernelGGL(reset_ctrl_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, ctrl, nwords,
                       value, batch);
    return (int)hipGetLastError();
}

__global__ void status_out_kernel(const int *firstfail, int *status, int batch) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += gridDim.x * blockDim.x)
        status[i] = firstfail[i] == INT_MAX ? -1 : firstfail[i];
}

int launch_status_out(const int *firstfail, int *status, int batch, void *stream) {
    hipLaunchKernelGGL(status_out_kernel, dim3((batch + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       firstfail, status, batch);
    return (int)hipGetLastError();
}

int launch_refactor_init(const RefactorArgs &a, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (int64_t)a.n * a.batch;
    const dim3 grid((unsigned)((waves + WAVES - 1) / WAVES));
    if (waves == 0) return 0;
    if (a.fp32) hipLaunchKernelGGL((refactor_init_kernel<float>), grid, dim3(WG), 0, st, a);
    else hipLaunchKernelGGL((refactor_init_kernel<double>), grid, dim3(WG), 0, st, a);
    return (int)hipGetLastError();
}

int launch_refactor_level(const RefactorArgs &a, int cbeg, int cend, int pbeg, int pend, int tbeg, int tend,
                          void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (int64_t)((cend - cbeg) + (pend - pbeg) + (tend - tbeg)) * a.batch;
    if (waves == 0) return 0;
    const dim3 grid((unsigned)((waves + WAVES - 1) / WAVES));
#define CKTLU_LEVEL(T, C) \
    hipLaunchKernelGGL((refactor_level_kernel<T, C>), grid, dim3(WG), 0, st, a, cbeg, cend, pbeg, pend, tbeg, tend)
    if (a.fp32) {
        if (a.check) CKTLU_LEVEL(float, true); else CKTLU_LEVEL(float, false);
    } else {
        if (a.check) CKTLU_LEVEL(double, true); else CKTLU_LEVEL(double, false);
    }
#undef CKTLU_LEVEL
    return (int)hipGetLastError();
}

// ----------------------------------------------------------------- solves
// y holds one cache line (YS doubles) per row and instance: y[(inst*n + i)*YS + r].
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(WG) void trisolve_level_kernel(SolveArgs a, int lbeg, int lend) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t t = (int64_t)lbeg * a.batch + (int64_t)blockIdx.x * WAVES + wv;
    if (t >= (int64_t)lend * a.batch) return;
    const int inst = (int)(t % a.batch);
    if (a.skip && a.skip[inst] != -1) return;
    const int i = (UPPER ? a.useq : a.lseq)[t / a.batch];
    const int *rp = UPPER ? a.Urp : a.Lrp;
    const int *rj = UPPER ? a.Urj : a.Lrj;
    const int *rs = UPPER ? a.Ursrc : a.Lrsrc;
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    double *y = a.y + (size_t)inst * a.n * YS;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    // rows of the dense block take only their L entries in sparse columns here
    const int qend = (!UPPER && i >= a.tail0) ? a.tail_rend[i - a.tail0] : rp[i + 1];
    for (int q = rp[i] + lane; q < qend; q += WAVE) {
        const int j = rj[q];
        const double l = (double)Fx[rs[q]];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] += l * y[(size_t)j * YS + r];
    }
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = wave_sum(acc[r]);
    double mine = acc[0];
#pragma unroll
    for (int r = 1; r < NR; r++)
        if (lane == r) mine = acc[r];
    if (lane < NR) {
        double v = y[(size_t)i * YS + lane] - mine;
        if (UPPER) v = v / (double)Fx[a.udiag[i]];
        y[(size_t)i * YS + lane] = v;
    }
}

template <bool UPPER>
static int launch_solve_level_impl(const SolveArgs &a, int lbeg, int lend, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (int64_t)(lend - lbeg) * a.batch;
    const dim3 grid((unsigned)((waves + WAVES - 1) / WAVES));
#define CKTLU_SOLVE_CASE(NRV)                                                                          \
    case NRV:                                                                                          \
        if (a.fp32)                                                                                    \
            hipLaunchKernelGGL((trisolve_level_kernel<float, NRV, UPPER>), grid, dim3(WG), 0, st, a, lbeg, lend); \
        else                                                                                           \
            hipLaunchKernelGGL((trisolve_level_kernel<double, NRV, UPPER>), grid, dim3(WG), 0, st, a, lbeg, lend); \
        break;
    switch (a.nrhs) {
        CKTLU_SOLVE_CASE(1)
        CKTLU_SOLVE_CASE(2)
        CKTLU_SOLVE_CASE(4)
        CKTLU_SOLVE_CASE(8)
        default: return (int)hipErrorInvalidValue;
    }
#undef CKTLU_SOLVE_CASE
    return (int)hipGetLastError();
}

int launch_lsolve_level(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_level_impl<false>(a, lbeg, lend, stream);
}
int launch_usolve_level(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_level_impl<true>(a, lbeg, lend, stream);
}

// --------------------------------------------------------------- helpers
__global__ void gather_rhs_kernel(int n, int nrhs, int batch, const double *b, int64_t ldb,
                                  const int *perm, double *y) {
    const int64_t total = (int64_t)n * nrhs * batch;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t % nrhs);
        const int64_t ik = t / nrhs;
        const int k = (int)(ik % n);
        const int64_t i = ik / n;
        y[ik * YS + r] = b[(i * nrhs + r) * ldb + perm[k]];
    }
}

__global__ void scatter_sol_kernel(int n, int nrhs, int batch, const double *z, const int *perm,
                                   double *x, int64_t ldx, int accumulate, const int *skip) {
    const int64_t total = (int64_t)n * nrhs * batch;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t % nrhs);
        const int64_t ik = t / nrhs;
        const int k = (int)(ik % n);
        const int64_t i = ik / n;
        if (skip && skip[i] != -1) continue;
        double *dst = x + (i * nrhs + r) * ldx + perm[k];
        const double v = z[ik * YS + r];
        *dst = accumulate ? *dst + v : v;
    }
}

static inline int grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

int launch_gather_rhs(int n, int nrhs, int batch, const double *b, int64_t ldb, const int *perm,
                      double *y, void *stream) {
    hipLaunchKernelGGL(gather_rhs_kernel, dim3(grid_for((int64_t)n * nrhs * batch, 256)), dim3(256), 0,
                       (hipStream_t)stream, n, nrhs, batch, b, ldb, perm, y);
    return (int)hipGetLastError();
}

int launch_scatter_sol(int n, int nrhs, int batch, const double *z, const int *perm, double *x,
                       int64_t ldx, int accumulate, const int *skip, void *stream) {
    hipLaunchKernelGGL(scatter_sol_kernel, dim3(grid_for((int64_t)n * nrhs * batch, 256)), dim3(256), 0,
                       (hipStream_t)stream, n, nrhs, batch, z, perm, x, ldx, accumulate, skip);
    return (int)hipGetLastError();
}

// non-negative doubles order like their bit patterns as signed 64-bit integers
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__global__ void residual_kernel(int n, int nrhs, const int *Acp, const int *Acj, const int *Acsrc,
                                const double *Aval, const double *x, int64_t ldx, const double *b,
                                int64_t ldb, double *r, int64_t ldr, double *norms) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int rr = 0; rr < nrhs; rr++) {
            const double *xv = x + rr * ldx;
            double s = b[rr * ldb + i];
            for (int p = Acp[i]; p < Acp[i + 1]; p++) s -= Aval[Acsrc[p]] * xv[Acj[p]];
            r[rr * ldr + i] = s;
            atomic_max_nonneg(&norms[3 * rr + 0], fabs(s));
            atomic_max_nonneg(&norms[3 * rr + 1], fabs(xv[i]));
            atomic_max_nonneg(&norms[3 * rr + 2], fabs(b[rr * ldb + i]));
        }
    }
}

int launch_residual(int n, int nrhs, const int *Acp, const int *Acj, const int *Acsrc,
                    const double *Aval, const double *x, int64_t ldx, const double *b, int64_t ldb,
                    double *r, int64_t ldr, double *norms, void *stream) {
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, nrhs,
                       Acp, Acj, Acsrc, Aval, x, ldx, b, ldb, r, ldr, norms);
    return (int)hipGetLastError();
}

__global__ void anorm_kernel(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int p = Acp[i]; p < Acp[i + 1]; p++) s += fabs(Aval[Acsrc[p]]);
        atomic_max_nonneg(out, s);
    }
}

int launch_anorm(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out, void *stream) {
    hipLaunchKernelGGL(anorm_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, Acp, Acsrc,
                       Aval, out);
    return (int)hipGetLastError();
}

__global__ void copy_f64_kernel(const double *src, double *dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void f64_to_f32_kernel(const double *src, float *dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

__global__ void fill_i32_kernel(int *dst, int64_t count, int value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

int launch_copy_f64(const double *src, double *dst, int64_t count, void *stream) {
    hipLaunchKernelGGL(copy_f64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, src, dst,
                       count);
    return (int)hipGetLastError();
}

int launch_f64_to_f32(const double *src, float *dst, int64_t count, void *stream) {
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, src, dst,
                       count);
    return (int)hipGetLastError();
}

int launch_fill_i32(int *dst, int64_t count, int value, void *stream) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, dst, count,
                       value);
    return (int)hipGetLastError();
}

}  // namespace cktlu_dev
