// Device kernels of the cktlu hot path (gfx950).
//
// refactor_level_kernel: fast factorization with pivot check (Section IV-B),
//   cluster mode: one launch per dependency level of the column graph, one
//   wavefront per (column, instance) of the level.  Every predecessor of a
//   column sits in an earlier level, so it is complete when the launch starts
//   and no wavefront ever waits on another.  A column applies the
//   left-looking updates of its predecessors in ascending order on a work
//   vector in LDS, tests its pivot against eps times the largest entry of its
//   L part, stores U and L = x / pivot, and on failure records its index
//   (atomic minimum) and raises the instance's interrupt word, which makes all
//   later levels of that instance return at once (Algorithm 3: the level runs
//   to its barrier, then the threads exit).
//
// trisolve_level_kernel: triangular solves (Section II-C, Algorithm 2) in the
//   row ("pull") form, one launch per level of the solve dependency graph, one
//   wavefront per (row, instance); each row reduces its dot product in a fixed
//   order.  Deterministic.
//
// The level kernels keep all communication between wavefronts at kernel
// boundaries, where the runtime makes device memory coherent across the
// MI355X's eight XCDs (each has its own L2).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"

namespace cktlu_dev {

constexpr int WAVE = 64;
constexpr int WG = 256;
constexpr int WAVES = WG / WAVE;
constexpr int CAP = 1024;   // LDS work-vector slots per wavefront

// Orders this wavefront's work-vector accesses (LDS or global) across lanes.
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

// first index in rows[0, len) with rows[idx] >= r
__device__ __forceinline__ int find_slot(const int *rows, int len, int r) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rows[mid] < r) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ refactorize
template <typename T, bool CHECK>
__global__ __launch_bounds__(WG) void refactor_level_kernel(RefactorArgs a, int lbeg, int lend) {
    __shared__ T xs_all[WAVES][CAP];
    __shared__ int rows_all[WAVES][CAP];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t t = (int64_t)lbeg * a.batch + (int64_t)blockIdx.x * WAVES + wv;
    if (t >= (int64_t)lend * a.batch) return;
    const int inst = (int)(t % a.batch);
    int *interrupted = a.ctrl + 1;
    int *firstfail = a.ctrl + 1 + a.batch;
    if (CHECK && interrupted[inst]) return;          // an earlier level failed its check
    const int k = a.seq[t / a.batch];
    const int base = a.Dp[k], len = a.Dlen[k], nu = a.nU[k];
    const int *rowsg = a.Fi + base;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    const double *Av = a.Aval + (size_t)inst * a.nnzA;
    const bool inlds = len <= CAP;
    T *xl = xs_all[wv];
    int *rl = rows_all[wv];
    T *x = inlds ? xl : reinterpret_cast<T *>(a.scratch) + (size_t)(blockIdx.x * WAVES + wv) * a.max_col;
    const int *rows = inlds ? rl : rowsg;
    for (int i = lane; i < len; i += WAVE) {
        x[i] = T(0);
        if (inlds) rl[i] = rowsg[i];
    }
    wave_sync();
    const int c = a.colperm[k];
    for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) x[a.amap[p]] = (T)Av[p];
    wave_sync();
    // left-looking update by every predecessor j (rows of U(:,k) above the diagonal), ascending
    for (int u = 0; u < nu - 1; ++u) {
        const int j = rows[u];
        const T xj = x[u];
        const int lb = a.Dp[j] + a.nU[j], le = a.Dp[j] + a.Dlen[j];
        for (int q = lb + lane; q < le; q += WAVE) {
            const int r = a.Fi[q];
            const T l = Fx[q];
            const int s = find_slot(rows, len, r);
            if (s < len) x[s] -= l * xj;   // always found: struct(L(:,j)) is inside struct(col k)
        }
        wave_sync();
    }
    const T d = x[nu - 1];
    if (CHECK) {
        double m = 0.0;
        int bad = 0;
        for (int i = nu + lane; i < len; i += WAVE) {
            const double v = (double)x[i];
            if (!isfinite(v)) bad = 1;
            m = fmax(m, fabs(v));
        }
        m = wave_max(m);
        bad = __any(bad);
        const double dd = (double)d;
        if (bad || !isfinite(dd) || dd == 0.0 || fabs(dd) < a.eps * m || k == a.force_fail_col) {
            if (lane == 0) {
                atomicMin(&firstfail[inst], k);
                atomicExch(&interrupted[inst], 1);
            }
            return;
        }
    }
    for (int i = lane; i < nu; i += WAVE) Fx[base + i] = x[i];
    for (int i = nu + lane; i < len; i += WAVE) Fx[base + i] = x[i] / d;
    if (CHECK && lane == 0) a.done[(size_t)inst * a.n + k] = (int)a.epoch;
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

int launch_refactor_level(const RefactorArgs &a, int lbeg, int lend, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (int64_t)(lend - lbeg) * a.batch;
    const dim3 grid((unsigned)((waves + WAVES - 1) / WAVES));
    if (a.fp32) {
        if (a.check) hipLaunchKernelGGL((refactor_level_kernel<float, true>), grid, dim3(WG), 0, st, a, lbeg, lend);
        else hipLaunchKernelGGL((refactor_level_kernel<float, false>), grid, dim3(WG), 0, st, a, lbeg, lend);
    } else {
        if (a.check) hipLaunchKernelGGL((refactor_level_kernel<double, true>), grid, dim3(WG), 0, st, a, lbeg, lend);
        else hipLaunchKernelGGL((refactor_level_kernel<double, false>), grid, dim3(WG), 0, st, a, lbeg, lend);
    }
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
    for (int q = rp[i] + lane; q < rp[i + 1]; q += WAVE) {
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
