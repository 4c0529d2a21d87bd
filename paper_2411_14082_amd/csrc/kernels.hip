// Device kernels of the cktlu hot path (gfx950).
//
// refactor_kernel: fast factorization with pivot check (Section IV-B).  The
//   paper's cluster mode (level by level) and pipeline mode (an atomic
//   counter hands out the next node of a dependency-ordered sequence; a node
//   waits until each predecessor has finished, watching a shared
//   "interrupted" flag) become one persistent kernel: every wavefront takes
//   the next column of the level-ordered sequence from a device counter,
//   applies the left-looking updates of its predecessors in ascending order
//   as they become ready, tests its pivot against eps times the largest entry
//   of its L part, stores L and U and publishes a per-column ready flag.  A
//   failed test records the column and raises the instance's interrupt flag;
//   waiters see it and stop.  Because the counter hands out columns in
//   topological order and only running wavefronts hold columns, every awaited
//   column belongs to a running wavefront; a bounded wait (watchdog) turns any
//   violation into an error instead of a hang.
//
// trisolve_kernel: triangular solves (Section II-C, Section V) in the row
//   ("pull") form with per-row ready flags: each wavefront takes the next row,
//   waits for the solution entries it reads, reduces its dot product in a
//   fixed order and publishes its own entry.  Deterministic.
//
// Cross-workgroup visibility on a multi-XCD MI355X: each XCD has its own L2,
// and a plain store can stay in the writer's L2 until the kernel ends.  So
// every flag is written with an atomic exchange and read with an atomic
// compare-and-swap (both are performed at the device coherence point), data is
// written back (release fence) before its flag is set, and every column of the
// factor storage and every row of the solve vectors starts on its own cache
// line, so no XCD can hold a line of data it has not yet been signalled for.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"

namespace cktlu_dev {

constexpr int WAVE = 64;
constexpr int WG = 256;
constexpr int WAVES = WG / WAVE;
constexpr int CAP = 1024;   // LDS work-vector slots per wavefront

__device__ __forceinline__ int flag_read(int *p, int expect) {
    return atomicCAS(p, expect, expect);   // an RMW: never served from a stale cache line
}
__device__ __forceinline__ void flag_write(int *p, int v) { atomicExch(p, v); }
__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

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

// Watchdog: the first wait that exceeds the limit records (waiter, awaited, ticket).
__device__ __forceinline__ void watchdog_trip(int *err, int code, int waiter, int awaited, int ticket) {
    if (atomicCAS(err, 0, code) == 0) {
        atomicExch(err + 1, waiter);
        atomicExch(err + 2, awaited);
        atomicExch(err + 3, ticket);
    }
}

// ------------------------------------------------------------ refactorize
template <typename T, bool CHECK>
__global__ __launch_bounds__(WG) void refactor_kernel(RefactorArgs a) {
    __shared__ T xs_all[WAVES][CAP];
    __shared__ int rows_all[WAVES][CAP];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    T *xl = xs_all[wv];
    int *rl = rows_all[wv];
    T *xg = a.scratch ? reinterpret_cast<T *>(a.scratch) + (size_t)(blockIdx.x * WAVES + wv) * a.max_col
                      : nullptr;
    int *interrupted = a.ctrl + 1;
    int *firstfail = a.ctrl + 1 + a.batch;
    const int total = a.n * a.batch;
    const int epoch = (int)a.epoch;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(a.ctrl, 1);
        t = __shfl(t, 0);
        if (t >= total) break;
        const int inst = t % a.batch;
        const int k = a.seq[t / a.batch];
        const int base = a.Dp[k], len = a.Dlen[k], nu = a.nU[k];
        const int *rowsg = a.Fi + base;
        T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
        const double *Av = a.Aval + (size_t)inst * a.nnzA;
        int *ready = a.ready + (size_t)inst * a.n;
        const bool inlds = len <= CAP;
        T *x = inlds ? xl : xg;
        const int *rows = inlds ? rl : rowsg;
        for (int i = lane; i < len; i += WAVE) {
            x[i] = T(0);
            if (inlds) rl[i] = rowsg[i];
        }
        wave_sync();
        const int c = a.colperm[k];
        for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) x[a.amap[p]] = (T)Av[p];
        wave_sync();
        int abort = 0, ready_upto = 0;
        for (int u = 0; u < nu - 1; ++u) {
            if (u >= ready_upto) {
                // poll the next 64 dependencies in parallel; proceed with the ready prefix
                int spins = 0;
                for (;;) {
                    const int idx = u + lane;
                    bool ok = true;
                    if (idx < nu - 1) ok = flag_read(&ready[rows[idx]], epoch) == epoch;
                    const unsigned long long notok = __ballot(!ok);
                    const int prefix = notok ? __ffsll((long long)notok) - 1 : WAVE;
                    if (prefix > 0) { ready_upto = u + prefix; break; }
                    int stop = 0;
                    if (lane == 0) {
                        if (flag_read(&interrupted[inst], 1) != 0) stop = 1;
                        else if (++spins > a.spin_limit) {
                            watchdog_trip(a.err, 1, k, rows[u], t);
                            flag_write(&interrupted[inst], 1);
                            stop = 1;
                        }
                    }
                    stop = __shfl(stop, 0);
                    if (stop) { abort = 1; break; }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (abort) break;
                acquire_agent();
            }
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
        if (abort) continue;
        const T d = x[nu - 1];
        double m = 0.0;
        int bad = 0;
        for (int i = nu + lane; i < len; i += WAVE) {
            const double v = (double)x[i];
            if (!isfinite(v)) bad = 1;
            m = fmax(m, fabs(v));
        }
        bool fail = false;
        if (CHECK) {
            m = wave_max(m);
            bad = __any(bad);
            const double dd = (double)d;
            fail = bad || !isfinite(dd) || dd == 0.0 || fabs(dd) < a.eps * m || k == a.force_fail_col;
        }
        if (fail) {
            if (lane == 0) {
                atomicMin(&firstfail[inst], k);
                flag_write(&interrupted[inst], 1);
            }
            continue;
        }
        for (int i = lane; i < nu; i += WAVE) Fx[base + i] = x[i];
        for (int i = nu + lane; i < len; i += WAVE) Fx[base + i] = x[i] / d;
        release_agent();
        if (lane == 0) flag_write(&ready[k], epoch);
    }
}

__global__ void reset_ctrl_kernel(int *ctrl, int nwords, int value, int batch) {
    // ctrl[0] = 0 (ticket); ctrl[1..batch] = 0 (interrupt); the rest = value
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        ctrl[i] = (i == 0 || i <= batch) ? 0 : value;
}

int launch_reset_ctrl(int *ctrl, int nwords, int value, void *stream) {
    // layout: [ticket][interrupt x batch][firstfail x batch]; batch = (nwords-1)/2
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

int launch_refactor(const RefactorArgs &a, int grid, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.fp32) {
        if (a.check) hipLaunchKernelGGL((refactor_kernel<float, true>), dim3(grid), dim3(WG), 0, st, a);
        else hipLaunchKernelGGL((refactor_kernel<float, false>), dim3(grid), dim3(WG), 0, st, a);
    } else {
        if (a.check) hipLaunchKernelGGL((refactor_kernel<double, true>), dim3(grid), dim3(WG), 0, st, a);
        else hipLaunchKernelGGL((refactor_kernel<double, false>), dim3(grid), dim3(WG), 0, st, a);
    }
    return (int)hipGetLastError();
}

// ----------------------------------------------------------------- solves
// y holds one cache line (YS doubles) per row and instance: y[(inst*n + i)*YS + r].
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(WG) void trisolve_kernel(SolveArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int total = a.n * a.batch;
    const int epoch = (int)a.epoch;
    const int *rp = UPPER ? a.Urp : a.Lrp;
    const int *rj = UPPER ? a.Urj : a.Lrj;
    const int *rs = UPPER ? a.Ursrc : a.Lrsrc;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(a.ctrl, 1);
        t = __shfl(t, 0);
        if (t >= total) break;
        const int inst = t % a.batch;
        const int i = UPPER ? a.n - 1 - t / a.batch : t / a.batch;
        if (a.skip && a.skip[inst] != -1) continue;
        const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
        double *y = a.y + (size_t)inst * a.n * YS;
        int *ready = a.ready + (size_t)inst * a.n;
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] = 0.0;
        for (int q0 = rp[i]; q0 < rp[i + 1]; q0 += WAVE) {
            const int q = q0 + lane;
            const bool act = q < rp[i + 1];
            const int j = act ? rj[q] : 0;
            const double l = act ? (double)Fx[rs[q]] : 0.0;
            bool ok = !act || flag_read(&ready[j], epoch) == epoch;
            int spins = 0;
            while (!__all(ok)) {
                if (!ok) ok = flag_read(&ready[j], epoch) == epoch;
                if (++spins > a.spin_limit) {   // watchdog: never wait forever
                    if (lane == 0) watchdog_trip(a.err, 2, i, j, t);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            acquire_agent();
            if (act) {
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] += l * y[(size_t)j * YS + r];
            }
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
        release_agent();
        if (lane == 0) flag_write(&ready[i], epoch);
    }
}

template <bool UPPER>
static int launch_solve_impl(const SolveArgs &a, int grid, void *stream) {
    hipStream_t st = (hipStream_t)stream;
#define CKTLU_SOLVE_CASE(NRV)                                                                    \
    case NRV:                                                                                    \
        if (a.fp32)                                                                              \
            hipLaunchKernelGGL((trisolve_kernel<float, NRV, UPPER>), dim3(grid), dim3(WG), 0, st, a); \
        else                                                                                     \
            hipLaunchKernelGGL((trisolve_kernel<double, NRV, UPPER>), dim3(grid), dim3(WG), 0, st, a); \
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

int launch_lsolve(const SolveArgs &a, int grid, void *stream) { return launch_solve_impl<false>(a, grid, stream); }
int launch_usolve(const SolveArgs &a, int grid, void *stream) { return launch_solve_impl<true>(a, grid, stream); }

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

// Resident workgroups of the persistent kernels (kind 0: refactorize, 1: solve).
int occupancy_grid(int kind, int *grid) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    if (kind == 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, refactor_kernel<double, true>, WG, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, trisolve_kernel<double, 1, false>, WG, 0);
    if (e != hipSuccess) return (int)e;
    if (per < 1) per = 1;
    *grid = cus * per;
    return 0;
}

}  // namespace cktlu_dev
