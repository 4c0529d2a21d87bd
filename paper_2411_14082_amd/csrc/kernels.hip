// Device kernels of the cktlu hot path (gfx950), apart from the dense block and the
// supernodal sweep (dense.hip).
//
// Refactorization (fast factorization with pivot check, Section IV-B):
//   refactor_init_kernel   zeroes every factor column and scatters the matrix
//                          values into it (sixteen lanes per sparse column, a wavefront
//                          per dense-block column);
//   refactor_level_kernel  the column sweep (options.sweep_supernodes = -1), one launch
//                          per level l: (a) tests the pivot of every column of level l
//                          against eps times the largest entry of its L part (its values
//                          are final: every update came from an earlier level); (b)
//                          divides the L part of every column of level l-1 by its pivot;
//                          (c) runs the update tasks of level l: a task owns one target
//                          column k and applies x_k -= L(:,j) * U(j,k) for every source j
//                          of level l with U(j,k) != 0, in ascending j, so no two
//                          wavefronts write the same column and results are
//                          bit-reproducible.
// This is the paper's cluster mode (Algorithm 3) with the left-looking column update of
// the paper turned around: a column's updates are spread over the levels of its sources,
// so the critical path is the number of levels, not the length of a column's update list.
// A failed test records the column (atomic minimum) and the level in the instance's
// interrupt word; later levels of that instance return at once.  The default sweep works
// on supernodes (dense.hip) with the same ownership rules.
//
// Solves (Section II-C, Algorithm 2), row ("pull") form: sn_solve_kernel takes one level
// of supernodes per launch (the default; wide supernodes pull by runs of consecutive rows
// in one column); trisolve_level_kernel / trisolve_rowwg_kernel /
// trisolve_chain_kernel take one level of rows (the column sweep's schedule, and the rows
// of the dense block's L entries in sparse columns).
//
// All communication between workgroups happens at kernel boundaries, where the runtime
// makes device memory coherent across the MI355X's eight XCDs, except for the arrival
// counters of split supernodes: the units of one supernode publish partial sums with a
// release fence and an atomic increment, and the last to arrive (which never waits for
// another) reads them after an acquire fence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

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
// sixteen lanes per (sparse column, instance), one wavefront per (dense-block column,
// instance).  Columns of the dense block keep their rows >= T in S (column k at
// S + (k - T) D), so those rows are zeroed there.
template <typename T>
__global__ __launch_bounds__(WG) void refactor_init_kernel(RefactorArgs a, unsigned nsb) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const double *Av;
    if (blockIdx.x < nsb) {
        // sparse columns: sixteen per workgroup
        const int l16 = threadIdx.x & 15;
        const int64_t g = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
        if (g >= (int64_t)a.T * a.batch) return;
        const int inst = (int)(g % a.batch);
        const int k = (int)(g / a.batch);
        T *x = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[k];
        Av = a.Aval + (size_t)inst * a.nnzA;
        const int len = a.Dlen[k];
        const int c = a.colperm[k];
        for (int i = l16; i < len; i += 16) x[i] = T(0);
        wave_sync();
        for (int p = a.Ap[c] + l16; p < a.Ap[c + 1]; p += 16) x[a.amap[p]] = (T)(a.ascale ? Av[p] * a.ascale[p] : Av[p]);
        return;
    }
    const int64_t w = (int64_t)(blockIdx.x - nsb) * WAVES + wv;
    if (w >= (int64_t)(a.n - a.T) * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int k = a.T + (int)(w / a.batch);
    T *x = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[k];
    Av = a.Aval + (size_t)inst * a.nnzA;
    const int len = a.Dlen[k];
    const int c = a.colperm[k];
    T *Sk = reinterpret_cast<T *>(a.S) + (size_t)inst * a.D * a.D + (size_t)(k - a.T) * a.D;
    const int *rows = a.Fi + a.Dp[k];
    for (int i = lane; i < len; i += WAVE) x[i] = T(0);
    for (int i = lane; i < a.D; i += WAVE) Sk[i] = T(0);
    wave_sync();
    for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) {
        const int slot = a.amap[p];
        const int r = rows[slot];
        const double v = a.ascale ? Av[p] * a.ascale[p] : Av[p];
        if (r >= a.T) Sk[r - a.T] = (T)v;
        else x[slot] = (T)v;
    }
}

// S = A22 (one instance): the dense columns' matrix values in rows >= T, zeros
// elsewhere; their rows < T (already final) are not touched.  One wavefront per column.
__global__ __launch_bounds__(WG) void dense_reinit_kernel(RefactorArgs a) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t w = (int64_t)blockIdx.x * WAVES + wv;
    if (w >= a.D) return;
    const int k = a.T + (int)w;
    double *Sk = reinterpret_cast<double *>(a.S) + (size_t)w * a.D;
    const int *rows = a.Fi + a.Dp[k];
    const int c = a.colperm[k];
    for (int i = lane; i < a.D; i += WAVE) Sk[i] = 0.0;
    wave_sync();
    for (int p = a.Ap[c] + lane; p < a.Ap[c + 1]; p += WAVE) {
        const int r = rows[a.amap[p]];
        if (r >= a.T) Sk[r - a.T] = a.ascale ? a.Aval[p] * a.ascale[p] : a.Aval[p];
    }
}

int launch_dense_reinit(const RefactorArgs &a, void *stream) {
    if (a.D <= 0) return 0;
    hipLaunchKernelGGL(dense_reinit_kernel, dim3((unsigned)((a.D + WAVES - 1) / WAVES)), dim3(WG), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

constexpr int kItemChunk = 4;      // entries of a source column per lane per pass (longer sources)

// x_k -= L(:,j) U(j,k) for one source j (item {pivot position, L begin, L end,
// slot of row j}) of an update task, kItemChunk entries per lane per pass.  A pass
// loads its entries, locates their rows in the target (rows >= T of a dense-block
// target directly in Sk; others by a branch-free binary search over the searched
// part of column k, the same range for every entry, run in lockstep, in LDS when
// staged), loads every target value and only then stores: the rows of one source
// are distinct, so no store of a pass can feed a load of the same pass.
// With the slot map (MAP) the caller's r0 and the entries loaded here are the slots
// themselves (mp: the map of this item) and there is no search.
template <typename T, int U, bool MAP>
__device__ __forceinline__ void apply_item_u(const RefactorArgs &a, const T *Fx, T *xk, T *Sk, const int *rowsk,
                                             const int *lrows, bool staged, int slen, int lb, int le, int lo0,
                                             T iv, T m, int lane, const int (&r0)[kItemChunk],
                                             const T (&l0)[kItemChunk], const int *mp) {
    for (int q0 = lb; q0 < le; q0 += U * WAVE) {
        int r[U];
        T l[U];
        if (q0 == lb) {                                   // the first pass was loaded by the caller
#pragma unroll
            for (int u = 0; u < U; u++) { r[u] = r0[u]; l[u] = l0[u]; }
        } else {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = q0 + u * WAVE + lane;
                r[u] = q < le ? (MAP ? mp[q - lb] : a.Fi[q]) : -1;
                l[u] = q < le ? Fx[q] : T(0);
            }
        }
        // target slot of each entry: >= 0 in xk, < -1 as -(2 + offset) in Sk, -1 none
        int pos[U];
        if constexpr (MAP) {
#pragma unroll
            for (int u = 0; u < U; u++) pos[u] = r[u];
        } else {
            int base[U];
#pragma unroll
            for (int u = 0; u < U; u++) base[u] = lo0;
            int cnt = slen - lo0;                              // lower bound of r in rows [lo0, slen)
            if (staged) {
                while (cnt > 1) {
                    const int half = cnt >> 1;
#pragma unroll
                    for (int u = 0; u < U; u++) base[u] = lrows[base[u] + half - 1] < r[u] ? base[u] + half : base[u];
                    cnt -= half;
                }
                if (cnt == 1) {
#pragma unroll
                    for (int u = 0; u < U; u++) base[u] += lrows[base[u]] < r[u] ? 1 : 0;
                }
            } else {
                while (cnt > 1) {
                    const int half = cnt >> 1;
#pragma unroll
                    for (int u = 0; u < U; u++) base[u] = rowsk[base[u] + half - 1] < r[u] ? base[u] + half : base[u];
                    cnt -= half;
                }
                if (cnt == 1) {
#pragma unroll
                    for (int u = 0; u < U; u++) base[u] += rowsk[base[u]] < r[u] ? 1 : 0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (r[u] < 0) pos[u] = -1;
                else if (Sk && r[u] >= a.T) pos[u] = -(2 + (r[u] - a.T));
                else pos[u] = base[u] < slen ? base[u] : -1;  // always found: struct(L(:,j)) is inside struct(col k)
            }
        }
        T tv[U];
#pragma unroll
        for (int u = 0; u < U; u++) tv[u] = pos[u] >= 0 ? xk[pos[u]] : (pos[u] < -1 ? Sk[-(pos[u] + 2)] : T(0));
#pragma unroll
        for (int u = 0; u < U; u++) {
            const T v = tv[u] - l[u] * iv * m;
            if (pos[u] >= 0) xk[pos[u]] = v;
            else if (pos[u] < -1) Sk[-(pos[u] + 2)] = v;
        }
    }
}

// Sources of at most one entry per lane take the single-entry path (one search
// per lane); longer ones kItemChunk entries per lane per pass.
template <typename T, bool MAP>
__device__ __forceinline__ void apply_item(const RefactorArgs &a, const T *Fx, T *xk, T *Sk, const int *rowsk,
                                           const int *lrows, bool staged, int slen, int lb, int le, int lo0,
                                           T iv, T m, int lane, const int (&r0)[kItemChunk],
                                           const T (&l0)[kItemChunk], const int *mp) {
    if (le - lb <= WAVE)
        apply_item_u<T, 1, MAP>(a, Fx, xk, Sk, rowsk, lrows, staged, slen, lb, le, lo0, iv, m, lane, r0, l0, mp);
    else
        apply_item_u<T, kItemChunk, MAP>(a, Fx, xk, Sk, rowsk, lrows, staged, slen, lb, le, lo0, iv, m, lane, r0,
                                         l0, mp);
}

// one wavefront per (task, instance); tasks: [checks | normalisations | updates].
// The interrupt word of an instance holds 1 + the level whose check failed first (0:
// none).  Every part of launch `lev` stops only for a failure of an earlier level, never
// for one of its own level, so which columns finish does not depend on the order in
// which the launch's wavefronts run: after a failure at level f the columns of levels
// below f are final and normalised, those of levels >= f are not.
template <typename T, bool CHECK, bool MAP>
__global__ __launch_bounds__(WG) void refactor_level_kernel(RefactorArgs a, int cbeg, int cend, int pbeg,
                                                             int pend, int tbeg, int tend, int lev) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t w = (int64_t)blockIdx.x * WAVES + wv;
    const int nchk = cend - cbeg, nnorm = pend - pbeg, nupd = tend - tbeg;
    if (w >= (int64_t)(nchk + nnorm + nupd) * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int idx = (int)(w / a.batch);
    int *interrupted = a.ctrl + 1;
    int *firstfail = a.ctrl + 1 + a.batch;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int4 *colrec = reinterpret_cast<const int4 *>(a.colrec);
    if (idx < nchk) {
        // (a) pivot check of a column of this level
        if (!CHECK) return;
        const int4 cr = colrec[cbeg + idx];
        const int stop = interrupted[inst];
        const int j = cr.w, nu = cr.y, len = cr.z;
        const T *x = Fx + cr.x;
        double m = 0.0;
        int bad = 0;
        for (int i0 = nu; i0 < len; i0 += 4 * WAVE) {   // four loads in flight per lane
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) v[u] = i0 + u * WAVE + lane < len ? (double)x[i0 + u * WAVE + lane] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (!isfinite(v[u])) bad = 1;
                m = fmax(m, fabs(v[u]));
            }
        }
        const double d = (double)x[nu - 1];
        if (stop && stop <= lev) return;                  // an earlier level failed its check
        m = wave_max(m);
        bad = __any(bad);
        if (bad || !isfinite(d) || d == 0.0 || fabs(d) < a.eps * m || j == a.force_fail_col) {
            if (lane == 0) {
                atomicMin(&firstfail[inst], j);
                atomicExch(&interrupted[inst], lev + 1);  // every writer of this launch writes the same
            }
        }
        return;
    }
    if (idx < nchk + nnorm) {
        // (b) L(:,j) = x / pivot for a column of the previous level
        const int4 cr = colrec[pbeg + idx - nchk];
        const int stop = CHECK ? interrupted[inst] : 0;
        const int j = cr.w, nu = cr.y, len = cr.z;
        T *x = Fx + cr.x;
        const T d = x[nu - 1];
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = nu + u * WAVE + lane < len ? x[nu + u * WAVE + lane] : T(0);
        if (stop && stop <= lev) return;                  // level lev-1 passed: normalised whatever lev does
        for (int i0 = nu; i0 < len; i0 += 4 * WAVE) {
            if (i0 != nu) {
#pragma unroll
                for (int u = 0; u < 4; u++) v[u] = i0 + u * WAVE + lane < len ? x[i0 + u * WAVE + lane] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (i0 + u * WAVE + lane < len) x[i0 + u * WAVE + lane] = v[u] / d;
        }
        if (lane == 0) a.done[(size_t)inst * a.n + j] = (int)a.epoch;
        return;
    }
    // (c) update task: target column k, sources j of this level in ascending order.
    // Every load that does not depend on another is issued before the first wait:
    // the task record, then the first item's pivot, multiplier and first entries,
    // the extra items and the target rows to stage in LDS.
    const int t = tbeg + idx - nchk - nnorm;
    const int4 *task8 = reinterpret_cast<const int4 *>(a.task8);
    const int4 h = task8[2 * t], it0 = task8[2 * t + 1];
    const int xend = task8[2 * t + 2].w;
    const int stop = CHECK ? interrupted[inst] : 0;
    const int k = h.x, bk = h.y, slen = h.z, xbeg = h.w;
    T *xk = Fx + bk;
    const int *rowsk = a.Fi + bk;
    T *Sk = k >= a.T ? reinterpret_cast<T *>(a.S) + (size_t)inst * a.D * a.D + (size_t)(k - a.T) * a.D : nullptr;
    const T piv0 = Fx[it0.x];                             // the pivot of j (not yet divided into L(:,j))
    const T mult0 = xk[it0.w];                            // U(j,k): final, no source of this level updates it
    const int *mp = MAP ? a.smap + a.tmoff[t] : nullptr;   // slots of this task's entries, item by item
    int r0[kItemChunk];
    T l0[kItemChunk];
#pragma unroll
    for (int u = 0; u < kItemChunk; u++) {
        const int q = it0.y + u * WAVE + lane;
        r0[u] = q < it0.z ? (MAP ? mp[q - it0.y] : a.Fi[q]) : -1;
        l0[u] = q < it0.z ? Fx[q] : T(0);
    }
    int4 itx = make_int4(0, 0, 0, 0);
    if (xbeg + lane < xend) itx = reinterpret_cast<const int4 *>(a.item4)[xbeg + lane];
    __shared__ int srows[MAP ? 1 : WAVES][MAP ? 1 : kStageRows];
    int *lrows = srows[MAP ? 0 : wv];
    const bool staged = !MAP && slen <= kStageRows;
    if (staged) {
        for (int i0 = 0; i0 < slen; i0 += 4 * WAVE) {
            int rr[4];
#pragma unroll
            for (int u = 0; u < 4; u++) rr[u] = i0 + u * WAVE + lane < slen ? rowsk[i0 + u * WAVE + lane] : 0;
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (i0 + u * WAVE + lane < slen) lrows[i0 + u * WAVE + lane] = rr[u];
        }
    }
    if (stop && stop <= lev) return;                      // an earlier level failed its check
    wave_sync();                                          // staged rows visible to the whole wavefront
    apply_item<T, MAP>(a, Fx, xk, Sk, rowsk, lrows, staged, slen, it0.y, it0.z, it0.w + 1, T(1) / piv0, mult0,
                       lane, r0, l0, mp);
    if (xend == xbeg) return;
    if (MAP) mp += it0.z - it0.y;
    // further sources of this task (lane u holds the record of the u-th)
    T invx = T(0), multx = T(0);
    const int nx = min(WAVE, xend - xbeg);
    wave_sync();                                          // this item's updates visible before the next reads
    if (lane < nx) {
        invx = T(1) / Fx[itx.x];
        multx = xk[itx.w];
    }
    for (int u = 0; u < nx; ++u) {
        const int lb = __shfl(itx.y, u), le = __shfl(itx.z, u), lo0 = __shfl(itx.w, u) + 1;
        const T iv = __shfl(invx, u), m = __shfl(multx, u);
#pragma unroll
        for (int v = 0; v < kItemChunk; v++) {
            const int q = lb + v * WAVE + lane;
            r0[v] = q < le ? (MAP ? mp[q - lb] : a.Fi[q]) : -1;
            l0[v] = q < le ? Fx[q] : T(0);
        }
        apply_item<T, MAP>(a, Fx, xk, Sk, rowsk, lrows, staged, slen, lb, le, lo0, iv, m, lane, r0, l0, mp);
        if (MAP) mp += le - lb;
        wave_sync();
    }
    // more than WAVE sources in one task: the rest one at a time
    for (int i = xbeg + WAVE; i < xend; ++i) {
        const int4 it = reinterpret_cast<const int4 *>(a.item4)[i];
        const T iv = T(1) / Fx[it.x], m = xk[it.w];
#pragma unroll
        for (int v = 0; v < kItemChunk; v++) {
            const int q = it.y + v * WAVE + lane;
            r0[v] = q < it.z ? (MAP ? mp[q - it.y] : a.Fi[q]) : -1;
            l0[v] = q < it.z ? Fx[q] : T(0);
        }
        apply_item<T, MAP>(a, Fx, xk, Sk, rowsk, lrows, staged, slen, it.y, it.z, it.w + 1, iv, m, lane, r0, l0,
                           mp);
        if (MAP) mp += it.z - it.y;
        wave_sync();
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
    const int64_t sparse = (int64_t)a.T * a.batch, dense = (int64_t)(a.n - a.T) * a.batch;
    const int64_t nsb = (sparse + 15) / 16, blocks = nsb + (dense + WAVES - 1) / WAVES;
    if (blocks == 0) return 0;
    if (blocks > UINT_MAX) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (a.fp32) hipLaunchKernelGGL((refactor_init_kernel<float>), grid, dim3(WG), 0, st, a, (unsigned)nsb);
    else hipLaunchKernelGGL((refactor_init_kernel<double>), grid, dim3(WG), 0, st, a, (unsigned)nsb);
    return (int)hipGetLastError();
}

int launch_refactor_level(const RefactorArgs &a, int cbeg, int cend, int pbeg, int pend, int tbeg, int tend,
                          int lev, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (int64_t)((cend - cbeg) + (pend - pbeg) + (tend - tbeg)) * a.batch;
    if (waves == 0) return 0;
    const dim3 grid((unsigned)((waves + WAVES - 1) / WAVES));
#define CKTLU_LEVEL(T, C)                                                                                     \
    do {                                                                                                      \
        if (a.smap)                                                                                           \
            hipLaunchKernelGGL((refactor_level_kernel<T, C, true>), grid, dim3(WG), 0, st, a, cbeg, cend, pbeg, \
                               pend, tbeg, tend, lev);                                                       \
        else                                                                                                  \
            hipLaunchKernelGGL((refactor_level_kernel<T, C, false>), grid, dim3(WG), 0, st, a, cbeg, cend, pbeg,\
                               pend, tbeg, tend, lev);                                                       \
    } while (0)
    if (a.fp32) {
        if (a.check) CKTLU_LEVEL(float, true); else CKTLU_LEVEL(float, false);
    } else {
        if (a.check) CKTLU_LEVEL(double, true); else CKTLU_LEVEL(double, false);
    }
#undef CKTLU_LEVEL
    return (int)hipGetLastError();
}

// ----------------------------------------------------------------- solves
// y holds NR doubles per row and instance (NR: the right-hand sides padded to 1, 2, 4 or 8):
// y[(inst*n + i)*NR + r].
// One row of a triangular solve, by one wavefront: its record, then its entries
// {column, value position}, then the values and the y rows they multiply.
// sum over the row entries [beg, end) of value * y(column), per right-hand side, over the
// wavefront (two entries in flight per lane), totals in every lane
template <typename T, int NR>
__device__ __forceinline__ void row_pull(const int2 *rjs, const T *Fx, const double *y, int beg, int end, int lane,
                                         double (&acc)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    for (int q0 = beg; q0 < end; q0 += 2 * WAVE) {
        int2 e[2];
#pragma unroll
        for (int u = 0; u < 2; u++) e[u] = q0 + u * WAVE + lane < end ? rjs[q0 + u * WAVE + lane] : make_int2(-1, 0);
        double l[2];
#pragma unroll
        for (int u = 0; u < 2; u++) l[u] = e[u].x >= 0 ? (double)Fx[e[u].y] : 0.0;
#pragma unroll
        for (int u = 0; u < 2; u++)
            if (e[u].x >= 0) {
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] += l[u] * y[(size_t)e[u].x * NR + r];
            }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = wave_sum(acc[r]);
}

template <typename T, int NR, bool UPPER>
__device__ __forceinline__ void solve_row_rec(const SolveArgs &a, int inst, int4 rec, int lane) {
    const int2 *rjs = reinterpret_cast<const int2 *>(UPPER ? a.Urjs : a.Lrjs);
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    double *y = a.y + (size_t)inst * a.n * NR;
    const int i = rec.x;
    const double diag = UPPER ? (double)Fx[rec.w] : 1.0;
    const double yi = lane < NR ? y[(size_t)i * NR + lane] : 0.0;
    double acc[NR];
    row_pull<T, NR>(rjs, Fx, y, rec.y, rec.z, lane, acc);
    double mine = acc[0];
#pragma unroll
    for (int r = 1; r < NR; r++)
        if (lane == r) mine = acc[r];
    if (lane < NR) {
        double v = yi - mine;
        if (UPPER) v = v / diag;
        y[(size_t)i * NR + lane] = v;
    }
}

template <typename T, int NR, bool UPPER>
__device__ __forceinline__ void solve_row(const SolveArgs &a, int inst, int pos, int lane) {
    solve_row_rec<T, NR, UPPER>(a, inst, reinterpret_cast<const int4 *>(UPPER ? a.urec : a.lrec)[pos], lane);
}

// One level: one wavefront per (row, instance).
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(WG) void trisolve_level_kernel(SolveArgs a, int lbeg, int lend) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t t = (int64_t)lbeg * a.batch + (int64_t)blockIdx.x * WAVES + wv;
    if (t >= (int64_t)lend * a.batch) return;
    const int inst = (int)(t % a.batch);
    if (a.skip && a.skip[inst] != -1) return;
    solve_row<T, NR, UPPER>(a, inst, (int)(t / a.batch), lane);
}

// One level of long rows: a workgroup of kSolveRowWG threads per (row, instance);
// thread t takes entries t, t + kSolveRowWG, ... (four in flight), the wavefront
// sums are added in wavefront order.
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(kSolveRowWG) void trisolve_rowwg_kernel(SolveArgs a, int lbeg, int lend) {
    constexpr int NW = kSolveRowWG / WAVE;
    __shared__ double part[NW][NR];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int64_t t = (int64_t)lbeg * a.batch + blockIdx.x;
    const int inst = (int)(t % a.batch);
    if (a.skip && a.skip[inst] != -1) return;            // the whole workgroup
    const int4 rec = reinterpret_cast<const int4 *>(UPPER ? a.urec : a.lrec)[t / a.batch];
    const int2 *rjs = reinterpret_cast<const int2 *>(UPPER ? a.Urjs : a.Lrjs);
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    double *y = a.y + (size_t)inst * a.n * NR;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    for (int q0 = rec.y; q0 < rec.z; q0 += 4 * kSolveRowWG) {
        int2 e[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int q = q0 + u * kSolveRowWG + tid;
            e[u] = q < rec.z ? rjs[q] : make_int2(-1, 0);
        }
        double l[4];
#pragma unroll
        for (int u = 0; u < 4; u++) l[u] = e[u].x >= 0 ? (double)Fx[e[u].y] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (e[u].x >= 0) {
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] += l[u] * y[(size_t)e[u].x * NR + r];
            }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = wave_sum(acc[r]);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < NR; r++) part[wv][r] = acc[r];
    }
    __syncthreads();
    if (wv == 0 && lane < NR) {
        double sum = part[0][lane];
#pragma unroll
        for (int w = 1; w < NW; w++) sum += part[w][lane];
        const int i = rec.x;
        double v = y[(size_t)i * NR + lane] - sum;
        if (UPPER) v = v / (double)Fx[rec.w];
        y[(size_t)i * NR + lane] = v;
    }
}

// ------------------------------------------------------------ supernodal solves
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The dense triangle of supernode [s0, s0 + w) in one wavefront, lane c holding row s0 + c with
// t = its right-hand sides minus the pulled sums: L: y_c -= L(c, c') y_c' for c' < c in
// ascending c' (unit diagonal); U: x_c = t_c * (1 / U(c, c)) in descending c (the reciprocals
// formed by all lanes at once before the chain, not a division per step and right-hand side),
// then t_c'' -= U(c'', c) x_c for c'' < c.  The triangle's entries come from the factor columns
// (sn_cb: offset of the supernode's first row in each column); the results go to y.
// elem(c, r): the diagonal block's entry in column c, row r (both local to the supernode)
template <typename T, int NR, bool UPPER, typename Elem>
__device__ __forceinline__ void sn_triangle(Elem elem, double *y, int s0, int w, double (&t)[NR], int lane) {
    if (!UPPER) {
        for (int c0 = 0; c0 < w; c0 += 8) {
            double lv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int c = c0 + u;
                lv[u] = (c < w && lane > c && lane < w) ? elem(c, lane) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int c = c0 + u;
                if (c < w) {
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        const double uc = readlane_f64(t[r], c);
                        if (lane > c) t[r] = fma(-lv[u], uc, t[r]);
                    }
                }
            }
        }
    } else {
        const double rdiag = lane < w ? 1.0 / elem(lane, lane) : 1.0;
        for (int c0 = w - 1; c0 >= 0; c0 -= 8) {
            double lv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int c = c0 - u;
                lv[u] = (c >= 0 && lane < c) ? elem(c, lane) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int c = c0 - u;
                if (c >= 0) {
                    const double rd = readlane_f64(rdiag, c);
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        const double xc = readlane_f64(t[r], c) * rd;
                        if (lane == c) t[r] = xc;
                        if (lane < c) t[r] = fma(-lv[u], xc, t[r]);
                    }
                }
            }
        }
    }
    if (lane < w) {
#pragma unroll
        for (int r = 0; r < NR; r++) y[(size_t)(s0 + lane) * NR + r] = t[r];
    }
}

// One level of the supernodal L (U) solve.  Singletons with a short row get sixteen lanes per
// (row, instance).  Other supernodes of at most kSnSmallW rows with a short pull get a
// wavefront per (supernode, instance): a singleton as in the row kernel; a wider one pulls all
// its rows at once (a group of lanes per row) and solves its triangle.  Every other supernode
// [s0, s0 + w) pulls by runs: a run is a column j and the rows of the supernode present in it,
// consecutive rows at consecutive positions of j's storage, so lane c (row s0 + c) reads its
// entry of the run next to its neighbours' and y_j once per run instead of once per entry.  The
// supernode's runs are cut into P units, a workgroup of sixteen wavefronts per (unit,
// instance); wavefront v takes the unit's runs v, v + 16, ... (eight in flight, their solution
// rows loaded by one instruction and broadcast) and its lanes add the products to their rows'
// sums in that order; the sixteen wavefronts' sums meet in LDS
// by a fixed tree.  With P = 1 the workgroup then solves the triangle; with P > 1 each unit
// stores its row sums in its scratch block and counts its arrival, and the last unit to arrive
// adds the P blocks (the even units and the odd units in ascending order, by two halves of its
// threads, then the two halves: the same sums whichever unit is last) and solves the triangle.
// Every unit loads the diagonal block into LDS while it pulls.  sw holds, per position of the
// level sequence, the supernode's first column and width (int2).
constexpr int kSnSolveWG = 1024;                     // threads of a supernodal solve workgroup
constexpr int kSolveWholeBatch = 8;
constexpr int kSnSolveWaves = kSnSolveWG / WAVE;
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(kSnSolveWG) void sn_solve_kernel(SolveArgs a, const int *sw, const int *units,
                                                              const int *urange, const int *runs, int sbeg, int stiny,
                                                              int smid, int ubeg, int *cnt, int whole) {
    __shared__ double wsum[8][8][WAVE];                  // the wavefronts' sums, [wavefront][rhs][row]
    __shared__ double red[2][512];
    __shared__ double tri[64][65];                       // a unit's diagonal block, column-major
    __shared__ int arrived;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t ntiny = (int64_t)(stiny - sbeg) * a.batch;
    const int64_t ntb = (ntiny + kSnSolveWG / 16 - 1) / (kSnSolveWG / 16);
    const int64_t nsingle = (int64_t)(smid - stiny) * a.batch;
    const int64_t nsw = ntb + (nsingle + kSnSolveWaves - 1) / kSnSolveWaves;
    const int *rp = UPPER ? a.Urp : a.Lrp;
    const int2 *rjs = reinterpret_cast<const int2 *>(UPPER ? a.Urjs : a.Lrjs);
    if ((int64_t)blockIdx.x < ntb) {
        // a short singleton row on sixteen lanes: two entries per lane in flight, the sums
        // reduced over the sixteen lanes
        const int64_t gid = (int64_t)blockIdx.x * (kSnSolveWG / 16) + threadIdx.x / 16;
        if (gid >= ntiny) return;
        const int inst = (int)(gid % a.batch);
        if (a.skip && a.skip[inst] != -1) return;
        const int i = sw[2 * (sbeg + (int)(gid / a.batch))];
        const int l16 = lane & 15;
        const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
        double *y = a.y + (size_t)inst * a.n * NR;
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] = 0.0;
        const int beg = rp[i], end = rp[i + 1];
        for (int q0 = beg; q0 < end; q0 += 32) {
            int2 e[2];
#pragma unroll
            for (int u = 0; u < 2; u++) e[u] = q0 + 16 * u + l16 < end ? rjs[q0 + 16 * u + l16] : make_int2(-1, 0);
            double l[2];
#pragma unroll
            for (int u = 0; u < 2; u++) l[u] = e[u].x >= 0 ? (double)Fx[e[u].y] : 0.0;
#pragma unroll
            for (int u = 0; u < 2; u++)
                if (e[u].x >= 0) {
#pragma unroll
                    for (int r = 0; r < NR; r++) acc[r] += l[u] * y[(size_t)e[u].x * NR + r];
                }
        }
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 16);
        double mine = acc[0];
#pragma unroll
        for (int r = 1; r < NR; r++)
            if (l16 == r) mine = acc[r];
        if (l16 < NR) {
            double v = y[(size_t)i * NR + l16] - mine;
            if (UPPER) v = v / (double)Fx[a.sn_cb[i]];
            y[(size_t)i * NR + l16] = v;
        }
        return;
    }
    if ((int64_t)blockIdx.x < nsw) {
        const int64_t wid = ((int64_t)blockIdx.x - ntb) * kSnSolveWaves + wv;
        if (wid >= nsingle) return;
        const int inst = (int)(wid % a.batch);
        if (a.skip && a.skip[inst] != -1) return;
        const int2 rec = reinterpret_cast<const int2 *>(sw)[stiny + (int)(wid / a.batch)];
        const int s0 = rec.x, w = rec.y;
        if (w == 1) {
            solve_row_rec<T, NR, UPPER>(a, inst, make_int4(s0, rp[s0], rp[s0 + 1], a.sn_cb[s0]), lane);
            return;
        }
        const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
        double *y = a.y + (size_t)inst * a.n * NR;
        // the rows pull at the same time: G = 64 / 2^ceil(log2 w) lanes per row (at least 4),
        // two entries per lane in flight, the sums reduced over the G lanes
        const int lg = 32 - __builtin_clz((unsigned)(w - 1));   // w <= 2^lg
        const int G = WAVE >> lg, c = lane / G, lq = lane % G;
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] = 0.0;
        if (c < w) {
            const int i = s0 + c;
            const int beg = UPPER ? rp[i] + (w - 1 - c) : rp[i], end = UPPER ? rp[i + 1] : rp[i + 1] - c;
            for (int q0 = beg; q0 < end; q0 += 2 * G) {
                int2 e[2];
#pragma unroll
                for (int u = 0; u < 2; u++) e[u] = q0 + u * G + lq < end ? rjs[q0 + u * G + lq] : make_int2(-1, 0);
                double l[2];
#pragma unroll
                for (int u = 0; u < 2; u++) l[u] = e[u].x >= 0 ? (double)Fx[e[u].y] : 0.0;
#pragma unroll
                for (int u = 0; u < 2; u++)
                    if (e[u].x >= 0) {
#pragma unroll
                        for (int r = 0; r < NR; r++) acc[r] += l[u] * y[(size_t)e[u].x * NR + r];
                    }
            }
        }
        for (int off = G >> 1; off > 0; off >>= 1) {
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] += __shfl_xor(acc[r], off);
        }
        // lane c takes row c's sums from the first lane of its group
        double t[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double sr = __shfl(acc[r], (lane < w ? lane : 0) * G);
            t[r] = lane < w ? y[(size_t)(s0 + lane) * NR + r] - sr : 0.0;
        }
        const int *cb = a.sn_cb + s0;
        sn_triangle<T, NR, UPPER>([=](int cc, int r) { return (double)Fx[cb[cc] + r]; }, y, s0, w, t, lane);
        return;
    }
    const int64_t pu = (int64_t)blockIdx.x - nsw;
    const int inst = (int)(pu % a.batch);
    if (a.skip && a.skip[inst] != -1) return;            // the whole workgroup
    const int ui = ubeg + (int)(pu / a.batch);
    int4 un = reinterpret_cast<const int4 *>(units)[ui];
    int4 ur = reinterpret_cast<const int4 *>(urange)[ui];   // runs [x, y) of supernode [z, z + w)
    if (whole && un.z > 1) {
        // one workgroup per supernode: the first unit takes every unit's runs (they are
        // consecutive), the others leave
        if (un.y > 0) return;
        ur.y = reinterpret_cast<const int4 *>(urange)[ui + un.z - 1].y;
        un.z = 1;
    }
    const int s0 = ur.z, w = ur.w;
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    double *y = a.y + (size_t)inst * a.n * NR;
    // the diagonal block, loaded now and stored to LDS after the pull (up to four per thread)
    double dv[4];
    {
        const int *cb = a.sn_cb + s0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = threadIdx.x + u * kSnSolveWG;
            dv[u] = e < w * w ? (double)Fx[cb[e / w] + e % w] : 0.0;
        }
    }
    // eight runs per round: lanes 0-7 load the runs, lane l then the solution row entry
    // (l % 8) of run l / 8's column, broadcast by readlane
    const int4 *rr = reinterpret_cast<const int4 *>(runs);
    double sum[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) sum[r] = 0.0;
    for (int q0 = ur.x + wv; q0 < ur.y; q0 += 8 * kSnSolveWaves) {   // uniform per wavefront
        const int qa = q0 + (lane & 7) * kSnSolveWaves;
        const int4 gl = lane < 8 && qa < ur.y ? rr[qa] : make_int4(0, 0, 0, 0);
        const int jl = __shfl(gl.x, lane >> 3), nl = __shfl(gl.w, lane >> 3);
        const double yl = nl > 0 && (lane & 7) < NR ? y[(size_t)jl * NR + (lane & 7)] : 0.0;
        double lv[8];
        bool on[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = lane - __builtin_amdgcn_readlane(gl.z, u);
            on[u] = c >= 0 && c < __builtin_amdgcn_readlane(gl.w, u);
            lv[u] = on[u] ? (double)Fx[__builtin_amdgcn_readlane(gl.y, u) + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const double yv = readlane_f64(yl, 8 * u + r);
                if (on[u]) sum[r] = fma(lv[u], yv, sum[r]);
            }
        }
    }
    // the sixteen wavefronts' sums: v + 8 into v, then v + 4 into v, ... (a fixed tree)
    for (int h = kSnSolveWaves / 2; h >= 1; h >>= 1) {
        if (wv >= h && wv < 2 * h) {
#pragma unroll
            for (int r = 0; r < NR; r++) wsum[wv - h][r][lane] = sum[r];
        }
        __syncthreads();
        if (wv < h) {
#pragma unroll
            for (int r = 0; r < NR; r++) sum[r] += wsum[wv][r][lane];
        }
        __syncthreads();
    }
    if (un.z > 1) {
        double *blk = a.sn_part + ((size_t)un.w * a.batch + inst) * 512;
        const size_t bstride = (size_t)a.batch * 512;
        if (wv == 0 && lane < w) {
#pragma unroll
            for (int r = 0; r < NR; r++) blk[un.y * bstride + lane * 8 + r] = sum[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        int *ctr = cnt + (size_t)un.x * a.batch + inst;
        if (threadIdx.x == 0) {
            const int prev = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            arrived = prev == un.z - 1;
            if (arrived) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!arrived) return;                            // not the last unit of this supernode
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        {
            const int v = threadIdx.x & 511, h = threadIdx.x >> 9, c = v >> 3, r = v & 7;
            double acc = 0.0;
            if (c < w && r < NR) {
                int p = h;
                for (; p + 6 < un.z; p += 8) {         // four loads in flight
                    const double x0 = blk[(size_t)p * bstride + v], x1 = blk[(size_t)(p + 2) * bstride + v];
                    const double x2 = blk[(size_t)(p + 4) * bstride + v], x3 = blk[(size_t)(p + 6) * bstride + v];
                    acc = (((acc + x0) + x1) + x2) + x3;
                }
                for (; p < un.z; p += 2) acc += blk[(size_t)p * bstride + v];
            }
            red[h][v] = acc;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int e = threadIdx.x + u * kSnSolveWG;
        if (e < w * w) tri[e / w][e % w] = dv[u];
    }
    __syncthreads();
    if (wv != 0) return;
    if (un.z > 1 && lane < w) {
#pragma unroll
        for (int r = 0; r < NR; r++) sum[r] = red[0][lane * 8 + r] + red[1][lane * 8 + r];
    }
    double t[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) t[r] = lane < w ? y[(size_t)(s0 + lane) * NR + r] - sum[r] : 0.0;
    sn_triangle<T, NR, UPPER>([&](int cc, int r) { return tri[cc][r]; }, y, s0, w, t, lane);
}

template <bool UPPER>
static int launch_sn_solve_impl(const SolveArgs &a, const int *sw, const int *units, const int *urange,
                                const int *runs, int sbeg, int stiny, int smid, int ubeg, int uend, int *cnt,
                                void *stream) {
    // a batch of kSolveWholeBatch instances or more fills the device with one workgroup per
    // supernode and instance: split units would only add combines
    const int whole = a.batch >= kSolveWholeBatch ? 1 : 0;
    const int64_t ntb = ((int64_t)(stiny - sbeg) * a.batch + kSnSolveWG / 16 - 1) / (kSnSolveWG / 16);
    const int64_t nsw = ntb + ((int64_t)(smid - stiny) * a.batch + kSnSolveWaves - 1) / kSnSolveWaves;
    const int64_t units_n = nsw + (int64_t)(uend - ubeg) * a.batch;
    if (units_n == 0) return 0;
    const dim3 grid((unsigned)units_n);
    hipStream_t st = (hipStream_t)stream;
#define CKTLU_SNS_CASE(NRV)                                                                             \
    case NRV:                                                                                           \
        if (a.fp32)                                                                                     \
            hipLaunchKernelGGL((sn_solve_kernel<float, NRV, UPPER>), grid, dim3(kSnSolveWG), 0, st, a, sw, units, \
                               urange, runs, sbeg, stiny, smid, ubeg, cnt, whole);                      \
        else                                                                                            \
            hipLaunchKernelGGL((sn_solve_kernel<double, NRV, UPPER>), grid, dim3(kSnSolveWG), 0, st, a, sw, units, \
                               urange, runs, sbeg, stiny, smid, ubeg, cnt, whole);                      \
        break;
    switch (a.nrhs) {
        CKTLU_SNS_CASE(1)
        CKTLU_SNS_CASE(2)
        CKTLU_SNS_CASE(4)
        CKTLU_SNS_CASE(8)
        default: return (int)hipErrorInvalidValue;
    }
#undef CKTLU_SNS_CASE
    return (int)hipGetLastError();
}

int launch_sn_lsolve(const SolveArgs &a, const int *sw, const int *units, const int *urange, const int *runs, int sbeg,
                     int stiny, int smid, int ubeg, int uend, int *cnt, void *stream) {
    return launch_sn_solve_impl<false>(a, sw, units, urange, runs, sbeg, stiny, smid, ubeg, uend, cnt, stream);
}
int launch_sn_usolve(const SolveArgs &a, const int *sw, const int *units, const int *urange, const int *runs, int sbeg,
                     int stiny, int smid, int ubeg, int uend, int *cnt, void *stream) {
    return launch_sn_solve_impl<true>(a, sw, units, urange, runs, sbeg, stiny, smid, ubeg, uend, cnt, stream);
}

// A run of narrow levels [l0, l1): one workgroup per instance takes the rows of a
// level round-robin over its wavefronts, then waits at a barrier before the next
// level (the barrier orders the workgroup's global stores before its later loads).
constexpr int kChainWG = 1024;
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(kChainWG) void trisolve_chain_kernel(SolveArgs a, const int *lvptr, int l0, int l1) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int inst = blockIdx.x;
    if (a.skip && a.skip[inst] != -1) return;          // the whole workgroup
    int beg = lvptr[l0];
    for (int l = l0; l < l1; l++) {
        const int end = lvptr[l + 1];
        for (int p = beg + wv; p < end; p += kChainWG / WAVE) solve_row<T, NR, UPPER>(a, inst, p, lane);
        beg = end;
        __syncthreads();
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

template <bool UPPER>
static int launch_solve_chain_impl(const SolveArgs &a, const int *lvptr, int l0, int l1, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)a.batch);
#define CKTLU_CHAIN_CASE(NRV)                                                                          \
    case NRV:                                                                                          \
        if (a.fp32)                                                                                    \
            hipLaunchKernelGGL((trisolve_chain_kernel<float, NRV, UPPER>), grid, dim3(kChainWG), 0, st, a, lvptr, l0, l1); \
        else                                                                                           \
            hipLaunchKernelGGL((trisolve_chain_kernel<double, NRV, UPPER>), grid, dim3(kChainWG), 0, st, a, lvptr, l0, l1); \
        break;
    switch (a.nrhs) {
        CKTLU_CHAIN_CASE(1)
        CKTLU_CHAIN_CASE(2)
        CKTLU_CHAIN_CASE(4)
        CKTLU_CHAIN_CASE(8)
        default: return (int)hipErrorInvalidValue;
    }
#undef CKTLU_CHAIN_CASE
    return (int)hipGetLastError();
}

template <bool UPPER>
static int launch_solve_rowwg_impl(const SolveArgs &a, int lbeg, int lend, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)((int64_t)(lend - lbeg) * a.batch));
#define CKTLU_ROWWG_CASE(NRV)                                                                          \
    case NRV:                                                                                          \
        if (a.fp32)                                                                                    \
            hipLaunchKernelGGL((trisolve_rowwg_kernel<float, NRV, UPPER>), grid, dim3(kSolveRowWG), 0, st, a, lbeg, lend); \
        else                                                                                           \
            hipLaunchKernelGGL((trisolve_rowwg_kernel<double, NRV, UPPER>), grid, dim3(kSolveRowWG), 0, st, a, lbeg, lend); \
        break;
    switch (a.nrhs) {
        CKTLU_ROWWG_CASE(1)
        CKTLU_ROWWG_CASE(2)
        CKTLU_ROWWG_CASE(4)
        CKTLU_ROWWG_CASE(8)
        default: return (int)hipErrorInvalidValue;
    }
#undef CKTLU_ROWWG_CASE
    return (int)hipGetLastError();
}

int launch_lsolve_level_wg(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_rowwg_impl<false>(a, lbeg, lend, stream);
}
int launch_usolve_level_wg(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_rowwg_impl<true>(a, lbeg, lend, stream);
}

int launch_lsolve_chain(const SolveArgs &a, const int *lvptr, int l0, int l1, void *stream) {
    return launch_solve_chain_impl<false>(a, lvptr, l0, l1, stream);
}
int launch_usolve_chain(const SolveArgs &a, const int *lvptr, int l0, int l1, void *stream) {
    return launch_solve_chain_impl<true>(a, lvptr, l0, l1, stream);
}

int launch_lsolve_level(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_level_impl<false>(a, lbeg, lend, stream);
}
int launch_usolve_level(const SolveArgs &a, int lbeg, int lend, void *stream) {
    return launch_solve_level_impl<true>(a, lbeg, lend, stream);
}

// --------------------------------------------------------------- helpers
// fills the solve slots [0, solve_slots(nrhs)) of each row; slots past nrhs get zeros
// scale (may be null): per solve position, the static row scaling of its user row
__global__ void gather_rhs_kernel(int n, int nrhs, int nslots, int batch, const double *b, int64_t ldb,
                                  const int *perm, double *y, const double *scale) {
    const int64_t total = (int64_t)n * nslots * batch;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t % nslots);
        const int64_t ik = t / nslots;
        const int k = (int)(ik % n);
        const int64_t i = ik / n;
        const double v = r < nrhs ? b[(i * nrhs + r) * ldb + perm[k]] : 0.0;
        y[ik * nslots + r] = scale ? v * scale[k] : v;
    }
}

// x[(i*nrhs + r)*ldx + j] (+)= z[(i*n + inv[j])*nslots + r]: a thread per (user index j,
// instance), so that the writes of each right-hand side are consecutive in j; inv: user index ->
// solve position.  scale (may be null): per solve position, the static column scaling of its
// user column
__global__ void scatter_sol_kernel(int n, int nrhs, int nslots, int batch, const double *z, const int *inv,
                                   double *x, int64_t ldx, int accumulate, const int *skip, const double *scale) {
    const int64_t total = (int64_t)n * batch;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t % n);
        const int64_t i = t / n;
        if (skip && skip[i] != -1) continue;
        const int k = inv[j];
        const double *zr = z + ((size_t)i * n + k) * nslots;
        for (int r = 0; r < nrhs; r++) {
            double *dst = x + (i * nrhs + r) * ldx + j;
            const double v = scale ? zr[r] * scale[k] : zr[r];
            *dst = accumulate ? *dst + v : v;
        }
    }
}

static inline int grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

int launch_gather_rhs(int n, int nrhs, int batch, const double *b, int64_t ldb, const int *perm,
                      double *y, void *stream, const double *scale) {
    const int ns = solve_slots(nrhs);
    hipLaunchKernelGGL(gather_rhs_kernel, dim3(grid_for((int64_t)n * ns * batch, 256)), dim3(256), 0,
                       (hipStream_t)stream, n, nrhs, ns, batch, b, ldb, perm, y, scale);
    return (int)hipGetLastError();
}

int launch_scatter_sol(int n, int nrhs, int batch, const double *z, const int *inv, double *x,
                       int64_t ldx, int accumulate, const int *skip, void *stream, const double *scale) {
    hipLaunchKernelGGL(scatter_sol_kernel, dim3(grid_for((int64_t)n * batch, 256)), dim3(256), 0,
                       (hipStream_t)stream, n, nrhs, solve_slots(nrhs), batch, z, inv, x, ldx, accumulate, skip,
                       scale);
    return (int)hipGetLastError();
}

// non-negative doubles order like their bit patterns as signed 64-bit integers
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

// maximum of non-negative values that keeps a NaN (whose bit pattern orders above +inf)
__device__ __forceinline__ double max_keep_nan(double m, double v) { return (v != v || v > m) ? v : m; }
__device__ __forceinline__ double wave_max_keep_nan(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max_keep_nan(v, __shfl_xor(v, off));
    return v;
}

// r = b - A x for up to eight right-hand sides [r0, r0 + nr) of one instance: every thread takes
// rows i (grid stride) and reads row i of A once for all of them, keeps running maxima of
// |r|, |x|, |b| and the wavefront adds them to norms with one atomic each.
template <int NRM>
__device__ __forceinline__ void residual_rows(int n, int nr, const int *Acp, const int *Acj, const int *Acsrc,
                                              const double *Aval, const double *x, int64_t ldx, const double *b,
                                              int64_t ldb, double *r, int64_t ldr, double *norms, int64_t i0,
                                              int64_t stride) {
    constexpr int E = NRM == 1 ? 4 : 2;                 // entries whose loads are in flight together
    double mr[8], mx[8], mb[8];
#pragma unroll
    for (int u = 0; u < 8; u++) mr[u] = mx[u] = mb[u] = 0.0;
    for (int64_t i = i0; i < n; i += stride) {
        double acc[NRM];
#pragma unroll
        for (int u = 0; u < NRM; u++) acc[u] = u < nr ? b[u * ldb + i] : 0.0;
#pragma unroll
        for (int u = 0; u < NRM; u++) mb[u] = max_keep_nan(mb[u], fabs(acc[u]));
        const int pe = Acp[i + 1];
        for (int p0 = Acp[i]; p0 < pe; p0 += E) {       // E entries' loads in flight, then in order
            int src[E], j[E];
#pragma unroll
            for (int q = 0; q < E; q++) {
                src[q] = p0 + q < pe ? Acsrc[p0 + q] : 0;
                j[q] = p0 + q < pe ? Acj[p0 + q] : 0;
            }
            double v[E], xv[E][NRM];
#pragma unroll
            for (int q = 0; q < E; q++) {
                v[q] = p0 + q < pe ? Aval[src[q]] : 0.0;
#pragma unroll
                for (int u = 0; u < NRM; u++) xv[q][u] = (p0 + q < pe && u < nr) ? x[u * ldx + j[q]] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < E; q++)
                if (p0 + q < pe) {
#pragma unroll
                    for (int u = 0; u < NRM; u++)
                        if (u < nr) acc[u] -= v[q] * xv[q][u];
                }
        }
#pragma unroll
        for (int u = 0; u < NRM; u++)
            if (u < nr) {
                r[u * ldr + i] = acc[u];
                mr[u] = max_keep_nan(mr[u], fabs(acc[u]));
                mx[u] = max_keep_nan(mx[u], fabs(x[u * ldx + i]));
            }
    }
    // maxima over the workgroup (four wavefronts), then one atomic per norm and workgroup: the
    // norms share a cache line, where atomics serialize
    __shared__ double wmax[4][24];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < NRM; u++) {
        const double a0 = wave_max_keep_nan(mr[u]), a1 = wave_max_keep_nan(mx[u]), a2 = wave_max_keep_nan(mb[u]);
        if (lane == 0) {
            wmax[wv][3 * u + 0] = a0;
            wmax[wv][3 * u + 1] = a1;
            wmax[wv][3 * u + 2] = a2;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 3 * nr) {
        double m = wmax[0][threadIdx.x];
        for (int q = 1; q < 4; q++) m = max_keep_nan(m, wmax[q][threadIdx.x]);
        atomic_max_nonneg(&norms[threadIdx.x], m);
    }
    __syncthreads();
}

template <int NRM>
__global__ __launch_bounds__(256) void residual_kernel(int n, int nrhs, const int *Acp, const int *Acj,
                                                       const int *Acsrc, const double *Aval, const double *x,
                                                       int64_t ldx, const double *b, int64_t ldb, double *r,
                                                       int64_t ldr, double *norms, const int *skip) {
    if (skip && *skip != -1) return;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int r0 = 0; r0 < nrhs; r0 += 8)
        residual_rows<NRM>(n, min(8, nrhs - r0), Acp, Acj, Acsrc, Aval, x + r0 * ldx, ldx, b + r0 * ldb, ldb,
                      r + r0 * ldr, ldr, norms + 3 * r0, i0, stride);
}

int launch_residual(int n, int nrhs, const int *Acp, const int *Acj, const int *Acsrc,
                    const double *Aval, const double *x, int64_t ldx, const double *b, int64_t ldb,
                    double *r, int64_t ldr, double *norms, void *stream, const int *skip) {
    const int grid = std::min(grid_for(n, 256), 1024);   // a few rows per thread, few atomics
    if (nrhs == 1)
        hipLaunchKernelGGL(residual_kernel<1>, dim3(grid), dim3(256), 0, (hipStream_t)stream, n, nrhs,
                           Acp, Acj, Acsrc, Aval, x, ldx, b, ldb, r, ldr, norms, skip);
    else
        hipLaunchKernelGGL(residual_kernel<8>, dim3(grid), dim3(256), 0, (hipStream_t)stream, n, nrhs,
                           Acp, Acj, Acsrc, Aval, x, ldx, b, ldb, r, ldr, norms, skip);
    return (int)hipGetLastError();
}

// max over rows i (grid stride from i0) of sum |A(i, :)|, four entries' loads in flight; the
// workgroup's maximum goes to *out with one atomic (they serialize on one address)
__device__ __forceinline__ void anorm_rows(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out,
                                           int i0, int stride) {
    double m = 0.0;
    for (int i = i0; i < n; i += stride) {
        double s = 0.0;
        const int pe = Acp[i + 1];
        for (int p0 = Acp[i]; p0 < pe; p0 += 4) {
            int src[4];
#pragma unroll
            for (int q = 0; q < 4; q++) src[q] = p0 + q < pe ? Acsrc[p0 + q] : -1;
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; q++) v[q] = src[q] >= 0 ? fabs(Aval[src[q]]) : 0.0;
#pragma unroll
            for (int q = 0; q < 4; q++) s += v[q];
        }
        m = max_keep_nan(m, s);
    }
    __shared__ double wm[4];
    m = wave_max_keep_nan(m);
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = wm[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) w = max_keep_nan(w, wm[q]);
        atomic_max_nonneg(out, w);
    }
}

__global__ __launch_bounds__(256) void anorm_kernel(int n, const int *Acp, const int *Acsrc, const double *Aval,
                                                    double *out) {
    anorm_rows(n, Acp, Acsrc, Aval, out, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

int launch_anorm(int n, const int *Acp, const int *Acsrc, const double *Aval, double *out, void *stream) {
    hipLaunchKernelGGL(anorm_kernel, dim3(std::min(grid_for(n, 256), 1024)), dim3(256), 0, (hipStream_t)stream, n,
                       Acp, Acsrc, Aval, out);
    return (int)hipGetLastError();
}

// Batched refinement: instance i uses values Aval + i*nnzA and vectors at
// (i*nrhs + r)*n; skip[i] != -1 leaves an instance out.
// one instance per blockIdx.y
template <int NRM>
__global__ __launch_bounds__(256) void residual_batched_kernel(int n, int nrhs, int64_t nnzA, const int *Acp,
                                                               const int *Acj, const int *Acsrc, const double *Aval,
                                                               const double *x, const double *b, double *r,
                                                               double *norms, const int *skip) {
    const int inst = (int)blockIdx.y;
    if (skip[inst] != -1) return;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    const double *Av = Aval + (size_t)inst * nnzA;
    for (int r0 = 0; r0 < nrhs; r0 += 8) {
        const size_t o = ((size_t)inst * nrhs + r0) * n;
        residual_rows<NRM>(n, min(8, nrhs - r0), Acp, Acj, Acsrc, Av, x + o, n, b + o, n, r + o, n,
                      norms + ((size_t)inst * nrhs + r0) * 3, i0, stride);
    }
}

// one instance per blockIdx.y
__global__ __launch_bounds__(256) void anorm_batched_kernel(int n, int64_t nnzA, const int *Acp, const int *Acsrc,
                                                            const double *Aval, double *out) {
    const int inst = (int)blockIdx.y;
    anorm_rows(n, Acp, Acsrc, Aval + (size_t)inst * nnzA, &out[inst], blockIdx.x * blockDim.x + threadIdx.x,
               gridDim.x * blockDim.x);
}

// eta[i] = max over right-hand sides of |r| / (|A| |x| + |b|); an instance whose
// eta reaches tol leaves the refinement (skip = 1).
__global__ void ir_check_kernel(int batch, int nrhs, const double *norms, const double *anorm, double tol,
                                int *skip, double *eta) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += gridDim.x * blockDim.x) {
        if (skip[i] != -1) continue;
        double e = 0.0;
        for (int rr = 0; rr < nrhs; rr++) {
            const double *nm = norms + ((size_t)i * nrhs + rr) * 3;
            const double den = anorm[i] * nm[1] + nm[2];
            e = fmax(e, den > 0.0 ? nm[0] / den : 0.0);
        }
        eta[i] = e;
        if (e <= tol) skip[i] = 1;
    }
}

int launch_residual_batched(int n, int nrhs, int batch, int64_t nnzA, const int *Acp, const int *Acj,
                            const int *Acsrc, const double *Aval, const double *x, const double *b, double *r,
                            double *norms, const int *skip, void *stream) {
    if (batch <= 0 || n <= 0) return 0;
    const dim3 grid(std::min(grid_for(n, 256), 1024), (unsigned)batch);
    if (nrhs == 1)
        hipLaunchKernelGGL(residual_batched_kernel<1>, grid, dim3(256), 0, (hipStream_t)stream, n, nrhs, nnzA, Acp,
                           Acj, Acsrc, Aval, x, b, r, norms, skip);
    else
        hipLaunchKernelGGL(residual_batched_kernel<8>, grid, dim3(256), 0, (hipStream_t)stream, n, nrhs, nnzA, Acp,
                           Acj, Acsrc, Aval, x, b, r, norms, skip);
    return (int)hipGetLastError();
}

int launch_anorm_batched(int n, int batch, int64_t nnzA, const int *Acp, const int *Acsrc, const double *Aval,
                         double *out, void *stream) {
    if (batch <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(anorm_batched_kernel, dim3(grid_for(n, 256), (unsigned)batch), dim3(256), 0,
                       (hipStream_t)stream, n, nnzA, Acp, Acsrc, Aval, out);
    return (int)hipGetLastError();
}

int launch_ir_check(int batch, int nrhs, const double *norms, const double *anorm, double tol, int *skip,
                    double *eta, void *stream) {
    hipLaunchKernelGGL(ir_check_kernel, dim3(grid_for(batch, 256)), dim3(256), 0, (hipStream_t)stream, batch, nrhs,
                       norms, anorm, tol, skip, eta);
    return (int)hipGetLastError();
}

__global__ void copy_i32_kernel(const int *src, int *dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int launch_copy_i32(const int *src, int *dst, int64_t count, void *stream) {
    hipLaunchKernelGGL(copy_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, count);
    return (int)hipGetLastError();
}

__global__ void fill_f64_kernel(double *dst, int64_t count, double value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

int launch_fill_f64(double *dst, int64_t count, double value, void *stream) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, dst, count,
                       value);
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

// ------------------------------------------------------ allocation-free solve
// The work rows of cktlu_solve_noalloc.  Host code never hands this name to a kernel
// (on the host it is a stand-in, not a device address): noalloc_scratch looks up the
// array's address on the current device once and kernels receive that address.
static __device__ __align__(256) double scratch[(size_t)kNoAllocRows * YS];

int noalloc_scratch(double **out) {
    static std::mutex mu;
    static double *addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= 64) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return 0;
}

}  // namespace cktlu_dev
