// Dense trailing block of the factorization (gfx950).
//
// The last D columns of the factors are nearly dense: the paper's dense
// triangular block (Section V-A), whose order it picks from the fill density.
// After the sparse right-looking sweep over the first T = n - D columns, the
// trailing block S = A22 - L21 U12 (what the sweep left in those columns,
// rows >= T) is gathered into a dense column-major D x D matrix per instance and
// factored without pivoting by a blocked right-looking LU, panels of NB = 64:
//   dlu_diag   one workgroup factors the NB x NB diagonal block in LDS;
//   dlu_trsm   L21 = A21 U11^-1 (a thread per row) and U12 = L11^-1 A12 (a
//              wavefront per column);
//   dlu_gemm   A22 -= L21 U12 on the matrix cores: 64 x 64 output tiles, K = NB,
//              v_mfma_f64_16x16x4 (v_mfma_f32_16x16x4 for FP32 factors).
// dlu_check applies the pivot test of the sparse columns to every dense column
// c (x = L(:,c) u_cc are its values before division):
//   fail  <=>  u_cc not finite or zero, or max_{i>c} |x(i,c)| not finite, or
//              |u_cc| < eps * max_{i>c} |x(i,c)|.
// tail_scatter writes L and U back into the sparse factor storage (which the
// pivot-check fallback and the factor getters read).  The dense triangular
// solves run one launch per NB-row block: the launch for block b applies block
// b-1's solution to every row below it (the rectangle of the paper's trapezoid
// slices, Section V-A) and then solves block b (the triangle).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"

namespace cktlu_dev {

namespace {

constexpr int WAVE = 64;
constexpr int NB = kDenseBlock;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T *inst_S(const DenseArgs &a, int inst) {
    return reinterpret_cast<T *>(a.S) + (size_t)inst * a.D * a.D;
}

// the sparse sweep of this instance failed its pivot test: nothing to do here
__device__ __forceinline__ bool sweep_failed(const DenseArgs &a, int inst) {
    return a.ctrl[1 + inst] != 0 && a.ctrl[1 + a.batch + inst] < a.T;
}

// maximum that keeps a NaN
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// ------------------------------------------------------------- gather / scatter
// one wavefront per (tail column, instance)
template <typename T>
__global__ __launch_bounds__(256) void tail_gather_kernel(DenseArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= (int64_t)a.D * a.batch) return;
    const int inst = (int)(w % a.batch), c = (int)(w / a.batch);
    const int k = a.T + c;
    T *S = inst_S<T>(a, inst) + (size_t)c * a.D;
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[k];
    const int *rows = a.Fi + a.Dp[k];
    const int len = a.Dlen[k];
    for (int i = lane; i < a.D; i += WAVE) S[i] = T(0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < len; q += WAVE) {
        const int r = rows[q];
        if (r >= a.T) S[r - a.T] = Fx[q];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void tail_scatter_kernel(DenseArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= (int64_t)a.D * a.batch) return;
    const int inst = (int)(w % a.batch), c = (int)(w / a.batch);
    if (sweep_failed(a, inst)) return;
    const int k = a.T + c;
    const T *S = inst_S<T>(a, inst) + (size_t)c * a.D;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[k];
    const int *rows = a.Fi + a.Dp[k];
    const int len = a.Dlen[k];
    for (int q = lane; q < len; q += WAVE) {
        const int r = rows[q];
        if (r >= a.T) Fx[q] = S[r - a.T];
    }
    // columns before the first failing one are final
    if (lane == 0 && k < a.ctrl[1 + a.batch + inst]) a.done[(size_t)inst * a.n + k] = (int)a.epoch;
}

// ------------------------------------------------------------- blocked LU
// One workgroup per instance factors the diagonal block [p, p+nb) in LDS.
template <typename T>
__global__ __launch_bounds__(256) void dlu_diag_kernel(DenseArgs a, int p) {
    __shared__ T blk[NB][NB + 1];                     // blk[col][row]
    const int inst = blockIdx.x;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int nb = min(NB, a.D - p);
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += 256) {
        const int cc = e / nb, rr = e % nb;
        blk[cc][rr] = S[(size_t)(p + cc) * a.D + p + rr];
    }
    __syncthreads();
    for (int kk = 0; kk < nb; kk++) {
        const T piv = blk[kk][kk];
        for (int i = kk + 1 + tid; i < nb; i += 256) blk[kk][i] = blk[kk][i] / piv;
        __syncthreads();
        const int m = nb - kk - 1;
        for (int e = tid; e < m * m; e += 256) {
            const int cc = kk + 1 + e / m, rr = kk + 1 + e % m;
            blk[cc][rr] -= blk[kk][rr] * blk[cc][kk];
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int cc = e / nb, rr = e % nb;
        S[(size_t)(p + cc) * a.D + p + rr] = blk[cc][rr];
    }
}

// Panel [p, p+NB) with rows/columns below/right of it (only launched for full
// panels).  Workgroups [0, nrow_blocks) compute L21 = A21 U11^-1, a thread per
// row; the others U12 = L11^-1 A12, a wavefront per column.
template <typename T>
__global__ __launch_bounds__(256) void dlu_trsm_kernel(DenseArgs a, int p, int nrow_blocks) {
    __shared__ T blk[NB][NB + 1];                     // blk[col][row]: unit L11 below, U11 on and above
    const int inst = blockIdx.y;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) {
        const int cc = e / NB, rr = e % NB;
        blk[cc][rr] = S[(size_t)(p + cc) * a.D + p + rr];
    }
    __syncthreads();
    if ((int)blockIdx.x < nrow_blocks) {
        const int i = p + NB + blockIdx.x * 256 + tid;   // one row of A21
        if (i >= a.D) return;
        T l[NB];
#pragma unroll
        for (int m = 0; m < NB; m++) l[m] = S[(size_t)(p + m) * a.D + i];
        // row-vector solve l U11 = a, right-looking: independent updates per step
#pragma unroll
        for (int kk = 0; kk < NB; kk++) {
            l[kk] = l[kk] / blk[kk][kk];
#pragma unroll
            for (int m = kk + 1; m < NB; m++) l[m] -= l[kk] * blk[m][kk];
        }
#pragma unroll
        for (int m = 0; m < NB; m++) S[(size_t)(p + m) * a.D + i] = l[m];
        return;
    }
    const int lane = tid & (WAVE - 1);
    const int j = p + NB + (blockIdx.x - nrow_blocks) * 4 + tid / WAVE;
    if (j >= a.D) return;
    T *col = S + (size_t)j * a.D + p;                 // lane m holds row p + m
    T v = col[lane];
    for (int kk = 0; kk < NB; kk++) {
        const T u = __shfl(v, kk);
        if (lane > kk) v -= blk[kk][lane] * u;
    }
    col[lane] = v;
}

// A22 -= L21 U12 over the trailing block [p+NB, D)^2: a 64 x 64 output tile per
// workgroup, each wavefront a 32 x 32 quadrant of 2 x 2 MFMA 16 x 16 tiles.
// MFMA 16x16x4 operands: lane l holds A(l%16, l/16) and B(l/16, l%16).
template <typename T>
__global__ __launch_bounds__(256) void dlu_gemm_kernel(DenseArgs a, int p) {
    __shared__ T As[NB][64 + 1];                      // As[k][row]
    __shared__ T Bs[NB][64 + 1];                      // Bs[k][col]
    const int inst = blockIdx.z;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int base = p + NB;
    const int r0 = base + blockIdx.x * 64, c0 = base + blockIdx.y * 64;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * 64; e += 256) {
        const int kk = e / 64, rr = e % 64;
        As[kk][rr] = r0 + rr < a.D ? S[(size_t)(p + kk) * a.D + r0 + rr] : T(0);
        const int kb = e % NB, cc = e / NB;
        Bs[kb][cc] = c0 + cc < a.D ? S[(size_t)(c0 + cc) * a.D + p + kb] : T(0);
    }
    __syncthreads();
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int qr = wv >> 1, qc = wv & 1;
    const int li = lane & 15, lk = lane >> 4;
    if constexpr (sizeof(T) == 8) {
        d4 acc[2][2];
        for (int ti = 0; ti < 2; ti++)
            for (int tj = 0; tj < 2; tj++) acc[ti][tj] = d4{0, 0, 0, 0};
        for (int s = 0; s < NB / 4; s++) {
            const double a0 = As[4 * s + lk][32 * qr + li], a1 = As[4 * s + lk][32 * qr + 16 + li];
            const double b0 = Bs[4 * s + lk][32 * qc + li], b1 = Bs[4 * s + lk][32 * qc + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        // FP64 result: lane l, element q holds row 4q + l/16, column l%16
        for (int ti = 0; ti < 2; ti++)
            for (int tj = 0; tj < 2; tj++)
                for (int q = 0; q < 4; q++) {
                    const int row = r0 + 32 * qr + 16 * ti + 4 * q + lk;
                    const int col = c0 + 32 * qc + 16 * tj + li;
                    if (row < a.D && col < a.D) S[(size_t)col * a.D + row] -= acc[ti][tj][q];
                }
    } else {
        f4 acc[2][2];
        for (int ti = 0; ti < 2; ti++)
            for (int tj = 0; tj < 2; tj++) acc[ti][tj] = f4{0, 0, 0, 0};
        for (int s = 0; s < NB / 4; s++) {
            const float a0 = As[4 * s + lk][32 * qr + li], a1 = As[4 * s + lk][32 * qr + 16 + li];
            const float b0 = Bs[4 * s + lk][32 * qc + li], b1 = Bs[4 * s + lk][32 * qc + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        // FP32 result: lane l, element q holds row 4(l/16) + q, column l%16
        for (int ti = 0; ti < 2; ti++)
            for (int tj = 0; tj < 2; tj++)
                for (int q = 0; q < 4; q++) {
                    const int row = r0 + 32 * qr + 16 * ti + 4 * lk + q;
                    const int col = c0 + 32 * qc + 16 * tj + li;
                    if (row < a.D && col < a.D) S[(size_t)col * a.D + row] -= acc[ti][tj][q];
                }
    }
}

// Pivot test of every dense column: one wavefront per (column, instance).
template <typename T>
__global__ __launch_bounds__(256) void dlu_check_kernel(DenseArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= (int64_t)a.D * a.batch) return;
    const int inst = (int)(w % a.batch), c = (int)(w / a.batch);
    if (sweep_failed(a, inst)) return;
    const T *col = inst_S<T>(a, inst) + (size_t)c * a.D;
    double m = 0.0;
    for (int i = c + 1 + lane; i < a.D; i += WAVE) m = nanmax(m, fabs((double)col[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if (lane != 0) return;
    const double piv = (double)col[c];
    const double xmax = fabs(piv) * m;                // largest |value before division| below the pivot
    const int k = a.T + c;
    if (!isfinite(piv) || piv == 0.0 || !isfinite(xmax) || fabs(piv) < a.eps * xmax || k == a.force_fail_col) {
        atomicMin(&a.ctrl[1 + a.batch + inst], k);
        atomicExch(&a.ctrl[1 + inst], 1);
    }
}

// ------------------------------------------------------------- dense solves
// y rows T.. of each instance hold the partial solution (YS doubles per row).
// Lower, unit diagonal: launch b applies block b-1 to rows >= b*NB (a row per
// thread, 256-row chunks per workgroup); workgroup 0, which updated the rows of
// block b itself, then solves block b.
template <typename T, int NR>
__global__ __launch_bounds__(256) void dtrsv_lower_kernel(DenseArgs a, double *y, int b, const int *skip) {
    __shared__ double yb[NB][NR];
    __shared__ double ys[NB][NR];
    const int inst = blockIdx.y;
    if (skip && skip[inst] != -1) return;
    const T *S = inst_S<T>(a, inst);
    double *yt = y + ((size_t)inst * a.n + a.T) * YS;
    const int D = a.D, tid = threadIdx.x;
    if (b > 0) {
        const int pb = (b - 1) * NB;
        for (int e = tid; e < NB * NR; e += 256) yb[e / NR][e % NR] = yt[(size_t)(pb + e / NR) * YS + e % NR];
        __syncthreads();
        const int i = b * NB + blockIdx.x * 256 + tid;
        if (i < D) {
            double acc[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] = 0.0;
            for (int m = 0; m < NB; m++) {
                const double l = (double)S[(size_t)(pb + m) * D + i];
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] += l * yb[m][r];
            }
#pragma unroll
            for (int r = 0; r < NR; r++) yt[(size_t)i * YS + r] -= acc[r];
        }
        __syncthreads();
    }
    if (blockIdx.x != 0) return;
    const int p = b * NB, nb = min(NB, D - p);
    for (int e = tid; e < nb * NR; e += 256) ys[e / NR][e % NR] = yt[(size_t)(p + e / NR) * YS + e % NR];
    __syncthreads();
    for (int kk = 0; kk < nb; kk++) {
        const int r = tid % NR;
        for (int ii = kk + 1 + tid / NR; ii < nb; ii += 256 / NR)
            ys[ii][r] -= (double)S[(size_t)(p + kk) * D + p + ii] * ys[kk][r];
        __syncthreads();
    }
    for (int e = tid; e < nb * NR; e += 256) yt[(size_t)(p + e / NR) * YS + e % NR] = ys[e / NR][e % NR];
}

// Upper with its diagonal: launch b handles block blk = nblk-1-b: it applies
// block blk+1 to every row above it, then workgroup 0 solves block blk.
template <typename T, int NR>
__global__ __launch_bounds__(256) void dtrsv_upper_kernel(DenseArgs a, double *y, int b, const int *skip) {
    __shared__ double yb[NB][NR];
    __shared__ double ys[NB][NR];
    const int inst = blockIdx.y;
    if (skip && skip[inst] != -1) return;
    const T *S = inst_S<T>(a, inst);
    double *yt = y + ((size_t)inst * a.n + a.T) * YS;
    const int D = a.D, tid = threadIdx.x;
    const int nblk = (D + NB - 1) / NB;
    const int blk = nblk - 1 - b;
    const int p = blk * NB, nb = min(NB, D - p);
    if (b > 0) {
        const int pb = (blk + 1) * NB, nbb = min(NB, D - pb);
        for (int e = tid; e < nbb * NR; e += 256) yb[e / NR][e % NR] = yt[(size_t)(pb + e / NR) * YS + e % NR];
        __syncthreads();
        const int i = pb - 1 - (int)(blockIdx.x * 256 + tid);   // rows above block blk+1, bottom up
        if (i >= 0) {
            double acc[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] = 0.0;
            for (int m = 0; m < nbb; m++) {
                const double u = (double)S[(size_t)(pb + m) * D + i];
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] += u * yb[m][r];
            }
#pragma unroll
            for (int r = 0; r < NR; r++) yt[(size_t)i * YS + r] -= acc[r];
        }
        __syncthreads();
    }
    if (blockIdx.x != 0) return;
    for (int e = tid; e < nb * NR; e += 256) ys[e / NR][e % NR] = yt[(size_t)(p + e / NR) * YS + e % NR];
    __syncthreads();
    for (int kk = nb - 1; kk >= 0; kk--) {
        if (tid < NR) ys[kk][tid] = ys[kk][tid] / (double)S[(size_t)(p + kk) * D + p + kk];
        __syncthreads();
        const int r = tid % NR;
        for (int ii = tid / NR; ii < kk; ii += 256 / NR)
            ys[ii][r] -= (double)S[(size_t)(p + kk) * D + p + ii] * ys[kk][r];
        __syncthreads();
    }
    for (int e = tid; e < nb * NR; e += 256) yt[(size_t)(p + e / NR) * YS + e % NR] = ys[e / NR][e % NR];
}

template <typename T, int NR>
void dense_solve_impl(const DenseArgs &a, double *y, const int *skip, bool upper, hipStream_t st) {
    const int nblk = (a.D + NB - 1) / NB;
    for (int b = 0; b < nblk; b++) {
        // rows the launch updates: lower -> rows >= b*NB; upper -> rows above block nblk-b
        const int rows = b == 0 ? 1 : (upper ? (nblk - b) * NB : a.D - b * NB);
        const dim3 g((unsigned)((rows + 255) / 256), (unsigned)a.batch);
        if (upper) hipLaunchKernelGGL((dtrsv_upper_kernel<T, NR>), g, dim3(256), 0, st, a, y, b, skip);
        else hipLaunchKernelGGL((dtrsv_lower_kernel<T, NR>), g, dim3(256), 0, st, a, y, b, skip);
    }
}

inline dim3 wave_grid(int64_t waves) { return dim3((unsigned)((waves + 3) / 4)); }

}  // namespace

int launch_dense_gather(const DenseArgs &a, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.D <= 0) return 0;
    const dim3 gw = wave_grid((int64_t)a.D * a.batch);
    if (a.fp32) hipLaunchKernelGGL((tail_gather_kernel<float>), gw, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((tail_gather_kernel<double>), gw, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

int launch_dense_refactor(const DenseArgs &a, bool gather, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int D = a.D;
    if (D <= 0) return 0;
    const dim3 gw = wave_grid((int64_t)D * a.batch);
    if (gather) {
        const int e = launch_dense_gather(a, stream);
        if (e) return e;
    }
    for (int p = 0; p < D; p += NB) {
        const int nb = D - p < NB ? D - p : NB;
        const int rest = D - p - nb;
        if (a.fp32) hipLaunchKernelGGL((dlu_diag_kernel<float>), dim3(a.batch), dim3(256), 0, st, a, p);
        else hipLaunchKernelGGL((dlu_diag_kernel<double>), dim3(a.batch), dim3(256), 0, st, a, p);
        if (rest > 0) {   // nb == NB here
            const int nrb = (rest + 255) / 256, ncb = (rest + 3) / 4;
            const dim3 gt((unsigned)(nrb + ncb), (unsigned)a.batch);
            if (a.fp32) hipLaunchKernelGGL((dlu_trsm_kernel<float>), gt, dim3(256), 0, st, a, p, nrb);
            else hipLaunchKernelGGL((dlu_trsm_kernel<double>), gt, dim3(256), 0, st, a, p, nrb);
            const dim3 gg((unsigned)((rest + 63) / 64), (unsigned)((rest + 63) / 64), (unsigned)a.batch);
            if (a.fp32) hipLaunchKernelGGL((dlu_gemm_kernel<float>), gg, dim3(256), 0, st, a, p);
            else hipLaunchKernelGGL((dlu_gemm_kernel<double>), gg, dim3(256), 0, st, a, p);
        }
    }
    if (a.check) {
        if (a.fp32) hipLaunchKernelGGL((dlu_check_kernel<float>), gw, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((dlu_check_kernel<double>), gw, dim3(256), 0, st, a);
    }
    if (a.fp32) hipLaunchKernelGGL((tail_scatter_kernel<float>), gw, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((tail_scatter_kernel<double>), gw, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

int launch_dense_solve(const DenseArgs &a, double *y, int nrhs, const int *skip, bool upper, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.D <= 0) return 0;
#define CKTLU_DS(NRV)                                                      \
    case NRV:                                                              \
        if (a.fp32) dense_solve_impl<float, NRV>(a, y, skip, upper, st);  \
        else dense_solve_impl<double, NRV>(a, y, skip, upper, st);        \
        break;
    switch (nrhs) {
        CKTLU_DS(1)
        CKTLU_DS(2)
        CKTLU_DS(4)
        CKTLU_DS(8)
        default: return (int)hipErrorInvalidValue;
    }
#undef CKTLU_DS
    return (int)hipGetLastError();
}

}  // namespace cktlu_dev
