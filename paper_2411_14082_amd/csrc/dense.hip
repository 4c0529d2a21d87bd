// Dense trailing block of the factorization (gfx950).
//
// The last D columns of the factors are nearly dense: the paper's dense
// triangular block (Section V-A), whose order it picks from the fill density.
// After the sparse right-looking sweep over the first T = n - D columns, the
// trailing block S = A22 - L21 U12 (what the sweep left in those columns,
// rows >= T) is gathered into a dense column-major D x D matrix per instance and
// factored without pivoting by a blocked right-looking LU, panels of NB = 64:
//   dlu_panel  every workgroup factors the NB x NB diagonal block in registers
//              (one barrier per step), then computes its share of
//              L21 = A21 U11^-1 (four lanes per row) or U12 = L11^-1 A12 (a
//              wavefront per four columns);
//   dlu_gemm   A22 -= L21 U12 on the matrix cores: 128 x 128 output tiles,
//              K = NB in LDS-staged chunks, v_mfma_f64_16x16x4 (v_mfma_f32_16x16x4
//              for FP32 factors).
// dlu_check applies the pivot test of the sparse columns to every dense column
// c (x = L(:,c) u_cc are its values before division):
//   fail  <=>  u_cc not finite or zero, or max_{i>c} |x(i,c)| not finite, or
//              |u_cc| < eps * max_{i>c} |x(i,c)|.
// tail_scatter writes L and U back into the sparse factor storage (which the
// pivot-check fallback and the factor getters read).  The dense triangular
// solves run one launch per NB-row block: the launch for block b applies block
// b-1's solution to every row below it (the rectangle of the paper's trapezoid
// slices, Section V-A) and then one wavefront solves block b (the triangle).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

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
__device__ __forceinline__ double readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Factors the nb x nb diagonal block at (p, p) of S (padded to NB x NB with the
// identity) without pivoting, in the registers of the workgroup's four
// wavefronts: wavefront g holds rows 16g..16g+15, lane c column c.  Step kk
// publishes row kk through LDS (double-buffered, one barrier per step); the
// column-kk values come from lane kk by readlane.  L = x / u_kk is formed as
// x * (1 / u_kk).  On return blk[col][row] holds unit L below the diagonal and U
// on and above it, invd[k] = 1 / u_kk, and the workgroup is synchronised.
template <typename T>
__device__ void diag_factor(const T *S, int D, int p, int nb, T (*blk)[NB + 1], T *rowbuf, T *invd) {
    const int lane = threadIdx.x & (WAVE - 1), g = threadIdx.x / WAVE;
    T v[16];
#pragma unroll
    for (int e = 0; e < 16; e++) {
        const int r = 16 * g + e;
        v[e] = (lane < nb && r < nb) ? S[(size_t)(p + lane) * D + p + r] : (lane == r ? T(1) : T(0));
    }
#pragma unroll 1
    for (int kb = 0; kb < 4; kb++) {
#pragma unroll
        for (int e0 = 0; e0 < 16; e0++) {
            const int kk = 16 * kb + e0;
            T *rb = rowbuf + (kk & 1) * NB;
            if (g == kb) rb[lane] = v[e0];               // row kk: U(kk, c) for c >= kk
            __syncthreads();
            const T inv = T(1) / rb[kk];
            if (threadIdx.x == 0) invd[kk] = inv;
            // lanes c > kk subtract x * U(kk,c) / u_kk; lane kk keeps x / u_kk
            const T w = lane > kk ? rb[lane] * inv : (lane == kk ? -inv : T(0));
            const T keep = lane == kk ? T(0) : T(1);
            if (g >= kb) {
#pragma unroll
                for (int e = 0; e < 16; e++) {
                    if (16 * g + e > kk) {
                        const T x = readlane(v[e], kk);
                        v[e] = fma(-x, w, v[e] * keep);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; e++) blk[lane][16 * g + e] = v[e];
    __syncthreads();
}

// One panel [p, p+nb): every workgroup factors the diagonal block (workgroup 0
// writes it back); workgroups [1, 1+nrb) then compute L21 = A21 U11^-1 for 64
// rows each (four lanes per row, sixteen columns per lane), the others
// U12 = L11^-1 A12 for sixteen columns each (four per wavefront, lane m = row m).
template <typename T>
__global__ __launch_bounds__(256) void dlu_panel_kernel(DenseArgs a, int p, int nrb) {
    __shared__ T blk[NB][NB + 1];
    __shared__ T rowbuf[2 * NB];
    __shared__ T invd[NB];
    const int inst = blockIdx.y;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int D = a.D;
    const int nb = min(NB, D - p);
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    diag_factor<T>(S, D, p, nb, blk, rowbuf, invd);
    if (blockIdx.x == 0) {
        for (int e = tid; e < nb * nb; e += 256) {
            const int cc = e / nb, rr = e % nb;
            S[(size_t)(p + cc) * D + p + rr] = blk[cc][rr];
        }
        return;
    }
    if ((int)blockIdx.x <= nrb) {
        const int i = p + NB + ((int)blockIdx.x - 1) * 64 + tid / 4;
        const int sub = tid & 3;
        const bool act = i < D;
        T l[16];
#pragma unroll
        for (int e = 0; e < 16; e++) l[e] = act ? S[(size_t)(p + 16 * sub + e) * D + i] : T(0);
#pragma unroll 1
        for (int kb = 0; kb < 4; kb++) {
#pragma unroll
            for (int e0 = 0; e0 < 16; e0++) {
                const int kk = 16 * kb + e0;
                if (sub == kb) l[e0] = l[e0] * invd[kk];
                const T lk = __shfl(l[e0], (lane & ~3) | kb);
#pragma unroll
                for (int e = 0; e < 16; e++)
                    if (16 * sub + e > kk) l[e] -= lk * blk[16 * sub + e][kk];
            }
        }
        if (act) {
#pragma unroll
            for (int e = 0; e < 16; e++) S[(size_t)(p + 16 * sub + e) * D + i] = l[e];
        }
        return;
    }
    const int j0 = p + NB + (((int)blockIdx.x - 1 - nrb) * 4 + tid / WAVE) * 4;
    T v[4];
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = j0 + q < D ? S[(size_t)(j0 + q) * D + p + lane] : T(0);
    for (int kk = 0; kk < NB; kk++) {
        const T lmk = lane > kk ? blk[kk][lane] : T(0);   // L(lane, kk)
#pragma unroll
        for (int q = 0; q < 4; q++) v[q] -= lmk * readlane(v[q], kk);
    }
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (j0 + q < D) S[(size_t)(j0 + q) * D + p + lane] = v[q];
}

// A22 -= L21 U12 over the trailing block [p+NB, D)^2: a 128 x 128 output tile
// per workgroup, each wavefront 64 x 64 as 4 x 4 MFMA 16 x 16 tiles; K = NB in
// chunks of 16 staged through LDS (double-buffered, prefetched in registers).
// The MFMA computes the transposed tile (U12^T L21^T), so that a lane's results
// run down a column of S and the read-modify-write of C is coalesced.
// MFMA 16x16x4 operands: lane l holds A(l%16, l/16) and B(l/16, l%16).
template <typename T>
__global__ __launch_bounds__(256) void dlu_gemm_kernel(DenseArgs a, int p) {
    constexpr int TM = 128, KC = 16, LD = TM + 4;
    __shared__ T As[2][KC][LD];                       // [buf][k][row]
    __shared__ T Bs[2][KC][LD];                       // [buf][k][col]
    const int inst = blockIdx.z;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int D = a.D;
    const int r0 = p + NB + blockIdx.x * TM, c0 = p + NB + blockIdx.y * TM;
    const int tid = threadIdx.x;
    T ra[8], rb[8];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = tid + 256 * u;
            const int ka = e / TM, rr = e % TM;
            ra[u] = r0 + rr < D ? S[(size_t)(p + kc + ka) * D + r0 + rr] : T(0);
            const int kb = e % KC, cc = e / KC;
            rb[u] = c0 + cc < D ? S[(size_t)(c0 + cc) * D + p + kc + kb] : T(0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = tid + 256 * u;
            As[buf][e / TM][e % TM] = ra[u];
            Bs[buf][e % KC][e / KC] = rb[u];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int qr = wv >> 1, qc = wv & 1;
    const int li = lane & 15, lk = lane >> 4;
    typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
    acc_t acc[4][4];
#pragma unroll
    for (int ti = 0; ti < 4; ti++)
#pragma unroll
        for (int tj = 0; tj < 4; tj++) acc[ti][tj] = acc_t{0, 0, 0, 0};
#pragma unroll 1
    for (int ch = 0; ch < NB / KC; ch++) {
        const int buf = ch & 1;
        if (ch + 1 < NB / KC) fetch((ch + 1) * KC);
#pragma unroll
        for (int s = 0; s < KC / 4; s++) {
            T av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                av[t] = As[buf][4 * s + lk][64 * qr + 16 * t + li];
                bv[t] = Bs[buf][4 * s + lk][64 * qc + 16 * t + li];
            }
#pragma unroll
            for (int ti = 0; ti < 4; ti++)
#pragma unroll
                for (int tj = 0; tj < 4; tj++) {
                    if constexpr (sizeof(T) == 8)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
                    else
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
                }
        }
        if (ch + 1 < NB / KC) stash(buf ^ 1);
        __syncthreads();
    }
    // transposed tile: FP64 element q of lane l is C(row l%16, col 4q + l/16),
    // FP32 element q is C(row l%16, col 4(l/16) + q)
#pragma unroll
    for (int ti = 0; ti < 4; ti++)
#pragma unroll
        for (int tj = 0; tj < 4; tj++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = r0 + 64 * qr + 16 * ti + li;
                const int col = c0 + 64 * qc + 16 * tj + (sizeof(T) == 8 ? 4 * q + lk : 4 * lk + q);
                if (row < D && col < D) S[(size_t)col * D + row] -= acc[ti][tj][q];
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
    __shared__ double tri[NB][NB + 1];                // tri[col][row] of the diagonal block
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
    // block b: stage L(p.., p..) in LDS, then one wavefront substitutes (lane i = row p + i)
    const int p = b * NB, nb = min(NB, D - p);
    for (int e = tid; e < nb * nb; e += 256) tri[e / nb][e % nb] = (double)S[(size_t)(p + e / nb) * D + p + e % nb];
    __syncthreads();
    if (tid >= WAVE) return;
    double yv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) yv[r] = tid < nb ? yt[(size_t)(p + tid) * YS + r] : 0.0;
    for (int kk = 0; kk < nb; kk++) {
        const double lik = tid > kk && tid < nb ? tri[kk][tid] : 0.0;
#pragma unroll
        for (int r = 0; r < NR; r++) yv[r] -= lik * readlane(yv[r], kk);
    }
    if (tid < nb) {
#pragma unroll
        for (int r = 0; r < NR; r++) yt[(size_t)(p + tid) * YS + r] = yv[r];
    }
}

// Upper with its diagonal: launch b handles block blk = nblk-1-b: it applies
// block blk+1 to every row above it, then workgroup 0 solves block blk.
template <typename T, int NR>
__global__ __launch_bounds__(256) void dtrsv_upper_kernel(DenseArgs a, double *y, int b, const int *skip) {
    __shared__ double yb[NB][NR];
    __shared__ double tri[NB][NB + 1];                // tri[col][row] of the diagonal block
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
    for (int e = tid; e < nb * nb; e += 256) tri[e / nb][e % nb] = (double)S[(size_t)(p + e / nb) * D + p + e % nb];
    __syncthreads();
    if (tid >= WAVE) return;
    double yv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) yv[r] = tid < nb ? yt[(size_t)(p + tid) * YS + r] : 0.0;
    for (int kk = nb - 1; kk >= 0; kk--) {
        if (tid == kk) {
#pragma unroll
            for (int r = 0; r < NR; r++) yv[r] = yv[r] / tri[kk][kk];
        }
        const double uik = tid < kk ? tri[kk][tid] : 0.0;
#pragma unroll
        for (int r = 0; r < NR; r++) yv[r] -= uik * readlane(yv[r], kk);
    }
    if (tid < nb) {
#pragma unroll
        for (int r = 0; r < NR; r++) yt[(size_t)(p + tid) * YS + r] = yv[r];
    }
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
        const int rest = D - p - nb;   // > 0 only for full panels
        const int nrb = (rest + 63) / 64, ncb = (rest + 15) / 16;
        const dim3 gp((unsigned)(1 + nrb + ncb), (unsigned)a.batch);
        if (a.fp32) hipLaunchKernelGGL((dlu_panel_kernel<float>), gp, dim3(256), 0, st, a, p, nrb);
        else hipLaunchKernelGGL((dlu_panel_kernel<double>), gp, dim3(256), 0, st, a, p, nrb);
        if (rest > 0) {
            const dim3 gg((unsigned)((rest + 127) / 128), (unsigned)((rest + 127) / 128), (unsigned)a.batch);
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
