// Dense trailing block of the factorization, and the supernodal sweep of the sparse
// columns before it (gfx950).
//
// The last D columns of the factors are nearly dense: the paper's dense
// triangular block (Section V-A), whose order it picks from the fill density.
// After the sparse right-looking sweep over the first T = n - D columns, the
// trailing block S = A22 - L21 U12 (what the sweep left in those columns,
// rows >= T) is gathered into a dense column-major D x D matrix per instance and
// factored without pivoting by a blocked right-looking LU, panels of NB = 64 in
// groups of W (64, 128 or 256) columns:
//   dlu_panel  every workgroup factors the NB x NB diagonal block in registers
//              (four wavefronts, lane = row), then computes its share of
//              L21 = A21 U11^-1 or U12 = L11^-1 A12 (sixteen rows or columns
//              per wavefront) by block substitution on the matrix cores;
//   dlu_gemm   C -= L21 U12 on the matrix cores: 128 x 128 output tiles, K in
//              LDS-staged chunks, v_mfma_f64_16x16x4 (v_mfma_f32_16x16x4 for FP32
//              factors).  After a panel it updates only the rest of its group
//              (K = 64); after the group's last panel, the whole trailing block
//              with K = W, so that the trailing block is read and written once
//              per W columns instead of once per panel.
// dlu_check applies the pivot test of the sparse columns to every dense column
// c (x = L(:,c) u_cc are its values before division):
//   fail  <=>  u_cc not finite or zero, or max_{i>c} |x(i,c)| not finite, or
//              |u_cc| < eps * max_{i>c} |x(i,c)|.
// tail_scatter writes L and U back into the sparse factor storage (which the
// pivot-check fallback and the factor getters read).  The dense triangular
// solves run one launch per NB-row block: the launch for block b applies block
// b-1's solution to every row below it (the rectangle of the paper's trapezoid
// slices, Section V-A) and then one wavefront solves block b (the triangle).
// The Schur update S -= L21 U12 runs by supernode column runs (schur_sn_kernel)
// after a supernodal sweep, by bridge columns (schur_kernel) after a column sweep.
// The supernodal sweep itself (sn_*_kernel) is described at its section below.
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

// Workgroups are dispatched to the eight XCDs (each with its own L2) round-robin by index:
// renumber the n workgroups of a range so that each XCD gets a contiguous block of it, and
// neighbouring work items (which often read the same source columns) share an L2.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned i, unsigned n) {
    const unsigned q = n / 8, r = n % 8, x = i % 8;
    return x * q + (x < r ? x : r) + i / 8;
}

// lane l's value (l uniform)
__device__ __forceinline__ double readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

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
    for (int q0 = 0; q0 < len; q0 += 4 * WAVE) {      // four loads in flight per lane
        int r[4];
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int q = q0 + u * WAVE + lane;
            r[u] = q < len ? rows[q] : -1;
            x[u] = q < len ? Fx[q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (r[u] >= a.T) S[r[u] - a.T] = x[u];
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
    for (int q0 = 0; q0 < len; q0 += 4 * WAVE) {      // four loads in flight per lane
        int r[4];
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int q = q0 + u * WAVE + lane;
            r[u] = q < len ? rows[q] : -1;
            x[u] = r[u] >= a.T ? S[r[u] - a.T] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (r[u] >= a.T) Fx[q0 + u * WAVE + lane] = x[u];
    }
    // columns before the first failing one are final
    if (lane == 0 && k < a.ctrl[1 + a.batch + inst]) a.done[(size_t)inst * a.n + k] = (int)a.epoch;
}

// ------------------------------------------------------------- Schur update
// S(:, c) -= sum over the bridge rows j of dense column T + c (its U entries in rows
// < T, ascending) of L(rows >= T, j) U(j, T + c): the sparse columns' contribution to
// the dense block, applied after the sweep (all of L21 and U12 final).  A column's
// sources are cut into parts of similar cost (no column's chain then sets the time
// alone); one wavefront per (part, instance) applies its sources in ascending order,
// part 0 in place and each later part into a zeroed scratch column, which
// schur_add_kernel then adds to S in part order: deterministic, no atomics.  The L
// entries of four sources (up to 256 each) are loaded before any of them is applied,
// and each source reads all its targets before storing.
template <typename T>
__global__ __launch_bounds__(64) void schur_kernel(DenseArgs a, const int *parts, const int *l21) {
    constexpr int G = 4, CH = 4;                      // sources per group, 64-entry chunks loaded ahead
    const int lane = threadIdx.x;
    const int inst = (int)(blockIdx.x % (unsigned)a.batch);
    const int4 pr = reinterpret_cast<const int4 *>(parts)[blockIdx.x / (unsigned)a.batch];
    const int c = pr.x;
    if (sweep_failed(a, inst)) return;
    // part 0 of a column updates it in place; a later part accumulates into its zeroed
    // scratch column, which the add pass folds into S
    T *col = pr.w < 0 ? inst_S<T>(a, inst) + (size_t)c * a.D
                      : reinterpret_cast<T *>(a.scr) + ((size_t)inst * a.nscr + pr.w) * a.D;
    if (pr.w >= 0) {
        for (int i = lane; i < a.D; i += WAVE) col[i] = T(0);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int k = a.T + c;
    const int bb = a.Dp[k], nb = pr.z;                // bridge sources [pr.y, pr.z) of column k
    for (int s0 = pr.y; s0 < nb; s0 += WAVE) {
        int rb = 0, re = 0;
        T u = T(0);
        if (s0 + lane < nb) {
            const int j = a.Fi[bb + s0 + lane];
            u = Fx[bb + s0 + lane];                       // U(j, k)
            rb = l21[2 * j];
            re = l21[2 * j + 1];
        }
        const int ns = min(WAVE, nb - s0);
        for (int t = 0; t < ns; t += G) {
            int rr[G][CH], beg[G], end[G];
            T vv[G][CH], ug[G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int src = min(t + g, WAVE - 1);
                beg[g] = __shfl(rb, src);
                end[g] = t + g < ns ? __shfl(re, src) : beg[g];
                ug[g] = __shfl(u, src);
#pragma unroll
                for (int h = 0; h < CH; h++) {
                    const int q = beg[g] + h * WAVE + lane;
                    rr[g][h] = q < end[g] ? a.Fi[q] : -1;
                    vv[g][h] = q < end[g] ? Fx[q] : T(0);
                }
            }
#pragma unroll
            for (int g = 0; g < G; g++) {
                // one source: its rows are distinct, so all its targets are read before any store
                T tv[CH];
#pragma unroll
                for (int h = 0; h < CH; h++) tv[h] = rr[g][h] >= 0 ? col[rr[g][h] - a.T] : T(0);
#pragma unroll
                for (int h = 0; h < CH; h++)
                    if (rr[g][h] >= 0) col[rr[g][h] - a.T] = tv[h] - vv[g][h] * ug[g];
                for (int q0 = beg[g] + CH * WAVE; q0 < end[g]; q0 += WAVE) {   // very long sources
                    const int q = q0 + lane;
                    if (q < end[g]) col[a.Fi[q] - a.T] -= Fx[q] * ug[g];
                }
            }
        }
    }
}

// The Schur update by supernodes: a part of dense column c applies its items in order; item
// {S, c0, g, q} is the product of the rows >= T of columns s0 + c0 .. s0 + c0 + g - 1 of
// supernode S (shared rows, m - mlo of them, in every column after the block and the rows < T)
// with U(those columns, k), which sit at positions q .. q + g - 1 of column k = T + c.  Two rows
// per lane and up to sixteen loads in flight; each item reads all its targets before storing,
// and its rows are distinct.  Part 0 works in place, later parts in zeroed scratch columns
// that schur_add_kernel adds in part order.
template <typename T>
__global__ __launch_bounds__(64) void schur_sn_kernel(DenseArgs a, const int *parts, const int *items,
                                                      const int *sn_rec, const int *sn_cb) {
    const int lane = threadIdx.x;
    const int inst = (int)(blockIdx.x % (unsigned)a.batch);
    const int4 pr = reinterpret_cast<const int4 *>(parts)[blockIdx.x / (unsigned)a.batch];
    if (sweep_failed(a, inst)) return;
    T *col = pr.w < 0 ? inst_S<T>(a, inst) + (size_t)pr.x * a.D
                      : reinterpret_cast<T *>(a.scr) + ((size_t)inst * a.nscr + pr.w) * a.D;
    if (pr.w >= 0) {
        for (int i = lane; i < a.D; i += WAVE) col[i] = T(0);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    const T *Fx = reinterpret_cast<const T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int bb = a.Dp[a.T + pr.x];
    for (int it = pr.y; it < pr.z; it++) {
        const int4 item = reinterpret_cast<const int4 *>(items)[it];
        const int4 rec = reinterpret_cast<const int4 *>(sn_rec)[item.x];
        const int w = rec.y, mlo = rec.w, mhi = rec.z - rec.w, g = item.z;
        const int *cb = sn_cb + rec.x + item.y;
        const int *rows = a.Fi + sn_cb[rec.x + w - 1] + w + mlo;   // R's rows >= T
        const T uv = lane < g ? Fx[bb + item.w + lane] : T(0);
        for (int r0 = 0; r0 < mhi; r0 += 2 * WAVE) {
            const int ra = r0 + lane, rb = r0 + WAVE + lane;
            const bool ina = ra < mhi, inb = rb < mhi;
            const int ia = ina ? rows[ra] - a.T : 0, ib = inb ? rows[rb] - a.T : 0;
            T acca = T(0), accb = T(0);
            for (int c0 = 0; c0 < g; c0 += 8) {
                T la[8], lb[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int cc = c0 + u;
                    la[u] = (ina && cc < g) ? Fx[cb[cc] + w + mlo + ra] : T(0);
                    lb[u] = (inb && cc < g) ? Fx[cb[cc] + w + mlo + rb] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (c0 + u < g) {
                        const T uc = readlane(uv, c0 + u);
                        acca = fma(la[u], uc, acca);
                        accb = fma(lb[u], uc, accb);
                    }
            }
            const T ta = ina ? col[ia] : T(0), tb = inb ? col[ib] : T(0);
            if (ina) col[ia] = ta - acca;
            if (inb) col[ib] = tb - accb;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

// S(:, c) += the scratch columns of c's later parts, in part order: one wavefront per
// (split column, instance), four rows in flight per lane
template <typename T>
__global__ __launch_bounds__(256) void schur_add_kernel(DenseArgs a, const int *add, int nadd) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= (int64_t)nadd * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int4 r = reinterpret_cast<const int4 *>(add)[w / a.batch];
    if (sweep_failed(a, inst)) return;
    T *col = inst_S<T>(a, inst) + (size_t)r.x * a.D;
    const T *scr = reinterpret_cast<const T *>(a.scr) + ((size_t)inst * a.nscr + r.y) * a.D;
    for (int i0 = 0; i0 < a.D; i0 += 4 * WAVE) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = i0 + u * WAVE + lane < a.D ? col[i0 + u * WAVE + lane] : T(0);
        for (int p = 0; p < r.z; p++) {
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (i0 + u * WAVE + lane < a.D) v[u] += scr[(size_t)p * a.D + i0 + u * WAVE + lane];
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (i0 + u * WAVE + lane < a.D) col[i0 + u * WAVE + lane] = v[u];
    }
}

// ------------------------------------------------------------- blocked LU

// 1 / u.  FP64: the hardware reciprocal refined by two Newton-Raphson steps
// (r <- r + r (1 - u r)), each of which doubles the correct bits, for |u| in
// [2^-1000, 2^1000] (no overflow or underflow on the way); elsewhere, and for FP32,
// the division.  The branch is uniform: u comes from readlane.
__device__ __forceinline__ double recip(double u) {
    const double au = __builtin_fabs(u);
    if (au >= 0x1p-1000 && au <= 0x1p1000) {
        double r = __builtin_amdgcn_rcp(u);
        r = fma(r, fma(-u, r, 1.0), r);
        return fma(r, fma(-u, r, 1.0), r);
    }
    return 1.0 / u;
}
__device__ __forceinline__ float recip(float u) { return 1.0f / u; }

// Factors the nb x nb diagonal block at (p, p) of S (padded to NB x NB with the
// identity) without pivoting, with the workgroup's four wavefronts, two columns per
// step: lane r holds row r, wavefront W the column pairs (8a + 2W, 8a + 2W + 1) in
// v[2a], v[2a + 1].  Step (kk, kk+1): the owner of the pair (W = kk/2 % 4) forms
// L(:, kk) = x * (1 / u_kk), applies it to column kk+1 and forms L(:, kk+1), and
// passes both through LDS (two buffers, one barrier per step); every wavefront then
// updates its columns c > kk+1 with both, U(kk, c) read from lane kk by readlane and
// U(kk+1, c) = x(kk+1, c) - L(kk+1, kk) U(kk, c) formed as lane kk+1 would, so the
// result equals two single steps bit for bit.  The factors go to blk[col][row] (unit
// L below the diagonal, U on and above it) and invd[k] = 1 / u_kk.
// The block's element (row r, column c) comes from elem(c, r), which returns the identity's
// element outside the nb x nb block.
template <typename T, int W, typename Elem>
__device__ void diag_factor_part(Elem elem, T (*blk)[NB + 1], T *invd, T (*lbuf)[WAVE]) {
    const int lane = threadIdx.x & (WAVE - 1);
    T v[NB / 4];
#pragma unroll
    for (int j = 0; j < NB / 4; j++) {
        const int c = 8 * (j / 2) + 2 * W + (j % 2);
        v[j] = elem(c, lane);
    }
#pragma unroll
    for (int kk = 0; kk < NB; kk += 2) {
        const int buf = 2 * ((kk / 2) & 1);
        T l0, l1;
        if (((kk / 2) & 3) == W) {
            const int jk = 2 * (kk / 8);
            const T inv0 = recip(readlane(v[jk], kk));
            l0 = lane > kk ? v[jk] * inv0 : T(0);
            v[jk] = lane > kk ? l0 : v[jk];
            v[jk + 1] = fma(-l0, readlane(v[jk + 1], kk), v[jk + 1]);
            const T inv1 = recip(readlane(v[jk + 1], kk + 1));
            l1 = lane > kk + 1 ? v[jk + 1] * inv1 : T(0);
            v[jk + 1] = lane > kk + 1 ? l1 : v[jk + 1];
            if (lane == 0) {
                invd[kk] = inv0;
                invd[kk + 1] = inv1;
            }
            lbuf[buf][lane] = l0;
            lbuf[buf + 1][lane] = l1;
        }
        __syncthreads();
        if (((kk / 2) & 3) != W) {
            l0 = lbuf[buf][lane];
            l1 = lbuf[buf + 1][lane];
        }
        const T l0n = readlane(l0, kk + 1);            // L(kk+1, kk)
#pragma unroll
        for (int j = 0; j < NB / 4; j++) {
            if (8 * (j / 2) + 2 * W + (j % 2) > kk + 1) {
                const T u0 = readlane(v[j], kk);
                const T u1 = fma(-l0n, u0, readlane(v[j], kk + 1));
                v[j] = fma(-l1, u1, fma(-l0, u0, v[j]));
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NB / 4; j++) blk[8 * (j / 2) + 2 * W + (j % 2)][lane] = v[j];
}
template <typename T, typename Elem>
__device__ void diag_factor_elem(Elem elem, T (*blk)[NB + 1], T *invd, T (*lbuf)[WAVE], int wv) {
    switch (wv) {
    case 0: diag_factor_part<T, 0>(elem, blk, invd, lbuf); break;
    case 1: diag_factor_part<T, 1>(elem, blk, invd, lbuf); break;
    case 2: diag_factor_part<T, 2>(elem, blk, invd, lbuf); break;
    default: diag_factor_part<T, 3>(elem, blk, invd, lbuf); break;
    }
}
// the nb x nb diagonal block at (p, p) of S (column-major, leading dimension D)
template <typename T>
__device__ void diag_factor(const T *S, int D, int p, int nb, T (*blk)[NB + 1], T *invd, T (*lbuf)[WAVE], int wv) {
    auto elem = [=](int c, int r) -> T {
        return (r < nb && c < nb) ? S[(size_t)(p + c) * D + p + r] : (r == c ? T(1) : T(0));
    };
    diag_factor_elem<T>(elem, blk, invd, lbuf, wv);
}

// k of step s for lane group g (= lane / 16) in a 16 x 16 x 4 MFMA chain: the
// accumulator's element s is then the B operand of step s.  FP64 accumulators hold
// rows 4s + g, FP32 rows 4g + s (column lane % 16 in both).
template <typename T>
__device__ __forceinline__ int kidx(int s, int g) { return sizeof(T) == 8 ? 4 * s + g : 4 * g + s; }

template <typename T>
__device__ __forceinline__ auto mfma16(T a, T b, typename std::conditional<sizeof(T) == 8, d4, f4>::type c) {
    if constexpr (sizeof(T) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One panel [p, p+nb).  Every workgroup factors the diagonal block (workgroup 0
// writes it back).  The other
// workgroups compute L21 = A21 U11^-1 (the first nrb, 64 rows each) or
// U12 = L11^-1 A12 (64 columns each), sixteen rows (columns) per wavefront, as a
// block substitution over the four 16 x 16 diagonal blocks of U11 (L11):
//   X_b = (A_b - sum_{b'<b} X_b' U_b'b) U_bb^-1,   Y_b = L_bb^-1 (A_b - sum_{b'<b} L_bb' Y_b'),
// on the matrix cores; wavefront b first inverts diagonal block b (sixteen-step
// substitution, lane = column).  The row case runs transposed (X^T = U^-T ...)
// so that in both cases each product's accumulator is the next one's B operand.
template <typename T>
__global__ __launch_bounds__(256) void dlu_panel_kernel(DenseArgs a, int p, int nrb) {
    typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
    __shared__ T blk[NB][NB + 1];
    __shared__ T invd[NB];
    __shared__ T winv[4][16][17];                     // [b][row][col] of U_bb^-1 or L_bb^-1
    __shared__ T lbuf[4][WAVE];
    const int inst = blockIdx.y;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int D = a.D;
    const int nb = min(NB, D - p);
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int i16 = lane & 15, g = lane >> 4;
    // loads of this wavefront's rows / columns (accumulator layout), issued before the wait
    const bool rows = (int)blockIdx.x <= nrb;
    const int first = p + NB + (((int)blockIdx.x - 1 - (rows ? 0 : nrb)) * 4 + wv) * 16;
    const bool in = first + i16 < D;
    acc_t t[4];
    auto load = [&]() {
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = p + 16 * b + kidx<T>(q, g);
                t[b][q] = !in ? T(0) : rows ? S[(size_t)k * D + first + i16] : S[(size_t)(first + i16) * D + k];
            }
    };
    if (blockIdx.x != 0) load();
    diag_factor<T>(S, D, p, nb, blk, invd, lbuf, wv);
    __syncthreads();
    if (blockIdx.x == 0) {
        // Other workgroups of this launch still read the unfactored block from S, so the
        // factors go to the instance's scratch block, which the update launch of this panel
        // copies into S; a panel without other workgroups (the last) writes S directly.
        T *dst = gridDim.x == 1 ? S + (size_t)p * D + p : reinterpret_cast<T *>(a.Dg) + (size_t)inst * NB * NB;
        const int ld = gridDim.x == 1 ? D : NB;
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int rr = 16 * wv + e;
            if (lane < nb && rr < nb) dst[(size_t)lane * ld + rr] = blk[lane][rr];
        }
        return;
    }
    // (a full panel: nb = NB here) inverse of diagonal block b = wv, column i16
    {
        const int o = 16 * wv;
        T x[16];
        if (rows) {                                   // U_bb x = e_j, upper, from the bottom
#pragma unroll
            for (int i = 15; i >= 0; i--) {
                T acc = i == i16 ? T(1) : T(0);
#pragma unroll
                for (int k = i + 1; k < 16; k++) acc = fma(-blk[o + k][o + i], x[k], acc);
                x[i] = acc * invd[o + i];
            }
        } else {                                      // L_bb x = e_j, unit lower, from the top
#pragma unroll
            for (int i = 0; i < 16; i++) {
                T acc = i == i16 ? T(1) : T(0);
#pragma unroll
                for (int k = 0; k < i; k++) acc = fma(-blk[o + k][o + i], x[k], acc);
                x[i] = acc;
            }
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; i++) winv[wv][i][i16] = x[i];
        }
    }
    __syncthreads();
    if (first >= D) return;
    acc_t x[4];
#pragma unroll
    for (int b = 0; b < 4; b++) {
#pragma unroll
        for (int bp = 0; bp < b; bp++)
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const int k = 16 * bp + kidx<T>(s, g);
                // row case: (U_b'b)^T (i16, k) = U(k, 16b + i16); column case: L_bb'(i16, k) = L(16b + i16, k)
                const T av = rows ? -blk[16 * b + i16][k] : -blk[k][16 * b + i16];
                t[b] = mfma16<T>(av, x[bp][s], t[b]);
            }
        acc_t z = {};
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int k = kidx<T>(s, g);
            // row case: (U_bb^-1)^T (i16, k); column case: L_bb^-1 (i16, k)
            const T av = rows ? winv[b][k][i16] : winv[b][i16][k];
            z = mfma16<T>(av, t[b][s], z);
        }
        x[b] = z;
    }
    if (in) {
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = p + 16 * b + kidx<T>(q, g);
                if (rows) S[(size_t)k * D + first + i16] = x[b][q];
                else S[(size_t)(first + i16) * D + k] = x[b][q];
            }
    }
}

// C -= L(:, K) U(K, :) over up to two output rectangles of S, K = columns
// [kp, kp + KW) (KW = 64, 128 or 256): the whole trailing block after a group of
// panels, or the rest of the group after one of its panels.  A 128 x 128 output
// tile per workgroup, each wavefront 64 x 64 as 4 x 4 MFMA 16 x 16 tiles; K in
// chunks of 16 staged through LDS (double-buffered, prefetched in registers).
// TM = 64 (32 x 32 per wavefront) for the narrow in-group updates: four times as
// many workgroups, so that several share a CU and overlap their loads and MFMAs.
// The MFMA computes the transposed tile (U12^T L21^T), so that a lane's results
// run down a column of S and the read-modify-write of C is coalesced.
// MFMA 16x16x4 operands: lane l holds A(l%16, l/16) and B(l/16, l%16).
struct GemmRect {
    int r0, r1, c0, c1;        // rows [r0, r1) x columns [c0, c1) of S
    int ntx, nt;               // tiles down a tile column, tiles in all
};
template <typename T, int KW, int TM = 128>
__global__ __launch_bounds__(256) void dlu_gemm_kernel(DenseArgs a, int kp, GemmRect g0, GemmRect g1, int dgp) {
    constexpr int KC = 16, LD = TM + 4;
    constexpr int WT = TM / 2, NT = WT / 16, FE = KC * TM / 256;   // wave tile, MFMA tiles, staged per thread
    __shared__ T As[2][KC][LD];                       // [buf][k][row]
    __shared__ T Bs[2][KC][LD];                       // [buf][k][col]
    const int inst = blockIdx.z;
    if (sweep_failed(a, inst)) return;
    T *S = inst_S<T>(a, inst);
    const int D = a.D;
    const bool first = (int)blockIdx.x < g0.nt;
    const int t = first ? (int)blockIdx.x : (int)blockIdx.x - g0.nt;
    const int ntx = first ? g0.ntx : g1.ntx;
    const int r0 = (first ? g0.r0 : g1.r0) + (t % ntx) * TM, c0 = (first ? g0.c0 : g1.c0) + (t / ntx) * TM;
    const int R1 = first ? g0.r1 : g1.r1, C1 = first ? g0.c1 : g1.c1;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && dgp >= 0) {
        // the factored diagonal block of the panel at dgp (it had a trailing part, so its
        // factors went to the scratch block while its other workgroups still read S)
        const T *src = reinterpret_cast<const T *>(a.Dg) + (size_t)inst * NB * NB;
        T tv[16];
#pragma unroll
        for (int u = 0; u < 16; u++) tv[u] = src[tid + 256 * u];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int e = tid + 256 * u;
            S[(size_t)(dgp + e / NB) * D + dgp + e % NB] = tv[u];
        }
    }
    T ra[FE], rb[FE];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int u = 0; u < FE; u++) {
            const int e = tid + 256 * u;
            const int ka = e / TM, rr = e % TM;
            ra[u] = r0 + rr < R1 ? S[(size_t)(kp + kc + ka) * D + r0 + rr] : T(0);
            const int kb = e % KC, cc = e / KC;
            rb[u] = c0 + cc < C1 ? S[(size_t)(c0 + cc) * D + kp + kc + kb] : T(0);
        }
    };
    auto stash = [&](int buf) {                      // A is stored negated: acc = C + (-A) B
#pragma unroll
        for (int u = 0; u < FE; u++) {
            const int e = tid + 256 * u;
            As[buf][e / TM][e % TM] = -ra[u];
            Bs[buf][e % KC][e / KC] = rb[u];
        }
    };
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int qr = wv >> 1, qc = wv & 1;
    const int li = lane & 15, lk = lane >> 4;
    // C(row, col) of accumulator element q (transposed tile, see the epilogue)
    auto crow = [&](int ti) { return r0 + WT * qr + 16 * ti + li; };
    auto ccol = [&](int tj, int q) { return c0 + WT * qc + 16 * tj + (sizeof(T) == 8 ? 4 * q + lk : 4 * lk + q); };
    typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
    acc_t acc[NT][NT];
    // the accumulators start from C, loaded before any store of this workgroup
#pragma unroll
    for (int ti = 0; ti < NT; ti++)
#pragma unroll
        for (int tj = 0; tj < NT; tj++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = crow(ti), col = ccol(tj, q);
                acc[ti][tj][q] = (row < R1 && col < C1) ? S[(size_t)col * D + row] : T(0);
            }
    fetch(0);
    stash(0);
    __syncthreads();
    constexpr int nch = KW / KC;       // a compile-time trip count keeps the kernel at two waves per SIMD
#pragma unroll 1
    for (int ch = 0; ch < nch; ch++) {
        const int buf = ch & 1;
        if (ch + 1 < nch) fetch((ch + 1) * KC);
#pragma unroll
        for (int s = 0; s < KC / 4; s++) {
            T av[NT], bv[NT];
#pragma unroll
            for (int t = 0; t < NT; t++) {
                av[t] = As[buf][4 * s + lk][WT * qr + 16 * t + li];
                bv[t] = Bs[buf][4 * s + lk][WT * qc + 16 * t + li];
            }
#pragma unroll
            for (int ti = 0; ti < NT; ti++)
#pragma unroll
                for (int tj = 0; tj < NT; tj++) {
                    if constexpr (sizeof(T) == 8)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
                    else
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
                }
        }
        if (ch + 1 < nch) stash(buf ^ 1);
        __syncthreads();
    }
    // transposed tile: FP64 element q of lane l is C(row l%16, col 4q + l/16),
    // FP32 element q is C(row l%16, col 4(l/16) + q)
#pragma unroll
    for (int ti = 0; ti < NT; ti++)
#pragma unroll
        for (int tj = 0; tj < NT; tj++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = crow(ti), col = ccol(tj, q);
                if (row < R1 && col < C1) S[(size_t)col * D + row] = acc[ti][tj][q];
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
    for (int i0 = c + 1; i0 < a.D; i0 += 4 * WAVE) {
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = i0 + u * WAVE + lane < a.D ? col[i0 + u * WAVE + lane] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) m = nanmax(m, fabs((double)x[u]));
    }
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

// ------------------------------------------------- diagonal-block inverses
// For the dense solves: the inverses of each 64 x 64 diagonal block's unit-lower and
// upper triangles (the last block padded with the identity), FP64 whatever the factor
// type.  One wavefront per (block, instance); lane j forms column j of each inverse
// by substitution with the block read from LDS by broadcast.  Stored at
// Dinv + ((inst * nblk + b) * 2 + {0: L, 1: U}) * 64 * 64, column-major.
template <typename T>
__global__ __launch_bounds__(64) void dlu_inverse_kernel(DenseArgs a) {
    __shared__ double blk[NB][NB + 1];                // blk[col][row]
    // no early exit for instances whose sweep failed: S may be re-gathered after a fallback
    // while the status words still record the failure (a failed instance's solve is skipped)
    const int b = blockIdx.x, inst = blockIdx.y, j = threadIdx.x;
    const T *S = inst_S<T>(a, inst);
    const int D = a.D, p = b * NB, nb = min(NB, D - p), nblk = (D + NB - 1) / NB;
    for (int c = 0; c < NB; c++)
        blk[c][j] = (c < nb && j < nb) ? (double)S[(size_t)(p + c) * D + p + j] : (c == j ? 1.0 : 0.0);
    __syncthreads();
    double *out = a.Dinv + ((size_t)inst * nblk + b) * 2 * NB * NB;
    double x[NB];
    // L x = e_j, unit diagonal
#pragma unroll
    for (int i = 0; i < NB; i++) {
        double v = i == j ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; k++) v -= blk[k][i] * x[k];
        x[i] = v;
        asm volatile("" ::: "memory");                // each row's LDS reads stay with it
    }
#pragma unroll
    for (int i = 0; i < NB; i++) out[(size_t)j * NB + i] = x[i];
    // U x = e_j
#pragma unroll
    for (int i = NB - 1; i >= 0; i--) {
        double v = i == j ? 1.0 : 0.0;
#pragma unroll
        for (int k = i + 1; k < NB; k++) v -= blk[k][i] * x[k];
        x[i] = v / blk[i][i];
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int i = 0; i < NB; i++) out[(size_t)NB * NB + (size_t)j * NB + i] = x[i];
}

// ------------------------------------------------------------- dense solves
// y rows T.. of each instance hold the partial solution (NR doubles per row).  Launch b of a
// triangle applies one solved block to the rows that still need it and solves the next
// diagonal block.  A workgroup takes 64 rows, its four wavefronts a quarter of the applied
// block's 64 columns each (a row per lane, sixteen loads in flight); the quarters' sums meet in
// LDS in quarter order.  Workgroup 0 holds exactly the rows of the block it then solves: it
// keeps their updated values in LDS and multiplies them by the block's inverse (made at
// factorization time), again a quarter of the columns per wavefront.
// Lower, unit diagonal: launch b applies block b-1 to rows >= b*NB and solves block b.
// Upper with its diagonal: launch b applies block blk+1 (blk = nblk-1-b) to the rows above it
// and solves block blk.
template <typename T, int NR, bool UPPER>
__global__ __launch_bounds__(256) void dtrsv_kernel(DenseArgs a, double *y, int b, const int *skip) {
    __shared__ double yb[NB][NR];                     // the applied block's x, then the solved block's rows
    __shared__ double part[4][NR][NB];                // the quarters' sums, [quarter][rhs][row]
    __shared__ double tri[NB][NB + 1];                // tri[col][row] of the diagonal block's inverse
    const int inst = blockIdx.y;
    if (skip && skip[inst] != -1) return;
    const T *S = inst_S<T>(a, inst);
    double *yt = y + ((size_t)inst * a.n + a.T) * NR;
    const int D = a.D, tid = threadIdx.x, lane = tid & (NB - 1), q = tid / NB;
    const int nblk = (D + NB - 1) / NB;
    const int blk = UPPER ? nblk - 1 - b : b;         // the block this launch solves
    const int p = blk * NB, nb = min(NB, D - p);
    // the applied block (columns [pa, pa + na)) and this workgroup's rows
    const int pa = UPPER ? (blk + 1) * NB : (blk - 1) * NB;
    const int na = b > 0 ? min(NB, D - pa) : 0;
    const int i = UPPER ? p - (int)blockIdx.x * NB + lane : p + (int)blockIdx.x * NB + lane;
    const bool row = UPPER ? i >= 0 && i < p + nb : i < D;
    // workgroup 0: the inverse of the diagonal block, loaded before the rectangle
    const double *inv = a.Dinv + ((size_t)inst * nblk + blk) * 2 * NB * NB + (UPPER ? NB * NB : 0);   // [col][row]
    double t[16];
    if (blockIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < 16; u++) t[u] = inv[tid + 256 * u];
    }
    double yi[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) yi[r] = q == 0 && row ? yt[(size_t)i * NR + r] : 0.0;
    if (b > 0) {
        if (tid < NB * NR / 2) {                      // NB * NR <= 512: two loads per thread
            const int e1 = tid + NB * NR / 2;
            const double y0 = tid / NR < na ? yt[(size_t)(pa + tid / NR) * NR + tid % NR] : 0.0;
            const double y1 = e1 / NR < na ? yt[(size_t)(pa + e1 / NR) * NR + e1 % NR] : 0.0;
            yb[tid / NR][tid % NR] = y0;
            yb[e1 / NR][e1 % NR] = y1;
        }
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] = 0.0;
        double l[16];
#pragma unroll
        for (int m = 0; m < 16; m++) {
            const int c = 16 * q + m;
            l[m] = row && c < na ? (double)S[(size_t)(pa + c) * D + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; m++) {
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] = fma(l[m], yb[16 * q + m][r], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; r++) part[q][r][lane] = acc[r];
        __syncthreads();
        if (q == 0 && row) {
#pragma unroll
            for (int r = 0; r < NR; r++)
                yi[r] -= ((part[0][r][lane] + part[1][r][lane]) + part[2][r][lane]) + part[3][r][lane];
            if (blockIdx.x != 0) {
#pragma unroll
                for (int r = 0; r < NR; r++) yt[(size_t)i * NR + r] = yi[r];
            }
        }
    }
    if (blockIdx.x != 0) return;
    // the solved block: x = inverse * (its rows' values), row lane of the block from quarter q's
    // sixteen columns, the quarters added in order
    __syncthreads();                                  // yb's last reads (the rectangle) are done
    if (q == 0) {
#pragma unroll
        for (int r = 0; r < NR; r++) yb[lane][r] = lane < nb ? yi[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; u++) tri[(tid + 256 * u) / NB][(tid + 256 * u) % NB] = t[u];
    __syncthreads();
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int k = 16 * q + m;                     // the inverse is triangular: zero entries add nothing
        const bool in = UPPER ? k >= lane : k <= lane;
        if (in) {
            const double v = tri[k][lane];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] = fma(v, yb[k][r], acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) part[q][r][lane] = acc[r];
    __syncthreads();
    if (q == 0 && lane < nb) {
#pragma unroll
        for (int r = 0; r < NR; r++)
            yt[(size_t)(p + lane) * NR + r] = ((part[0][r][lane] + part[1][r][lane]) + part[2][r][lane]) + part[3][r][lane];
    }
}

template <typename T, int NR>
void dense_solve_impl(const DenseArgs &a, double *y, const int *skip, bool upper, hipStream_t st) {
    const int nblk = (a.D + NB - 1) / NB;
    for (int b = 0; b < nblk; b++) {
        // rows the launch takes: lower -> rows >= b*NB; upper -> rows above block nblk-b
        const int rows = b == 0 ? 1 : (upper ? (nblk - b) * NB : a.D - b * NB);
        const dim3 g((unsigned)((rows + NB - 1) / NB), (unsigned)a.batch);
        if (upper) hipLaunchKernelGGL((dtrsv_kernel<T, NR, true>), g, dim3(256), 0, st, a, y, b, skip);
        else hipLaunchKernelGGL((dtrsv_kernel<T, NR, false>), g, dim3(256), 0, st, a, y, b, skip);
    }
}

// ------------------------------------------------------- pivoted dense LU
// The re-factorization of the dense block when its pivot test failed (the
// sparse columns all passed, so only the block changes): the same blocked
// right-looking LU in panels of NB, with the threshold pivot rule applied to
// each column over the whole remaining height.  A step launch for column k
// (every workgroup finds the same pivot from column k, which no workgroup of
// that launch writes) exchanges rows k and p_k in the panel's later columns and
// applies the rank-1 update to them; column k itself is completed (exchange,
// division by the pivot) by the next step launch, which also carries the
// exchanges into the panel's earlier columns.  After a panel, its exchanges are
// applied to every other column, U12 = L11^-1 A12, and the trailing block gets
// the K = NB update.  FP64, one instance.

// pivot of column k over rows [k, D): returns the chosen row; *bad when no usable pivot
__device__ int dpiv_choose(const double *col, int k, int D, double eps, bool *bad) {
    __shared__ double s_best[256], s_oth[256];
    __shared__ int s_bi[256], s_bad[256];
    const int tid = threadIdx.x;
    double best = -1.0, oth = 0.0;
    int bi = INT_MAX, nf = 0;
    for (int i = k + tid; i < D; i += 256) {            // ascending rows: ties keep the first
        const double v = col[i], av = fabs(v);
        if (!isfinite(v)) nf = 1;
        if (i != k) oth = fmax(oth, av);
        if (av > best) { best = av; bi = i; }
    }
    s_best[tid] = best; s_bi[tid] = bi; s_oth[tid] = oth; s_bad[tid] = nf;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const double b2 = s_best[tid + off];
            const int i2 = s_bi[tid + off];
            if (b2 > s_best[tid] || (b2 == s_best[tid] && i2 < s_bi[tid])) { s_best[tid] = b2; s_bi[tid] = i2; }
            s_oth[tid] = fmax(s_oth[tid], s_oth[tid + off]);
            s_bad[tid] |= s_bad[tid + off];
        }
        __syncthreads();
    }
    const double xd = col[k];
    int pk = k;
    if (!(isfinite(xd) && xd != 0.0 && fabs(xd) >= eps * s_oth[0])) pk = s_bi[0];
    *bad = s_bad[0] != 0 || pk >= D || col[pk] == 0.0;
    const int r = pk < D ? pk : k;
    __syncthreads();                                     // the shared arrays are reused by the caller
    return r;
}

// blockIdx.x: 0 completes column k-1 (its exchange, its division, then this step's
// exchange); 1 carries this step's exchange into columns [p, k-1); 2 + t updates
// column k + 1 + t.  k == pe: only the completion of column pe - 1.
__global__ __launch_bounds__(256) void dpiv_step_kernel(DenseArgs a, int p, int pe, int k, int *swp, int *info) {
    double *S = reinterpret_cast<double *>(a.S);
    const int D = a.D, tid = threadIdx.x, role = blockIdx.x;
    int pk = -1;
    double xp = 0.0;
    if (k < pe) {
        bool bad = false;
        pk = dpiv_choose(S + (size_t)k * D, k, D, a.eps, &bad);
        xp = S[(size_t)k * D + pk];
        if (role == 0 && tid == 0) {
            swp[k] = pk;
            if (bad && *info == 0) *info = k + 1;
        }
    }
    auto exch = [&](double *col, int r1, int r2) {
        if (r1 != r2 && tid == 0) { const double t = col[r1]; col[r1] = col[r2]; col[r2] = t; }
    };
    if (role == 0) {
        if (k > p) {
            double *col = S + (size_t)(k - 1) * D;
            const int q = swp[k - 1];
            exch(col, k - 1, q);
            __syncthreads();
            const double u = col[k - 1];
            for (int i = k + tid; i < D; i += 256) col[i] = col[i] / u;
            __syncthreads();
            if (k < pe) exch(col, k, pk);
        }
        return;
    }
    if (k >= pe) return;
    if (role == 1) {
        for (int c = p + tid; c < k - 1; c += 256) {
            double *col = S + (size_t)c * D;
            if (pk != k) { const double t = col[k]; col[k] = col[pk]; col[pk] = t; }
        }
        return;
    }
    const int j = k + 1 + (role - 2);
    double *cj = S + (size_t)j * D;
    const double *ck = S + (size_t)k * D;
    exch(cj, k, pk);
    __syncthreads();
    const double ukj = cj[k];
    const double xk = ck[k];
    for (int i = k + 1 + tid; i < D; i += 256) {
        const double xi = i == pk ? xk : ck[i];            // column k after the exchange
        cj[i] -= (xi / xp) * ukj;
    }
}

// the exchanges of panel [p, pe) applied to the columns outside it, 64 columns per
// workgroup, the panel's rows staged in LDS
__global__ __launch_bounds__(64) void dpiv_swap_rest_kernel(DenseArgs a, int p, int pe, const int *swp) {
    __shared__ double rows[NB][NB + 1];
    double *S = reinterpret_cast<double *>(a.S);
    const int D = a.D, lane = threadIdx.x;
    const int nleft = p, nright = D - pe;
    const int c_idx = (int)blockIdx.x * NB + lane;
    const bool valid = c_idx < nleft + nright;
    const int c = c_idx < nleft ? c_idx : pe + (c_idx - nleft);
    const int nb = pe - p;
    double *col = S + (size_t)(valid ? c : 0) * D;
    if (valid)
        for (int r = 0; r < nb; r++) rows[r][lane] = col[p + r];
    for (int k = p; k < pe; k++) {
        const int q = swp[k];
        if (!valid || q == k) continue;
        if (q < pe) {
            const double t = rows[k - p][lane];
            rows[k - p][lane] = rows[q - p][lane];
            rows[q - p][lane] = t;
        } else {
            const double t = col[q];
            col[q] = rows[k - p][lane];
            rows[k - p][lane] = t;
        }
    }
    if (valid)
        for (int r = 0; r < nb; r++) col[p + r] = rows[r][lane];
}

// U12 = L11^-1 A12 for the columns past the panel: the unit lower L11 staged in LDS,
// a column per lane (64 rows in registers), 256 columns per workgroup
__global__ __launch_bounds__(256) void dpiv_u12_kernel(DenseArgs a, int p) {
    __shared__ double l11[NB][NB];                      // l11[col][row]
    double *S = reinterpret_cast<double *>(a.S);
    const int D = a.D, tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) l11[e / NB][e % NB] = S[(size_t)(p + e / NB) * D + p + e % NB];
    __syncthreads();
    const int j = p + NB + (int)blockIdx.x * 256 + tid;
    if (j >= D) return;
    double *col = S + (size_t)j * D + p;
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; r++) x[r] = col[r];
#pragma unroll
    for (int kk = 0; kk < NB; kk++)
#pragma unroll
        for (int m = kk + 1; m < NB; m++) x[m] -= l11[kk][m] * x[kk];
#pragma unroll
    for (int r = 0; r < NB; r++) col[r] = x[r];
}

__global__ void zero_int_kernel(int *v) { *v = 0; }

inline dim3 wave_grid(int64_t waves) { return dim3((unsigned)((waves + 3) / 4)); }

// ------------------------------------------------------------- supernodal sweep
// A supernode is a run of sparse columns [s0, s0 + w) with a dense diagonal block and the
// same rows R (m of them) below it; column s0 + c keeps rows s0 .. s0 + w - 1 and then R
// contiguously from offset sn_cb[s0 + c] of its storage.  The interrupt word of an
// instance holds 1 + the level whose pivot test failed first: a level's work stops only
// for failures of earlier levels, so which columns finish does not depend on timing.
__device__ __forceinline__ bool sn_stopped(const RefactorArgs &a, int inst, int lev) {
    if (!a.check) return false;
    const int st = a.ctrl[1 + inst];
    return st != 0 && st <= lev;
}
__device__ __forceinline__ void sn_fail(const RefactorArgs &a, int inst, int lev, int col) {
    atomicMin(&a.ctrl[1 + a.batch + inst], col);
    atomicExch(&a.ctrl[1 + inst], lev + 1);          // every writer of this launch writes the same
}

// Small supernodes (w <= kSnSmallW columns).  A singleton (one column j; sixteen lanes, see
// sn_single_kernel): the pivot test on its values before division (Section II-A: fail when
// x(j) is zero or not finite, or |x(j)| < eps max |L part|), then L(:,j) = x / x(j).  A small
// panel (one wavefront per unit and instance): lane r < w holds row r of the diagonal block, factored by
// right-looking steps (column c: L(r, c) = x(r, c) / u_cc below the diagonal, then
// x(r, c') -= L(r, c) U(c, c') for c' > c); the rows of R, 64 at a time (a row per lane), by
// the same steps with U11 read from the block's lanes.  The pivot test of column c is taken
// on its values before division: the block rows below c and every row of R.
template <typename T>
__device__ void sn_small_panel(const RefactorArgs &a, int inst, int lev, int s0, int w, int m, int4 un, int lane) {
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int *cb = a.sn_cb + s0;
    // this unit's rows of R: slice un.y of un.z
    const int rb = (int)((int64_t)m * un.y / un.z), re = (int)((int64_t)m * (un.y + 1) / un.z);
    T bv[kSnSmallW];
    double mx[kSnSmallW];
#pragma unroll
    for (int c = 0; c < kSnSmallW; c++) {
        bv[c] = (c < w && lane < w) ? Fx[cb[c] + lane] : T(0);
        mx[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < kSnSmallW; c++) {
        if (c < w) {                                       // uniform
            const T inv = recip(readlane(bv[c], c));
            const bool below = lane > c && lane < w;
            if (below) {
                mx[c] = nanmax(mx[c], fabs((double)bv[c]));
                bv[c] = bv[c] * inv;
            }
#pragma unroll
            for (int c2 = c + 1; c2 < kSnSmallW; c2++)
                if (c2 < w) {
                    const T u = readlane(bv[c2], c);
                    if (below) bv[c2] = fma(-bv[c], u, bv[c2]);
                }
        }
    }
    // the factored block goes back here when the panel is one unit, else by the last unit to
    // finish (the others may still be reading the original block)
    if (un.z == 1) {
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++)
            if (c < w && lane < w) Fx[cb[c] + lane] = bv[c];
    }
    for (int r0 = rb; r0 < re; r0 += WAVE) {
        const int row = r0 + lane;
        const bool in = row < re;
        T x[kSnSmallW];
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++) x[c] = (in && c < w) ? Fx[cb[c] + w + row] : T(0);
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++) {
            if (c < w) {
                mx[c] = nanmax(mx[c], fabs((double)x[c]));
                x[c] = x[c] * recip(readlane(bv[c], c));
#pragma unroll
                for (int c2 = c + 1; c2 < kSnSmallW; c2++)
                    if (c2 < w) x[c2] = fma(-x[c], readlane(bv[c2], c), x[c2]);
            }
        }
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++)
            if (in && c < w) Fx[cb[c] + w + row] = x[c];
    }
    // column maxima over the wavefront: lane c keeps column c's
    double M = 0.0;
#pragma unroll
    for (int c = 0; c < kSnSmallW; c++) {
        if (c >= w) continue;
        double v = mx[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off));
        if (lane == c) M = v;
    }
    if (un.z > 1) {
        // slices meet as in the wide panels: the last unit to arrive takes the maxima of all
        // slices, writes the block back and runs the test
        double *pm = a.sn_pmax + ((size_t)un.w * a.batch + inst) * NB;
        const size_t pstride = (size_t)a.batch * NB;
        if (lane < w) pm[un.y * pstride + lane] = M;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int prev = 0;
        int *ctr = a.sn_pcnt + (size_t)un.x * a.batch + inst;
        if (lane == 0) prev = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prev = __shfl(prev, 0);
        if (prev != un.z - 1) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane < w)
            for (int p = 0; p < un.z; p++) M = nanmax(M, pm[p * pstride + lane]);
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++)
            if (c < w && lane < w) Fx[cb[c] + lane] = bv[c];
    }
    if (lane < w) {
        // lane c holds u_cc in bv[c]
        double piv = 0.0;
#pragma unroll
        for (int c = 0; c < kSnSmallW; c++)
            if (c == lane) piv = (double)bv[c];
        const int col = s0 + lane;
        if (a.check && (!isfinite(piv) || piv == 0.0 || !isfinite(M) || fabs(piv) < a.eps * M ||
                        col == a.force_fail_col))
            sn_fail(a, inst, lev, col);
        else
            a.done[(size_t)inst * a.n + col] = (int)a.epoch;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void sn_small_kernel(RefactorArgs a, int lev, int ubeg, int uend) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= (int64_t)(uend - ubeg) * a.batch) return;
    const int inst = (int)(w % a.batch);
    const int4 un = reinterpret_cast<const int4 *>(a.sn_sunit)[ubeg + (int)(w / a.batch)];
    const int4 rec = reinterpret_cast<const int4 *>(a.sn_su2)[ubeg + (int)(w / a.batch)];
    if (sn_stopped(a, inst, lev)) return;
    sn_small_panel<T>(a, inst, lev, rec.x, rec.y, rec.z, un, lane);
}

// Singleton supernodes: sixteen lanes per (column, instance), four entries per lane in flight:
// the pivot test on the values before division (their maximum over the sixteen lanes), then
// L = x / pivot, as one wavefront per column would.
template <typename T>
__global__ __launch_bounds__(256) void sn_single_kernel(RefactorArgs a, int lev, int sbeg, int send) {
    const int l16 = threadIdx.x & 15;
    const int64_t g = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
    if (g >= (int64_t)(send - sbeg) * a.batch) return;
    const int inst = (int)(g % a.batch);
    const int j = a.sn_rec[4 * a.sn_seq[sbeg + (int)(g / a.batch)]];
    if (sn_stopped(a, inst, lev)) return;                 // uniform over the sixteen lanes
    T *x = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF + a.Dp[j];
    const int nu = a.nU[j], len = a.Dlen[j];
    const T d = x[nu - 1];
    double m = 0.0;
    for (int i0 = nu; i0 < len; i0 += 64) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = i0 + 16 * u + l16 < len ? x[i0 + 16 * u + l16] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            m = nanmax(m, fabs((double)v[u]));
            if (i0 + 16 * u + l16 < len) x[i0 + 16 * u + l16] = v[u] / d;
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) m = nanmax(m, __shfl_xor(m, off, 16));
    if (l16 != 0) return;
    const double dd = (double)d;
    if (a.check && (!isfinite(dd) || dd == 0.0 || !isfinite(m) || fabs(dd) < a.eps * m || j == a.force_fail_col))
        sn_fail(a, inst, lev, j);
    else
        a.done[(size_t)inst * a.n + j] = (int)a.epoch;
}

// Supernode panels (w > kSnSmallW): one workgroup of eight wavefronts per (supernode, instance).
// The w x w diagonal block (padded with the identity) is factored without pivoting by the dense
// block's four-wavefront step (diag_factor_part; the other wavefronts wait at the same barriers)
// and written back; then L21 = A21 U11^-1 for the m rows of R, sixteen rows per wavefront per
// pass, by the block substitution of
// dlu_panel_kernel (X_b = (A_b - sum X_b' U_b'b) U_bb^-1 on the matrix cores).  The pivot
// test of column c is the dense block's: |u_cc| >= eps |u_cc| max_{i>c} |L(i,c)|, i.e. on
// the values L(i,c) u_cc before division.
constexpr int kSnPanelWaves = 8;                     // wavefronts of a panel workgroup (16 would spill)
template <typename T>
__global__ __launch_bounds__(kSnPanelWaves * WAVE) void sn_panel_kernel(RefactorArgs a, int lev, int ubeg) {
    typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
    __shared__ T blk[NB][NB + 1];
    __shared__ T invd[NB];
    __shared__ T winv[4][16][17];
    __shared__ T lbuf[4][WAVE];
    __shared__ double cmax[kSnPanelWaves][NB];
    __shared__ double dmax[kSnPanelWaves][NB];           // L11's column maxima, by slices of eight rows
    __shared__ int arrived;
    const int inst = blockIdx.y;
    if (sn_stopped(a, inst, lev)) return;                 // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int i16 = lane & 15, g = lane >> 4;
    const int4 un = reinterpret_cast<const int4 *>(a.sn_punit)[ubeg + (int)blockIdx.x];
    const int4 rec = reinterpret_cast<const int4 *>(a.sn_pu2)[ubeg + (int)blockIdx.x];
    const int s0 = rec.x, w = rec.y, m = rec.z;
    // this unit's rows of R: slice un.y of un.z
    const int rb = (int)((int64_t)m * un.y / un.z), re = (int)((int64_t)m * (un.y + 1) / un.z);
    const int *cb = a.sn_cb + s0;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    auto elem = [=](int c, int r) -> T { return (r < w && c < w) ? Fx[cb[c] + r] : (r == c ? T(1) : T(0)); };
    if (wv < 4) {
        diag_factor_elem<T>(elem, blk, invd, lbuf, wv);
    } else {
        for (int kk = 0; kk < NB; kk += 2) __syncthreads();   // the factorization's barriers, one per step
    }
    __syncthreads();
    // the factored block goes back to the factor storage here when the panel is one unit, else
    // by the last unit to finish (the others may still be reading the original block)
    if (un.z == 1)
        for (int e = tid; e < w * w; e += kSnPanelWaves * WAVE) {
            const int c = e / w, r = e - c * w;
            Fx[cb[c] + r] = blk[c][r];
        }
    if (wv < 4) {
        // inverse of U11's diagonal block b = wv (upper, from the bottom), column i16
        const int o = 16 * wv;
        T x[16];
#pragma unroll
        for (int i = 15; i >= 0; i--) {
            T acc = i == i16 ? T(1) : T(0);
#pragma unroll
            for (int k = i + 1; k < 16; k++) acc = fma(-blk[o + k][o + i], x[k], acc);
            x[i] = acc * invd[o + i];
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; i++) winv[wv][i][i16] = x[i];
        }
    }
    __syncthreads();
    double mx[4][4];
#pragma unroll
    for (int b = 0; b < 4; b++)
#pragma unroll
        for (int q = 0; q < 4; q++) mx[b][q] = 0.0;
    for (int r0 = rb + 16 * wv; r0 < re; r0 += 16 * kSnPanelWaves) {   // uniform per wavefront
        const int row = r0 + i16;
        const bool in = row < re;
        acc_t t[4];
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = 16 * b + kidx<T>(q, g);
                t[b][q] = (in && k < w) ? Fx[cb[k] + w + row] : T(0);
            }
        acc_t x[4];
#pragma unroll
        for (int b = 0; b < 4; b++) {
#pragma unroll
            for (int bp = 0; bp < b; bp++)
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const int k = 16 * bp + kidx<T>(s, g);
                    t[b] = mfma16<T>(-blk[16 * b + i16][k], x[bp][s], t[b]);   // (U_b'b)^T (i16, k)
                }
            acc_t z = {};
#pragma unroll
            for (int s = 0; s < 4; s++) z = mfma16<T>(winv[b][kidx<T>(s, g)][i16], t[b][s], z);
            x[b] = z;
        }
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = 16 * b + kidx<T>(q, g);
                if (in && k < w) {
                    Fx[cb[k] + w + row] = x[b][q];
                    mx[b][q] = nanmax(mx[b][q], fabs((double)x[b][q]));
                }
            }
    }
    // column maxima over the rows of R: across the sixteen lanes of a group, then wavefronts
#pragma unroll
    for (int b = 0; b < 4; b++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            double v = mx[b][q];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) v = nanmax(v, __shfl_xor(v, off));
            if (i16 == 0) cmax[wv][16 * b + kidx<T>(q, g)] = v;
        }
    __syncthreads();
    double M = 0.0;
    if (tid < w)
        for (int q = 0; q < kSnPanelWaves; q++) M = nanmax(M, cmax[q][tid]);
    if (un.z > 1) {
        // slices meet: each stores its column maxima and counts its arrival; the last one to
        // arrive takes the maxima of all slices (a maximum does not depend on their order),
        // writes the block back and runs the test
        double *pm = a.sn_pmax + ((size_t)un.w * a.batch + inst) * NB;
        const size_t pstride = (size_t)a.batch * NB;
        if (tid < w) pm[un.y * pstride + tid] = M;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            int *ctr = a.sn_pcnt + (size_t)un.x * a.batch + inst;
            const int prev = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            arrived = prev == un.z - 1;
            if (arrived) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!arrived) return;                            // uniform: read after the barrier
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (tid < w)
            for (int p = 0; p < un.z; p++) M = nanmax(M, pm[p * pstride + tid]);
        for (int e = tid; e < w * w; e += kSnPanelWaves * WAVE) {
            const int c = e / w, r = e - c * w;
            Fx[cb[c] + r] = blk[c][r];
        }
    }
    {
        // L11's column maxima below the diagonal: every thread takes eight rows of a column
        const int c = tid & (NB - 1), sl = tid / NB;
        double mm = 0.0;
#pragma unroll
        for (int u = 0; u < NB / kSnPanelWaves; u++) {
            const int r = (NB / kSnPanelWaves) * sl + u;
            if (c < w && r > c && r < w) mm = nanmax(mm, fabs((double)blk[c][r]));
        }
        dmax[sl][c] = mm;
    }
    __syncthreads();
    if (tid < w) {
        const int c = tid;
        for (int q = 0; q < kSnPanelWaves; q++) M = nanmax(M, dmax[q][c]);
        const double piv = (double)blk[c][c];
        const double xmax = fabs(piv) * M;
        const int col = s0 + c;
        if (a.check && (!isfinite(piv) || piv == 0.0 || !isfinite(xmax) || fabs(piv) < a.eps * xmax ||
                        col == a.force_fail_col))
            sn_fail(a, inst, lev, col);
        else
            a.done[(size_t)inst * a.n + col] = (int)a.epoch;
    }
}

// U(S, k) = L11^-1 x_k(S) on the suffix of S's rows present in k (len rows; lane c holds row
// c), eight L11 loads in flight; returns this lane's value.  cbv: lane c holds the storage
// offset of the suffix's column c (read by readlane, no dependent load).
template <typename T>
__device__ __forceinline__ T sn_suffix_solve(const T *Fx, const T *xk, int cbv, int slot0, int off, int len,
                                             int lane) {
    T xv = lane < len ? xk[slot0 + lane] : T(0);
    for (int c0 = 0; c0 < len; c0 += 8) {
        T lv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = c0 + u;
            const int base = __builtin_amdgcn_readlane(cbv, c < len ? c : 0);
            lv[u] = (c < len && lane > c && lane < len) ? Fx[base + off + lane] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = c0 + u;
            if (c < len) {
                const T uc = readlane(xv, c);
                if (lane > c) xv = fma(-lv[u], uc, xv);
            }
        }
    }
    return xv;
}

// Sums over the suffix's columns [c_lo, c_hi) of L21(row, c) u_c for the rows r0 + lane and
// r0 + 64 + lane of R (two rows per lane, sixteen loads in flight).  u_c comes from get(c)
// (a readlane or an LDS read), the column offsets from cbv as above.
template <typename T, typename GetU>
__device__ __forceinline__ void sn_rows_partial(const T *Fx, int cbv, int w, int c_lo, int c_hi, int mcnt, int r0,
                                                int lane, GetU get, T &acca, T &accb) {
    const int ra = r0 + lane, rb = r0 + WAVE + lane;
    const bool ina = ra < mcnt, inb = rb < mcnt;
    acca = T(0);
    accb = T(0);
    for (int c0 = c_lo; c0 < c_hi; c0 += 8) {
        T la[8], lb[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = c0 + u;
            const int base = __builtin_amdgcn_readlane(cbv, c < c_hi ? c : c_lo) + w;
            la[u] = (ina && c < c_hi) ? Fx[base + ra] : T(0);
            lb[u] = (inb && c < c_hi) ? Fx[base + rb] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (c0 + u < c_hi) {
                const T uc = get(c0 + u);
                acca = fma(la[u], uc, acca);
                accb = fma(lb[u], uc, accb);
            }
    }
}

// x_k(R rows r0 + lane, r0 + 64 + lane) -= the sums above over all len columns; the rows'
// slots in k from mp.
template <typename T, typename GetU>
__device__ __forceinline__ void sn_rows_update(const T *Fx, T *xk, int cbv, const int *mp, int w, int len, int mcnt,
                                               int r0, int lane, GetU get) {
    const int ra = r0 + lane, rb = r0 + WAVE + lane;
    const int sla = ra < mcnt ? mp[ra] : 0, slb = rb < mcnt ? mp[rb] : 0;
    T acca, accb;
    sn_rows_partial<T>(Fx, cbv, w, 0, len, mcnt, r0, lane, get, acca, accb);
    if (ra < mcnt) xk[sla] -= acca;
    if (rb < mcnt) xk[slb] -= accb;
}

constexpr int kHeavyChunk = 16;                      // entries of a heavy group whose suffixes are solved together

// A heavy group (up to kGroupTargets target columns sharing most of their sources; one
// workgroup per (group, instance)).  Its sources are taken in ascending order, in chunks of at
// most kHeavyChunk (source, target) entries.  A chunk's suffix solves U(S, k) = L11^-1 x_k(S) go
// first, a wavefront each: they are independent of every row update of the level (its
// supernodes hold no rows of each other's R).  Then each source of the chunk, in order, reads
// its rows of R once for all the group's targets it reaches: x_k(R) -= L21 U(S, k) for each of
// them (its suffix columns only, in ascending order: each target row gets the operations of a
// single-target task in the same order), two rows per lane, R's rows split over the four
// wavefronts, a barrier between sources (their rows of R may meet in a target).
template <typename T, bool PF>
__device__ void sn_heavy_group(const RefactorArgs &a, int inst, int g, T (*us)[WAVE], int *gdp, int *eoff, int *edp,
                               int64_t *emoff, int lane, int wv) {
    const int tid = threadIdx.x;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int4 gr = reinterpret_cast<const int4 *>(a.sn_grp)[g];
    const int4 *gsrc = reinterpret_cast<const int4 *>(a.sn_gsrc);
    const int2 *gent = reinterpret_cast<const int2 *>(a.sn_gent);
    if (tid < gr.y) gdp[tid] = a.sn_task[4 * (gr.x + tid) + 1];
    __syncthreads();
    for (int s0r = gr.z; s0r < gr.w;) {
        // the chunk: sources [s0r, s1r) with at most kHeavyChunk entries (a source has at most
        // kGroupTargets of them)
        const int e_lo = gsrc[s0r].y;
        int s1r = s0r, e_hi = e_lo;
        while (s1r < gr.w && gsrc[s1r].y + gsrc[s1r].z - e_lo <= kHeavyChunk) {
            e_hi = gsrc[s1r].y + gsrc[s1r].z;
            s1r++;
        }
        for (int e = e_lo + wv; e < e_hi; e += 4) {       // uniform per wavefront
            const int2 en = gent[e];
            const int4 item = reinterpret_cast<const int4 *>(a.sn_item)[en.y];
            const int4 rec = reinterpret_cast<const int4 *>(a.sn_rec)[item.x];
            const int len = item.z, off = rec.y - len;
            T *xk = Fx + gdp[en.x];
            const int cbv = lane < len ? a.sn_cb[rec.x + off + lane] : 0;
            const T xv = sn_suffix_solve<T>(Fx, xk, cbv, item.y, off, len, lane);
            if (lane < len) {
                xk[item.y + lane] = xv;
                us[e - e_lo][off + lane] = xv;
            }
            if (lane < off) us[e - e_lo][lane] = T(0);
            if (lane == 0) {
                eoff[e - e_lo] = off;
                edp[e - e_lo] = gdp[en.x];
                emoff[e - e_lo] = a.sn_moff[en.y];
            }
        }
        __syncthreads();
        for (int sr = s0r; sr < s1r; sr++) {
            const int4 src = gsrc[sr];
            const int4 rec = reinterpret_cast<const int4 *>(a.sn_rec)[src.x];
            const int w = rec.y, ns = src.z, mcnt = src.w, e0 = src.y - e_lo;
            int ej[kGroupTargets];                       // first suffix column per target (w: none)
            int offmin = w;
#pragma unroll
            for (int j = 0; j < kGroupTargets; j++) {
                ej[j] = j < ns ? eoff[e0 + j] : w;
                offmin = min(offmin, ej[j]);
            }
            const int cbv = lane < w ? a.sn_cb[rec.x + lane] : 0;   // S's columns
            for (int r0 = 2 * WAVE * wv; r0 < mcnt; r0 += 8 * WAVE) {
                const int ra = r0 + lane, rb = r0 + WAVE + lane;
                const bool ina = ra < mcnt, inb = rb < mcnt;
                // PF: the pass's target slots and their values go out first, with the
                // columns' loads (the write-back then waits on no load): nothing else writes
                // them during the pass (the source's rows are distinct, the group's sources are
                // apart by a barrier, no other supernode of the level holds rows of R), so
                // x - sum stores the same bits as the read-modify-write at the end
                int sa[kGroupTargets], sb[kGroupTargets];
                T xa[kGroupTargets], xb[kGroupTargets];
                if constexpr (PF) {
#pragma unroll
                    for (int j = 0; j < kGroupTargets; j++) {
                        const int *mp = a.sn_map + emoff[e0 + j];
                        sa[j] = (j < ns && ina) ? mp[ra] : 0;
                        sb[j] = (j < ns && inb) ? mp[rb] : 0;
                    }
#pragma unroll
                    for (int j = 0; j < kGroupTargets; j++) {
                        const T *xk = Fx + edp[e0 + j];
                        xa[j] = (j < ns && ina) ? xk[sa[j]] : T(0);
                        xb[j] = (j < ns && inb) ? xk[sb[j]] : T(0);
                    }
                }
                T acca[kGroupTargets], accb[kGroupTargets];
#pragma unroll
                for (int j = 0; j < kGroupTargets; j++) acca[j] = accb[j] = T(0);
                for (int c0 = offmin; c0 < w; c0 += 8) {
                    T la[8], lb[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const int c = c0 + u;
                        const int base = __builtin_amdgcn_readlane(cbv, c < w ? c : offmin) + w;
                        la[u] = (ina && c < w) ? Fx[base + ra] : T(0);
                        lb[u] = (inb && c < w) ? Fx[base + rb] : T(0);
                    }
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const int c = c0 + u;
                        if (c < w) {
#pragma unroll
                            for (int j = 0; j < kGroupTargets; j++)
                                if (c >= ej[j]) {
                                    const T uc = us[e0 + j][c];
                                    acca[j] = fma(la[u], uc, acca[j]);
                                    accb[j] = fma(lb[u], uc, accb[j]);
                                }
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < kGroupTargets; j++)
                    if (j < ns) {
                        T *xk = Fx + edp[e0 + j];
                        if constexpr (PF) {
                            if (ina) xk[sa[j]] = xa[j] - acca[j];
                            if (inb) xk[sb[j]] = xb[j] - accb[j];
                        } else {
                            const int *mp = a.sn_map + emoff[e0 + j];
                            if (ina) xk[mp[ra]] -= acca[j];
                            if (inb) xk[mp[rb]] -= accb[j];
                        }
                    }
            }
            __syncthreads();
        }
        s0r = s1r;
    }
}

// Update tasks of a level: a task owns one target column k and applies the level's
// supernodes S with U(S, k) != 0 in ascending order.  Per supernode: U(S, k) = L11^-1 x_k(S)
// on the suffix of S's rows present in k, written to k; then x_k(R) -= L21 U(S, k) on R's
// rows (rows < T only for a dense-block target: its rows >= T are the Schur update's), their
// slots in k from sn_map.  Rows of one supernode are distinct, so the stores of one pass
// never feed its own loads.  Heavy tasks come in groups sn_grp [gbeg, ...) (nheavy
// workgroups: groups x instances, see sn_heavy_group); tasks [theavy, ttiny) get a wavefront
// per (task, instance), [ttiny, tend) sixteen lanes.  Every way, each row of k receives the
// same operations in the same order.
template <typename T, bool PF>
__global__ __launch_bounds__(256) void sn_update_kernel(RefactorArgs a, int lev, int gbeg, int theavy, int ttiny,
                                                        int tend, unsigned nheavy) {
    __shared__ T us[kHeavyChunk][WAVE];
    __shared__ int gdp[kGroupTargets];
    __shared__ int eoff[kHeavyChunk], edp[kHeavyChunk];
    __shared__ int64_t emoff[kHeavyChunk];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    // grid sizes fit 32 bits (one dimension of a launch); nheavy = heavy groups x instances
    const unsigned nlight = ((unsigned)(ttiny - theavy) * (unsigned)a.batch + 3) / 4;
    const unsigned bid = blockIdx.x, batch = (unsigned)a.batch;
    int t, inst;
    if (bid < nheavy) {
        const unsigned b = xcd_contiguous(bid, nheavy);
        inst = (int)(b % batch);
        if (sn_stopped(a, inst, lev)) return;            // uniform over the workgroup
        sn_heavy_group<T, PF>(a, inst, gbeg + (int)(b / batch), us, gdp, eoff, edp, emoff, lane, wv);
        return;
    } else if (bid < nheavy + nlight) {
        const unsigned wid = xcd_contiguous(bid - nheavy, nlight) * 4 + wv;
        if (wid >= (unsigned)(ttiny - theavy) * batch) return;
        inst = (int)(wid % batch);
        t = theavy + (int)(wid / batch);
    } else {
        // tiny tasks (every item at most kTinyRows suffix rows and kTinyRowsR rows of R):
        // sixteen lanes each, the same operations in the same order as a wavefront's: the
        // suffix solve with lane c holding suffix row c, then two rows of R per lane and pass.
        // Lane c holds the suffix's column c offset (shuffled, not re-read); eight columns'
        // loads go out before their multiply-adds
        const unsigned ntiny = gridDim.x - nheavy - nlight;
        const unsigned gid = xcd_contiguous(bid - nheavy - nlight, ntiny) * 16 + threadIdx.x / 16;
        if (gid >= (unsigned)(tend - ttiny) * batch) return;
        inst = (int)(gid % batch);
        if (sn_stopped(a, inst, lev)) return;
        const int l16 = lane & 15;
        T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
        const int4 tk = reinterpret_cast<const int4 *>(a.sn_task)[ttiny + (int)(gid / batch)];
        T *xk = Fx + tk.y;
        const int4 *items = reinterpret_cast<const int4 *>(a.sn_item);
        const int4 *items2 = reinterpret_cast<const int4 *>(a.sn_item2);
        for (int it = tk.z; it < tk.w; it++) {
            const int4 item = items[it], it2 = items2[it];
            const int w = it2.y, len = item.z, off = w - len, mcnt = item.w;
            const int cbl = l16 < len ? a.sn_cb[it2.x + l16] : 0;   // the suffix's columns
            const int *mp = a.sn_map + (int64_t)(((uint64_t)(uint32_t)it2.w << 32) | (uint32_t)it2.z);
            T xv = l16 < len ? xk[item.y + l16] : T(0);
            // every lane of the group takes part in the shuffles (a shuffle reads active lanes);
            // the loop bounds are the group's own
            for (int c0 = 0; c0 < len; c0 += 8) {
                T lv[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = c0 + u;
                    const int base = __shfl(cbl, c & 15, 16);
                    lv[u] = (c < len && l16 > c && l16 < len) ? Fx[base + off + l16] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = c0 + u;
                    if (c < len - 1) {
                        const T uc = __shfl(xv, c, 16);
                        if (l16 > c && l16 < len) xv = fma(-lv[u], uc, xv);
                    }
                }
            }
            if (l16 < len) xk[item.y + l16] = xv;
            for (int r0 = 0; r0 < mcnt; r0 += 32) {
                const int ra = r0 + l16, rb = r0 + 16 + l16;
                const bool ina = ra < mcnt, inb = rb < mcnt;
                const int sla = ina ? mp[ra] : 0, slb = inb ? mp[rb] : 0;
                T acca = T(0), accb = T(0);
                for (int c0 = 0; c0 < len; c0 += 8) {
                    T la[8], lb[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const int c = c0 + u;
                        const int base = __shfl(cbl, c & 15, 16) + w;
                        la[u] = (c < len && ina) ? Fx[base + ra] : T(0);
                        lb[u] = (c < len && inb) ? Fx[base + rb] : T(0);
                    }
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const int c = c0 + u;
                        if (c < len) {
                            const T uc = __shfl(xv, c, 16);
                            acca = fma(la[u], uc, acca);
                            accb = fma(lb[u], uc, accb);
                        }
                    }
                }
                if (ina) xk[sla] -= acca;
                if (inb) xk[slb] -= accb;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        return;
    }
    if (sn_stopped(a, inst, lev)) return;
    T *Fx = reinterpret_cast<T *>(a.Fx) + (size_t)inst * a.nnzF;
    const int4 tk = reinterpret_cast<const int4 *>(a.sn_task)[t];
    T *xk = Fx + tk.y;
    const int4 *items = reinterpret_cast<const int4 *>(a.sn_item);
    const int4 *items2 = reinterpret_cast<const int4 *>(a.sn_item2);
    for (int it = tk.z; it < tk.w; it++) {
        const int4 item = items[it], it2 = items2[it];
        const int w = it2.y, len = item.z, off = w - len, mcnt = item.w;
        const int cbv = lane < len ? a.sn_cb[it2.x + lane] : 0;   // the suffix's columns
        const int *mp = a.sn_map + (int64_t)(((uint64_t)(uint32_t)it2.w << 32) | (uint32_t)it2.z);
        const T xv = sn_suffix_solve<T>(Fx, xk, cbv, item.y, off, len, lane);
        if (lane < len) xk[item.y + lane] = xv;
        for (int r0 = 0; r0 < mcnt; r0 += 2 * WAVE)
            sn_rows_update<T>(Fx, xk, cbv, mp, w, len, mcnt, r0, lane, [&](int c) { return readlane(xv, c); });
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

int launch_dense_gather(const DenseArgs &a, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.D <= 0) return 0;
    const dim3 gw = wave_grid((int64_t)a.D * a.batch);
    if (a.fp32) hipLaunchKernelGGL((tail_gather_kernel<float>), gw, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((tail_gather_kernel<double>), gw, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

int launch_schur(const DenseArgs &a, const int *parts, int nparts, const int *add, int nadd, const int *l21,
                 void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.D <= 0 || a.T <= 0 || nparts <= 0) return 0;
    // in place (part 0) or in scratch: a column in LDS would limit the resident wavefronts
    const dim3 grid((unsigned)((int64_t)nparts * a.batch));
    if (a.fp32) hipLaunchKernelGGL((schur_kernel<float>), grid, dim3(64), 0, st, a, parts, l21);
    else hipLaunchKernelGGL((schur_kernel<double>), grid, dim3(64), 0, st, a, parts, l21);
    if (nadd > 0) {
        const dim3 ga((unsigned)(((int64_t)nadd * a.batch + 3) / 4));
        if (a.fp32) hipLaunchKernelGGL((schur_add_kernel<float>), ga, dim3(256), 0, st, a, add, nadd);
        else hipLaunchKernelGGL((schur_add_kernel<double>), ga, dim3(256), 0, st, a, add, nadd);
    }
    return (int)hipGetLastError();
}

int launch_schur_sn(const DenseArgs &a, const int *parts, int nparts, const int *add, int nadd, const int *sn_items,
                    const int *sn_rec, const int *sn_cb, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (a.D <= 0 || a.T <= 0 || nparts <= 0) return 0;
    const dim3 grid((unsigned)((int64_t)nparts * a.batch));
    if (a.fp32) hipLaunchKernelGGL((schur_sn_kernel<float>), grid, dim3(64), 0, st, a, parts, sn_items, sn_rec, sn_cb);
    else hipLaunchKernelGGL((schur_sn_kernel<double>), grid, dim3(64), 0, st, a, parts, sn_items, sn_rec, sn_cb);
    if (nadd > 0) {
        const dim3 ga((unsigned)(((int64_t)nadd * a.batch + 3) / 4));
        if (a.fp32) hipLaunchKernelGGL((schur_add_kernel<float>), ga, dim3(256), 0, st, a, add, nadd);
        else hipLaunchKernelGGL((schur_add_kernel<double>), ga, dim3(256), 0, st, a, add, nadd);
    }
    return (int)hipGetLastError();
}

int dense_lookahead_events(const DenseArgs &a) {
    const int groups = (a.D + a.W - 1) / a.W;
    return groups >= 2 ? 2 * (groups - 1) : 0;
}

int launch_dense_refactor(const DenseArgs &a, bool gather, const DenseStreams *la, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int D = a.D;
    if (D <= 0) return 0;
    const dim3 gw = wave_grid((int64_t)D * a.batch);
    if (gather) {
        const int e = launch_dense_gather(a, stream);
        if (e) return e;
    }
    // groups of W columns: each panel of 64 updates the rest of its group (the column strip
    // below and right of it, the row strip right of the group); the whole trailing block
    // is updated once per group with K = W
    auto rect = [](int r0, int r1, int c0, int c1, int tm = 128) {
        GemmRect g;
        g.r0 = r0; g.r1 = r1; g.c0 = c0; g.c1 = c1;
        g.ntx = r1 > r0 && c1 > c0 ? (r1 - r0 + tm - 1) / tm : 0;
        g.nt = g.ntx ? g.ntx * ((c1 - c0 + tm - 1) / tm) : 0;
        return g;
    };
    auto gemm = [&](hipStream_t s, int kp, int kw, const GemmRect &g0, const GemmRect &g1, int dgp) {
        const dim3 gg((unsigned)(g0.nt + g1.nt), 1, (unsigned)a.batch);
        if (kw == 64) {
            if (a.fp32) hipLaunchKernelGGL((dlu_gemm_kernel<float, 64>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
            else hipLaunchKernelGGL((dlu_gemm_kernel<double, 64>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
        } else if (kw == 128) {
            if (a.fp32) hipLaunchKernelGGL((dlu_gemm_kernel<float, 128>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
            else hipLaunchKernelGGL((dlu_gemm_kernel<double, 128>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
        } else {
            if (a.fp32) hipLaunchKernelGGL((dlu_gemm_kernel<float, 256>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
            else hipLaunchKernelGGL((dlu_gemm_kernel<double, 256>), gg, dim3(256), 0, s, a, kp, g0, g1, dgp);
        }
    };
    // the panels of the group [p, pe) and the updates inside the group
    auto chain = [&](hipStream_t s, int p, int pe) {
        for (int q = p; q < pe; q += NB) {
            const int nb = D - q < NB ? D - q : NB;
            const int rest = D - q - nb;               // > 0 only for full panels
            const int nrb = (rest + 63) / 64, ncb = (rest + 63) / 64;
            const dim3 gp((unsigned)(1 + nrb + ncb), (unsigned)a.batch);
            if (a.fp32) hipLaunchKernelGGL((dlu_panel_kernel<float>), gp, dim3(256), 0, s, a, q, nrb);
            else hipLaunchKernelGGL((dlu_panel_kernel<double>), gp, dim3(256), 0, s, a, q, nrb);
            const int q1 = q + NB;
            if (q1 < pe) {                             // the in-group update: 64 x 64 tiles
                const GemmRect g0 = rect(q1, D, q1, pe, 64), g1 = rect(q1, pe, pe, D, 64);
                const dim3 gg((unsigned)(g0.nt + g1.nt), 1, (unsigned)a.batch);
                if (a.fp32) hipLaunchKernelGGL((dlu_gemm_kernel<float, 64, 64>), gg, dim3(256), 0, s, a, q, g0, g1, q);
                else hipLaunchKernelGGL((dlu_gemm_kernel<double, 64, 64>), gg, dim3(256), 0, s, a, q, g0, g1, q);
            }
        }
    };
    const int W = a.W;
    const int nev = dense_lookahead_events(a);
    if (!la || !la->side || nev == 0 || la->nev < nev) {
        for (int p = 0; p < D; p += W) {
            const int pe = D - p < W ? D : p + W;
            chain(st, p, pe);
            if (pe < D) gemm(st, p, pe - p, rect(pe, D, pe, D), rect(0, 0, 0, 0), pe - NB);
        }
    } else {
        // look-ahead: after group g, its update of the next group's columns and rows comes
        // first; the next group's panels then run on the side stream while the rest of
        // the trailing block is updated here.  The two touch disjoint parts of S: the
        // panels and in-group updates of group g+1 stay in its rows or columns, the rest
        // of the update stays in rows and columns past it.
        hipStream_t sd = (hipStream_t)la->side;
        chain(st, 0, W);
        for (int g = 0, p = 0; p + W < D; g++, p += W) {
            const int pe = p + W, pe2 = D - pe < W ? D : pe + W;
            gemm(st, p, W, rect(pe, D, pe, pe2), rect(pe, pe2, pe2, D), pe - NB);
            hipEvent_t e0 = (hipEvent_t)la->ev[2 * g], e1 = (hipEvent_t)la->ev[2 * g + 1];
            hipError_t err = hipEventRecord(e0, st);
            if (err == hipSuccess) err = hipStreamWaitEvent(sd, e0, 0);
            if (err != hipSuccess) return (int)err;
            chain(sd, pe, pe2);
            if ((err = hipEventRecord(e1, sd)) != hipSuccess) return (int)err;
            if (pe2 < D) gemm(st, p, W, rect(pe2, D, pe2, D), rect(0, 0, 0, 0), -1);
            if ((err = hipStreamWaitEvent(st, e1, 0)) != hipSuccess) return (int)err;
        }
    }
    if (a.check) {
        if (a.fp32) hipLaunchKernelGGL((dlu_check_kernel<float>), gw, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((dlu_check_kernel<double>), gw, dim3(256), 0, st, a);
    }
    if (a.fp32) hipLaunchKernelGGL((tail_scatter_kernel<float>), gw, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((tail_scatter_kernel<double>), gw, dim3(256), 0, st, a);
    const int e = (int)hipGetLastError();
    return e ? e : launch_dense_inverses(a, stream);
}

int launch_dense_pivoted_lu(const DenseArgs &a, int *swp, int *info, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int D = a.D;
    if (D <= 0) return 0;
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, info);
    auto rect = [](int r0, int r1, int c0, int c1) {
        GemmRect g;
        g.r0 = r0; g.r1 = r1; g.c0 = c0; g.c1 = c1;
        g.ntx = r1 > r0 && c1 > c0 ? (r1 - r0 + 127) / 128 : 0;
        g.nt = g.ntx ? g.ntx * ((c1 - c0 + 127) / 128) : 0;
        return g;
    };
    for (int p = 0; p < D; p += NB) {
        const int pe = D - p < NB ? D : p + NB;
        for (int k = p; k <= pe; k++) {
            const int roles = k < pe ? 2 + (pe - k - 1) : 1;
            hipLaunchKernelGGL(dpiv_step_kernel, dim3((unsigned)roles), dim3(256), 0, st, a, p, pe, k, swp, info);
        }
        const int nrest = p + (D - pe);
        if (nrest > 0)
            hipLaunchKernelGGL(dpiv_swap_rest_kernel, dim3((unsigned)((nrest + NB - 1) / NB)), dim3(NB), 0, st, a, p,
                               pe, (const int *)swp);
        if (pe < D) {
            hipLaunchKernelGGL(dpiv_u12_kernel, dim3((unsigned)((D - pe + 255) / 256)), dim3(256), 0, st, a, p);
            const GemmRect g0 = rect(pe, D, pe, D), g1 = rect(0, 0, 0, 0);
            hipLaunchKernelGGL((dlu_gemm_kernel<double, 64>), dim3((unsigned)g0.nt, 1, 1), dim3(256), 0, st, a, p, g0,
                               g1, -1);
        }
    }
    return (int)hipGetLastError();
}

int launch_dense_inverses(const DenseArgs &a, void *stream) {
    if (a.D <= 0) return 0;
    const dim3 g((unsigned)((a.D + NB - 1) / NB), (unsigned)a.batch);
    if (a.fp32) hipLaunchKernelGGL((dlu_inverse_kernel<float>), g, dim3(NB), 0, (hipStream_t)stream, a);
    else hipLaunchKernelGGL((dlu_inverse_kernel<double>), g, dim3(NB), 0, (hipStream_t)stream, a);
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

int launch_sn_panels(const RefactorArgs &a, int lev, int sbeg, int s1, int sub, int sue, int ubeg, int uend,
                     void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t groups = (int64_t)(s1 - sbeg) * a.batch;   // sixteen lanes each
    if (groups > 0) {
        const dim3 grid((unsigned)((groups + 15) / 16));
        if (a.fp32) hipLaunchKernelGGL(sn_single_kernel<float>, grid, dim3(256), 0, st, a, lev, sbeg, s1);
        else hipLaunchKernelGGL(sn_single_kernel<double>, grid, dim3(256), 0, st, a, lev, sbeg, s1);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    const int64_t swaves = (int64_t)(sue - sub) * a.batch;
    if (swaves > 0) {
        const dim3 grid((unsigned)((swaves + 3) / 4));
        if (a.fp32) hipLaunchKernelGGL(sn_small_kernel<float>, grid, dim3(256), 0, st, a, lev, sub, sue);
        else hipLaunchKernelGGL(sn_small_kernel<double>, grid, dim3(256), 0, st, a, lev, sub, sue);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    if (uend > ubeg) {
        const dim3 grid((unsigned)(uend - ubeg), (unsigned)a.batch);
        const dim3 block(kSnPanelWaves * WAVE);
        if (a.fp32) hipLaunchKernelGGL(sn_panel_kernel<float>, grid, block, 0, st, a, lev, ubeg);
        else hipLaunchKernelGGL(sn_panel_kernel<double>, grid, block, 0, st, a, lev, ubeg);
    }
    return (int)hipGetLastError();
}

int launch_sn_updates(const RefactorArgs &a, int lev, int gbeg, int gend, int theavy, int ttiny, int tend,
                      void *stream) {
    const int64_t heavy = (int64_t)(gend - gbeg) * a.batch;
    const int64_t light = ((int64_t)(ttiny - theavy) * a.batch + 3) / 4;
    const int64_t tiny = ((int64_t)(tend - ttiny) * a.batch + 15) / 16;
    if (heavy + light + tiny == 0) return 0;
    if (heavy + light + tiny > INT_MAX || (int64_t)(tend - theavy) * a.batch > INT_MAX) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)(heavy + light + tiny));
    // a launch whose wavefronts all fit on the chip at four per SIMD (MI355X: 256 CUs of four
    // SIMDs; the upper separators' levels of a few hundred heavy groups) takes the kernel that
    // loads each pass's target slots and values up front, in registers that leave room for
    // four wavefronts per SIMD; a larger launch needs the occupancy of the other.  The same
    // operations in the same order either way
    const bool pf = (heavy + light + tiny) * 4 <= 256 * 4 * 4;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, (hipStream_t)stream, a, lev, gbeg, theavy, ttiny, tend,
                           (unsigned)heavy);
    };
    if (a.fp32) pf ? go(sn_update_kernel<float, true>) : go(sn_update_kernel<float, false>);
    else pf ? go(sn_update_kernel<double, true>) : go(sn_update_kernel<double, false>);
    return (int)hipGetLastError();
}

}  // namespace cktlu_dev
