// solve.hip -- a consumer of the GEMM: mixed-precision iterative refinement
// for A X = B (the technique the paper puts its precision refinement next
// to, Sec. V), with the O(n^3) work of the factorisation on the matrix
// cores through mfg_gemm.
//
//   LU:  right-looking blocked LU with partial pivoting of an FP32 copy of
//        A, panels of kNb = 64 columns: the panel is factored by one
//        workgroup (column by column: pivot search, row swap, scaling by
//        the pivot's reciprocal as in LAPACK's unblocked LU,
//        rank-1 update of the panel), its row swaps are applied to the rest
//        of the matrix, the block row is solved with the panel's unit lower
//        triangle (U12 = L11^-1 A12), and the trailing matrix is updated
//        A22 -= L21 U12 by one mfg_gemm call in the caller's mode (F32, F16,
//        or a refined split: the precision of the factorisation).
//   solve with the factors: the row permutation (one gather), then forward
//        and backward substitution by blocks of kNb rows, one launch per
//        block: the diagonal block solved in every workgroup, the rest of
//        the right-hand side updated in the same launch.
//   refinement: x0 from the factors; then r = b - A x in FP64, the normwise
//        backward error max_j |r_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf),
//        and while it is above the tolerance a correction d solved in FP32
//        from r and x += d in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "runtime.h"

namespace mfg {

namespace {

constexpr int kNb = 64;
constexpr int kPanelThreads = 1024;

// One panel A[j:n, j:j+w] (w <= kNb), factored in place with partial pivoting.
// ipiv[j + c] receives the row swapped with row j + c (0-based); info (if no
// earlier column had one) the 1-based index of the first exactly-zero pivot.
__global__ __launch_bounds__(kPanelThreads) void lu_panel(int64_t n, float* A, int64_t lda, int64_t j, int w,
                                                         int32_t* ipiv, int32_t* info) {
    __shared__ float prow[kNb];
    __shared__ float wv[kPanelThreads / 64];
    __shared__ int64_t wi[kPanelThreads / 64];
    __shared__ int64_t piv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int c = 0; c < w; ++c) {
        const int64_t col = j + c;
        // pivot: the largest |A[r, col]| over r >= col, the first such row on ties
        float best = -1.0f;
        int64_t bi = n;
        for (int64_t r = col + tid; r < n; r += kPanelThreads) {
            const float v = fabsf(A[r * lda + col]);
            if (v > best) best = v, bi = r;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(best, off);
            const int64_t oi = __shfl_xor(bi, off);
            if (ov > best || (ov == best && oi < bi)) best = ov, bi = oi;
        }
        if (lane == 0) wv[wave] = best, wi[wave] = bi;
        __syncthreads();
        if (tid == 0) {
            float b = wv[0];
            int64_t i = wi[0];
            for (int q = 1; q < kPanelThreads / 64; ++q)
                if (wv[q] > b || (wv[q] == b && wi[q] < i)) b = wv[q], i = wi[q];
            if (i >= n) i = col;  // (a column of NaNs only: keep the diagonal)
            piv = i;
            ipiv[col] = (int32_t)i;
            if (A[i * lda + col] == 0.0f && *info == 0) *info = (int32_t)(col + 1);
        }
        __syncthreads();
        const int64_t p = piv;
        if (p != col && tid < w) {
            const float t = A[col * lda + j + tid];
            A[col * lda + j + tid] = A[p * lda + j + tid];
            A[p * lda + j + tid] = t;
        }
        __syncthreads();
        if (tid < w) prow[tid] = A[col * lda + j + tid];
        __syncthreads();
        const float pv = prow[c];
        if (pv != 0.0f) {
            const float rp = 1.0f / pv;  // the column is scaled by the pivot's reciprocal
            for (int64_t r = col + 1 + tid; r < n; r += kPanelThreads) {
                float* row = A + r * lda + j;
                const float l = row[c] * rp;
                row[c] = l;
                for (int cc = c + 1; cc < w; ++cc) row[cc] = __builtin_fmaf(-l, prow[cc], row[cc]);
            }
        }
        __syncthreads();
    }
}

// A narrow panel A[j:n, j:j+w] (w <= 8), copied by lu_gather8 into the
// contiguous rows x 8 array W, held in registers for all of its columns:
// thread t owns panel rows i = t + kP8Threads q (row j + i), q < kP8Rows (so
// rows = n - j <= kP8Threads kP8Rows).  One barrier per column c:
//   - each wavefront finds its largest |value| among its rows at or below the
//     diagonal (first row on ties; value and row then packed in one key); lane 0
//     writes the key and the lane owning that row the row's values to the
//     wavefront's LDS slot, and thread c (owner of the diagonal row, q = 0)
//     writes that row;
//   - after the barrier every thread reduces the slots by the same rule, so
//     each knows the pivot row p and both rows to exchange; their owners swap
//     them in registers, and every owned row below the diagonal is scaled by
//     the pivot and gets the rank-1 update of the columns to its right.
// The slots alternate between two LDS buffers by column parity: a buffer is
// written again two columns later, by threads that passed the barrier of the
// column in between, which every thread reaches only after reading it.  Rows
// move in and out of W as two 16-byte pieces; lu_subpanel_post writes the
// factored columns back.  Same arithmetic, operation by operation, as lu_panel.
constexpr int kP8 = 8, kP8Threads = 512, kP8Rows = 16, kP8Waves = kP8Threads / 64;

// Pivot candidates as one 64-bit key: the bits of |value| (non-negative
// floats order as their bit patterns) above the complement of the row, so
// the larger value wins and the lower row on ties in one unsigned compare;
// 0 is "no candidate" (a NaN, a row above the diagonal or past the matrix).
using P8Key = unsigned long long;
__device__ __forceinline__ P8Key p8_key(float a, int i) {
    return ((P8Key)__builtin_bit_cast(uint32_t, a) << 32) | (P8Key)(~(uint32_t)i);
}

// One step of the key max across lanes: the partner lane given by the DPP
// control CTRL.
template <int CTRL>
__device__ __forceinline__ void p8_dpp_max(P8Key& k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)k, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(k >> 32), CTRL, 0xF, 0xF, false);
    const P8Key o = ((P8Key)hi << 32) | lo;
    k = o > k ? o : k;
}

__device__ __forceinline__ P8Key p8_lane_key(P8Key k, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), lane);
    return ((P8Key)hi << 32) | lo;
}

__global__ __launch_bounds__(kP8Threads) void lu_panel8(int rows, float* W, int64_t j, int w, int32_t* ipiv,
                                                       int32_t* info) {
    __shared__ P8Key skey[2][kP8Waves];
    __shared__ __attribute__((aligned(16))) float srow[2][kP8Waves][kP8];
    __shared__ __attribute__((aligned(16))) float sdiag[2][kP8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float x[kP8Rows][kP8];
#pragma unroll
    for (int q = 0; q < kP8Rows; ++q) {
        const int i = tid + kP8Threads * q;
        float4 u = make_float4(0.0f, 0.0f, 0.0f, 0.0f), v = u;
        if (i < rows) {
            const float4* rp = reinterpret_cast<const float4*>(W + (int64_t)i * kP8);
            u = rp[0], v = rp[1];
        }
        x[q][0] = u.x, x[q][1] = u.y, x[q][2] = u.z, x[q][3] = u.w;
        x[q][4] = v.x, x[q][5] = v.y, x[q][6] = v.z, x[q][7] = v.w;
    }
#pragma unroll
    for (int c = 0; c < kP8; ++c) {
        if (c >= w) break;
        const int buf = c & 1;
        // the thread's candidate: its largest |value| at or below the diagonal
        // (fmaxf ignores NaN; the row of slot 0 above the diagonal counts as
        // -1), then the first of its rows holding it; rows past the matrix
        // hold zeros and come after all real rows, so they are taken only
        // when the thread has no real candidate, and are then rejected
        const float v0 = tid >= c ? fabsf(x[0][c]) : -1.0f;
        float m = v0;
#pragma unroll
        for (int q = 1; q < kP8Rows; ++q) m = fmaxf(m, fabsf(x[q][c]));
        int qs = kP8Rows;
#pragma unroll
        for (int q = kP8Rows - 1; q > 0; --q) qs = fabsf(x[q][c]) == m ? q : qs;
        qs = v0 == m ? 0 : qs;
        const int is = tid + kP8Threads * qs;
        P8Key best = (qs < kP8Rows && is < rows && m >= 0.0f) ? p8_key(m, is) : 0;
        // wavefront reduction: DPP inside each 16-lane row (xor 1, xor 2,
        // rotate 4, rotate 8 cover the row), then the four rows by readlane
        p8_dpp_max<0xB1>(best);   // quad_perm [1,0,3,2]
        p8_dpp_max<0x4E>(best);   // quad_perm [2,3,0,1]
        p8_dpp_max<0x124>(best);  // row_ror 4
        p8_dpp_max<0x128>(best);  // row_ror 8
        P8Key wk = p8_lane_key(best, 0);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            const P8Key o = p8_lane_key(best, 16 * r);
            wk = o > wk ? o : wk;
        }
        // the wavefront's candidate key and the row's values, written by the
        // lane owning it (slot wi / kP8Threads, uniform)
        if (lane == 0) skey[buf][wave] = wk;
        const int wi = (int)~(uint32_t)wk;
        if (wk != 0 && (wi & (kP8Threads - 1)) == tid) {
#pragma unroll
            for (int q = 0; q < kP8Rows; ++q)
                if (q == wi / kP8Threads)
#pragma unroll
                    for (int cc = 0; cc < kP8; ++cc) srow[buf][wave][cc] = x[q][cc];
        }
        if (tid == c)
#pragma unroll
            for (int cc = 0; cc < kP8; ++cc) sdiag[buf][cc] = x[0][cc];
        __syncthreads();
        P8Key pk = skey[buf][0];
        int pw = 0;
#pragma unroll
        for (int q = 1; q < kP8Waves; ++q) {
            const P8Key o = skey[buf][q];
            if (o > pk) pk = o, pw = q;
        }
        int pi = (int)~(uint32_t)pk;
        if (pk == 0) pi = c, pw = -1;  // no candidate (every |value| NaN): the diagonal row
        pi = __builtin_amdgcn_readfirstlane(pi);
        pw = __builtin_amdgcn_readfirstlane(pw);
        // both rows read whole and at once (one LDS round trip), then chosen
        const float4* dp = reinterpret_cast<const float4*>(sdiag[buf]);
        const float4* sp = reinterpret_cast<const float4*>(srow[buf][pw >= 0 ? pw : 0]);
        const float4 d0 = dp[0], d1 = dp[1], s0 = sp[0], s1 = sp[1];
        const float dr[kP8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        const float sr[kP8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        float pr[kP8];
#pragma unroll
        for (int cc = 0; cc < kP8; ++cc) pr[cc] = pw >= 0 ? sr[cc] : dr[cc];
        if (tid == 0) ipiv[j + c] = (int32_t)(j + pi);
        if (pi != c) {  // two lanes exchange rows j + c (slot 0 of thread c) and j + pi
            if (tid == (pi & (kP8Threads - 1))) {
#pragma unroll
                for (int q = 0; q < kP8Rows; ++q)
                    if (q == pi / kP8Threads)
#pragma unroll
                        for (int cc = 0; cc < kP8; ++cc) x[q][cc] = dr[cc];
            }
            if (tid == c)
#pragma unroll
                for (int cc = 0; cc < kP8; ++cc) x[0][cc] = pr[cc];
        }
        const float pv = pr[c];  // the pivot row is now row j + c
        if (tid == 0 && pv == 0.0f && *info == 0) *info = (int32_t)(j + c + 1);
        if (pv != 0.0f) {
            // rows below the diagonal; rows past the matrix hold zeros, take the
            // update harmlessly (or skip it with their wavefront) and are never
            // stored or chosen as pivots
            const float rp = 1.0f / pv;
#pragma unroll
            for (int q = 0; q < kP8Rows; ++q) {
                if (kP8Threads * q + 64 * wave >= rows) continue;  // the wavefront's rows of slot q are all past the matrix
                const bool below = q > 0 || tid > c;
                const float l = x[q][c] * rp;
                x[q][c] = below ? l : x[q][c];
#pragma unroll
                for (int cc = c + 1; cc < kP8; ++cc) {
                    const float u = __builtin_fmaf(-l, pr[cc], x[q][cc]);
                    x[q][cc] = below ? u : x[q][cc];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kP8Rows; ++q) {
        const int i = tid + kP8Threads * q;
        if (i < rows) {
            float4* rp = reinterpret_cast<float4*>(W + (int64_t)i * kP8);
            rp[0] = make_float4(x[q][0], x[q][1], x[q][2], x[q][3]);
            rp[1] = make_float4(x[q][4], x[q][5], x[q][6], x[q][7]);
        }
    }
}

// The sub-panel A[j:j+rows, j:j+w] (w <= kP8) copied into W (rows x kP8,
// row-major, 16-byte aligned; columns from w on zero), one thread per row
// over as many workgroups as it takes (lu_subpanel_post writes it back the
// same way): A's rows are lda apart, and one workgroup fetching them all
// (each row a separate line and page) took most of the panel kernel's time.
// vec: w == kP8 and A's rows 16-byte aligned at column j (two 16-byte pieces
// per row), else element by element.
__global__ __launch_bounds__(256) void lu_gather8(const float* A, int64_t lda, int64_t j, int rows, int w, int vec,
                                                  float* W) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    const float* rp = A + (j + i) * lda + j;
    float4* wp = reinterpret_cast<float4*>(W + (int64_t)i * kP8);
    if (vec) {
        wp[0] = *reinterpret_cast<const float4*>(rp);
        wp[1] = *reinterpret_cast<const float4*>(rp + 4);
    } else {
        float v[kP8];
#pragma unroll
        for (int c = 0; c < kP8; ++c) v[c] = c < w ? rp[c] : 0.0f;
        wp[0] = make_float4(v[0], v[1], v[2], v[3]);
        wp[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

// After lu_panel8 on the sub-panel at column jj of the panel [c0, c1):
// blocks 0 .. nb-1 write the factored sub-panel back from W, one thread per
// row (as lu_gather8 read it); block nb gives each column of the panel
// outside the sub-panel one thread, which applies the sub-panel's row swaps
// to its column in order and, right of the sub-panel, solves the 8 rows jj ..
// jj+7 of its column with the unit lower block L11 (U12 = L11^-1 A12, L11
// from W).  The columns are independent, so swaps and solve need no barrier
// between them, and the write-back touches none of their elements.
__global__ __launch_bounds__(256) void lu_subpanel_post(float* A, int64_t lda, int64_t jj, int rows, int wi, int vec,
                                                        const float* W, const int32_t* ipiv, int64_t c0, int64_t c1,
                                                        int nb) {
    if ((int)blockIdx.x < nb) {
        const int i = blockIdx.x * 256 + threadIdx.x;
        if (i >= rows) return;
        float* rp = A + (jj + i) * lda + jj;
        const float4* wp = reinterpret_cast<const float4*>(W + (int64_t)i * kP8);
        if (vec) {
            *reinterpret_cast<float4*>(rp) = wp[0];
            *reinterpret_cast<float4*>(rp + 4) = wp[1];
        } else {
            const float4 u = wp[0], v = wp[1];
            const float e[kP8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
            for (int c = 0; c < kP8; ++c)
                if (c < wi) rp[c] = e[c];
        }
        return;
    }
    __shared__ float L[kP8][kP8];
    if (threadIdx.x < kP8 * kP8) L[threadIdx.x / kP8][threadIdx.x % kP8] = W[threadIdx.x];
    __syncthreads();
    const int64_t col = c0 + threadIdx.x;  // c1 - c0 <= kNb < 256
    if (col >= c1 || (col >= jj && col < jj + wi)) return;
    for (int c = 0; c < wi; ++c) {
        const int64_t k = jj + c, p = ipiv[k];
        if (p != k) {
            const float t = A[k * lda + col];
            A[k * lda + col] = A[p * lda + col];
            A[p * lda + col] = t;
        }
    }
    if (col < jj + wi) return;  // left of the sub-panel: swaps only
    // right of it (then wi == kP8: only the panel's last sub-panel is narrower)
    float x[kP8];
#pragma unroll
    for (int i = 0; i < kP8; ++i) x[i] = A[(jj + i) * lda + col];
#pragma unroll
    for (int i = 1; i < kP8; ++i)
#pragma unroll
        for (int k = 0; k < i; ++k) x[i] = __builtin_fmaf(-L[i][k], x[k], x[i]);
#pragma unroll
    for (int i = 0; i < kP8; ++i) A[(jj + i) * lda + col] = x[i];
}

// The rest of the panel after a factored sub-panel [jj, jj + 8): A[r, c] -=
// sum_k L21[r, k] U12[k, c] for rows r in [jj + 8, jj + 8 + below) and
// columns c in [jj + 8, c1), L21 from the sub-panel's copy W (its rows from 8
// on) and U12 = A[jj:jj+8, c] (solved by lu_subpanel_post), summed over k in
// order by fused multiply-adds.  One thread per row and group of 8 columns
// (threads of one row adjacent, so a row's groups are read and written
// together).  The first group is the next sub-panel: its updated values also
// go to that sub-panel's copy Wn (row r at r - jj - 8, columns from wn on
// zero), so it needs no gather.  vec: A's rows 16-byte aligned at these
// columns.
__global__ __launch_bounds__(256) void lu_subpanel_update(float* A, int64_t lda, int64_t jj, int below, int64_t c1,
                                                          const float* W, float* Wn, int wn, int vec) {
    __shared__ float U[kP8][kNb];
    const int cols = (int)(c1 - jj - kP8);  // 1 .. kNb - kP8
    for (int e = threadIdx.x; e < kP8 * cols; e += 256) U[e / cols][e % cols] = A[(jj + e / cols) * lda + jj + kP8 + e % cols];
    __syncthreads();
    const int groups = (cols + kP8 - 1) / kP8;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = (int)(t / groups), g = (int)(t % groups);
    if (r >= below) return;
    const int cg = g * kP8;                          // first column of the group, from jj + 8
    const int nc = cols - cg < kP8 ? cols - cg : kP8;  // columns in the group
    const float4* lp = reinterpret_cast<const float4*>(W + (int64_t)(kP8 + r) * kP8);
    const float4 l0 = lp[0], l1 = lp[1];
    const float l[kP8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
    float* cp = A + (jj + kP8 + r) * lda + jj + kP8 + cg;
    float acc[kP8];
    if (vec && nc == kP8) {
        const float4 a0 = reinterpret_cast<const float4*>(cp)[0], a1 = reinterpret_cast<const float4*>(cp)[1];
        acc[0] = a0.x, acc[1] = a0.y, acc[2] = a0.z, acc[3] = a0.w;
        acc[4] = a1.x, acc[5] = a1.y, acc[6] = a1.z, acc[7] = a1.w;
    } else {
#pragma unroll
        for (int cc = 0; cc < kP8; ++cc) acc[cc] = cc < nc ? cp[cc] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kP8; ++k)
#pragma unroll
        for (int cc = 0; cc < kP8; ++cc)
            if (cc < nc) acc[cc] = __builtin_fmaf(-l[k], U[k][cg + cc], acc[cc]);
    if (vec && nc == kP8) {
        reinterpret_cast<float4*>(cp)[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        reinterpret_cast<float4*>(cp)[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    } else {
#pragma unroll
        for (int cc = 0; cc < kP8; ++cc)
            if (cc < nc) cp[cc] = acc[cc];
    }
    if (g == 0) {
        float4* wp = reinterpret_cast<float4*>(Wn + (int64_t)r * kP8);
        float v[kP8];
#pragma unroll
        for (int cc = 0; cc < kP8; ++cc) v[cc] = cc < wn ? acc[cc] : 0.0f;
        wp[0] = make_float4(v[0], v[1], v[2], v[3]);
        wp[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

// The panel's row swaps (rows j .. j+w-1 with ipiv[.]) on every column
// outside the panel, one thread per column, swaps in order.
__global__ __launch_bounds__(256) void lu_laswp(int64_t n, float* A, int64_t lda, int64_t j, int w,
                                                const int32_t* ipiv) {
    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= n || (col >= j && col < j + w)) return;
    for (int c = 0; c < w; ++c) {
        const int64_t k = j + c, p = ipiv[k];
        if (p != k) {
            const float t = A[k * lda + col];
            A[k * lda + col] = A[p * lda + col];
            A[p * lda + col] = t;
        }
    }
}

// U12 = L11^-1 A12 for the block row A[j:j+kNb, j+kNb:n] (L11 unit lower,
// kept in LDS), one thread per column, the column in registers.  L11 comes
// in as 16 loads per thread issued together, then 16 LDS stores (stored as
// each arrived, the loads went out one latency at a time); every lane reads
// the same entries, four per LDS read, and the multiply-adds run in the same
// order as one entry at a time.
__global__ __launch_bounds__(256) void lu_trsm(int64_t n, float* A, int64_t lda, int64_t j) {
    __shared__ __attribute__((aligned(16))) float L[kNb][kNb];
    constexpr int kPer = kNb * kNb / 256;
    float lv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 256 * u;
        lv[u] = A[(j + e / kNb) * lda + j + e % kNb];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 256 * u;
        L[e / kNb][e % kNb] = lv[u];
    }
    __syncthreads();
    const int64_t col = j + kNb + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= n) return;
    float x[kNb];
#pragma unroll
    for (int i = 0; i < kNb; ++i) x[i] = A[(j + i) * lda + col];
#pragma unroll
    for (int i = 1; i < kNb; ++i)
#pragma unroll
        for (int k4 = 0; k4 < i; k4 += 4) {
            const float4 l = *reinterpret_cast<const float4*>(&L[i][k4]);
            const float lk[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
            for (int k = k4; k < k4 + 4 && k < i; ++k) x[i] = __builtin_fmaf(-lk[k - k4], x[k], x[i]);
        }
#pragma unroll
    for (int i = 0; i < kNb; ++i) A[(j + i) * lda + col] = x[i];
}

// Diagonal block [s, s+w) of the factors solved for the right-hand sides
// V[s:s+w, 0:nrhs] in place: unit lower (forward) or upper (backward, with
// the diagonal).  One wavefront per right-hand side, lane i holding row i:
// the lane's row of the block is loaded into registers once (every load in
// flight together), and each finished unknown reaches the other lanes by
// readlane, so the w dependent steps wait on no memory and no barrier.
static_assert(kNb == 64, "one wavefront per diagonal block");
template <bool LOWER>
__global__ __launch_bounds__(kNb) void lu_trsv_block(const float* LU, int64_t ldlu, int64_t s, int w, float* V,
                                                     int64_t ldv) {
    const int i = threadIdx.x;
    const int64_t q = blockIdx.x;
    const float* row = LU + (s + (i < w ? i : 0)) * ldlu + s;
    float r[kNb];
#pragma unroll
    for (int k = 0; k < kNb; ++k) r[k] = k < w ? row[k] : 0.0f;
    float xi = i < w ? V[(s + i) * ldv + q] : 0.0f;
    auto lane_value = [](float v, int k) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
    };
    if constexpr (LOWER) {
#pragma unroll
        for (int k = 0; k < kNb; ++k) {
            if (k < w) {
                const float xk = lane_value(xi, k);
                if (i > k && i < w) xi = __builtin_fmaf(-r[k], xk, xi);
            }
        }
    } else {
#pragma unroll
        for (int k = kNb - 1; k >= 0; --k) {
            if (k < w) {
                if (i == k) xi = xi / r[k];
                const float xk = lane_value(xi, k);
                if (i < k) xi = __builtin_fmaf(-r[k], xk, xi);
            }
        }
    }
    if (i < w) V[(s + i) * ldv + q] = xi;
}

// One block step of the substitution, for right-hand side q = blockIdx.y:
// the diagonal block [s, s+w) of the factors solved (unit lower, forward, or
// upper with the diagonal, backward) from In[s:s+w, q] by the first
// wavefront of every workgroup, as in lu_trsv_block (each workgroup solves
// the same small system, so none waits for another); workgroup 0 writes the
// solution to Out[s:s+w, q]; and the rows still to be solved (forward: below
// the block, backward: above it), one per thread, are updated in place,
// In[r, q] -= LU[r, s:s+w] . x, by multiply-adds in column order.  In and
// Out are distinct arrays, so no workgroup overwrites right-hand sides
// another still reads.  vec: LU's rows 16-byte aligned at column s.
template <bool LOWER>
__global__ __launch_bounds__(256) void lu_subst_step(const float* LU, int64_t ldlu, int64_t n, int64_t s, int w,
                                                     float* In, int64_t ldi, float* Out, int64_t ldo, int vec) {
    __shared__ float xs[kNb];
    const int64_t q = blockIdx.y;
    if (threadIdx.x < kNb) {
        const int i = threadIdx.x;
        const float* row = LU + (s + (i < w ? i : 0)) * ldlu + s;
        float r[kNb];
#pragma unroll
        for (int k = 0; k < kNb; ++k) r[k] = k < w ? row[k] : 0.0f;
        float xi = i < w ? In[(s + i) * ldi + q] : 0.0f;
        auto lane_value = [](float v, int k) {
            return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
        };
        if constexpr (LOWER) {
#pragma unroll
            for (int k = 0; k < kNb; ++k) {
                if (k < w) {
                    const float xk = lane_value(xi, k);
                    if (i > k && i < w) xi = __builtin_fmaf(-r[k], xk, xi);
                }
            }
        } else {
#pragma unroll
            for (int k = kNb - 1; k >= 0; --k) {
                if (k < w) {
                    if (i == k) xi = xi / r[k];
                    const float xk = lane_value(xi, k);
                    if (i < k) xi = __builtin_fmaf(-r[k], xk, xi);
                }
            }
        }
        xs[i] = xi;  // 0 for i >= w
        if (blockIdx.x == 0 && i < w) Out[(s + i) * ldo + q] = xi;
    }
    __syncthreads();
    const int64_t r0 = LOWER ? s + w : 0, r1 = LOWER ? n : s;
    const int64_t rr = r0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (rr >= r1) return;
    const float* lr = LU + rr * ldlu + s;
    float acc = In[rr * ldi + q];
    if (vec && w == kNb) {
#pragma unroll
        for (int k4 = 0; k4 < kNb / 4; ++k4) {
            const float4 a = reinterpret_cast<const float4*>(lr)[k4];
            acc = __builtin_fmaf(-a.x, xs[4 * k4], acc);
            acc = __builtin_fmaf(-a.y, xs[4 * k4 + 1], acc);
            acc = __builtin_fmaf(-a.z, xs[4 * k4 + 2], acc);
            acc = __builtin_fmaf(-a.w, xs[4 * k4 + 3], acc);
        }
    } else {
        for (int k = 0; k < w; ++k) acc = __builtin_fmaf(-lr[k], xs[k], acc);
    }
    In[rr * ldi + q] = acc;
}

// dst[i, :] = src[perm[i], :] (rows of nrhs FP32 values).
__global__ __launch_bounds__(256) void gather_rows(int64_t n, int64_t nrhs, const int32_t* perm, const float* src,
                                                   int64_t lds, float* dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e / nrhs, q = e % nrhs;
    dst[i * ldd + q] = src[(int64_t)perm[i] * lds + q];
}

__global__ __launch_bounds__(256) void f64_to_f32(int64_t rows, int64_t cols, const double* X, int64_t ldx, float* Y,
                                                  int64_t ldy) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols, q = e % cols;
    Y[i * ldy + q] = (float)X[i * ldx + q];
}

// X = D (first) or X += D, X FP64, D FP32.
__global__ __launch_bounds__(256) void accumulate_f64(int64_t rows, int64_t cols, const float* D, int64_t ldd,
                                                      double* X, int64_t ldx, int first) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols, q = e % cols;
    const double d = (double)D[i * ldd + q];
    X[i * ldx + q] = first ? d : X[i * ldx + q] + d;
}

// R = B - A X in FP64: one wavefront per (row, right-hand side), lanes over K.
__global__ __launch_bounds__(256) void residual_f64(int64_t n, int64_t nrhs, const double* A, int64_t lda,
                                                   const double* X, int64_t ldx, const double* B, int64_t ldb,
                                                   double* R, int64_t ldr) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n * nrhs) return;
    const int64_t i = w / nrhs, q = w % nrhs;
    double acc = 0.0;
    for (int64_t k = lane; k < n; k += 64) acc = fma(A[i * lda + k], X[k * ldx + q], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) R[i * ldr + q] = B[i * ldb + q] - acc;
}

// Row sums of |A| (FP64), one wavefront per row.
__global__ __launch_bounds__(256) void abs_row_sums(int64_t n, const double* A, int64_t lda, double* out) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t k = lane; k < n; k += 64) acc += fabs(A[i * lda + k]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) out[i] = acc;
}

// out[q] = max_i |V[i, q]| for each of the nrhs columns of V (one workgroup
// per column); with rows_only (nrhs = 1 of a vector v), the max of v.
__global__ __launch_bounds__(256) void col_abs_max(int64_t n, int64_t nrhs, const double* V, int64_t ldv,
                                                   double* out) {
    __shared__ double red[256];
    const int64_t q = blockIdx.x;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(V[i * ldv + q]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
}

unsigned blocks(int64_t work, int per) { return (unsigned)std::max<int64_t>(1, (work + per - 1) / per); }

bool factor_mode_ok(int mode) {
    const int m = mode & MFG_MODE_MASK;
    return (mode & ~MFG_MODE_MASK) == 0 && m >= 0 && m < MFG_NUM_MODES;
}

}  // namespace

// Floats of the two sub-panel copies that lu_factor_impl needs (each at
// least the 8 x 8 diagonal block lu_subpanel_post reads).
int64_t lu_copy_floats(int64_t n) {
    return std::max<int64_t>(std::min<int64_t>(n, (int64_t)kP8Threads * kP8Rows), kP8) * kP8;
}
int64_t lu_scratch_floats(int64_t n) { return 2 * lu_copy_floats(n); }

// Blocked LU (see the file comment).  A, ipiv, info, W (lu_scratch_floats(n)
// floats): device.  A 64-wide panel is itself factored by 8-column
// sub-panels: each held in a contiguous copy (the panel's first gathered by
// lu_gather8, the others written by the previous sub-panel's update; the two
// halves of W alternate), factored there in registers (lu_panel8), written
// back with its swaps applied across the panel and its block row solved
// (lu_subpanel_post), and the rest of the panel updated with K = 8
// (lu_subpanel_update, L21 read from the copy): the same elimination, with
// the panel's updates blocked.  Panels taller than lu_panel8 holds go column
// by column (lu_panel).

int lu_factor_impl(int64_t n, float* A, int64_t lda, int32_t* ipiv, int32_t* info, float* W, int mode,
                   hipStream_t s) {
    MFG_HIP_CHECK(hipMemsetAsync(info, 0, sizeof(int32_t), s));
    for (int64_t j = 0; j < n; j += kNb) {
        const int w = (int)std::min<int64_t>(kNb, n - j);
        if (n - j <= (int64_t)kP8Threads * kP8Rows) {
            const bool aligned = lda % 4 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0;
            float* const copies[2] = {W, W + lu_copy_floats(n)};
            int cur = 0;
            bool held = false;  // copies[cur] already holds this sub-panel
            for (int64_t jj = j; jj < j + w; jj += kP8) {
                const int wi = (int)std::min<int64_t>(kP8, j + w - jj);
                const int vec = wi == kP8 && aligned;
                const int rows = (int)(n - jj);
                float* const Wc = copies[cur];
                if (!held) {
                    hipLaunchKernelGGL(lu_gather8, dim3(blocks(rows, 256)), dim3(256), 0, s, A, lda, jj, rows, wi, vec,
                                       Wc);
                    MFG_LAUNCH_CHECK();
                }
                hipLaunchKernelGGL(lu_panel8, dim3(1), dim3(kP8Threads), 0, s, rows, Wc, jj, wi, ipiv, info);
                MFG_LAUNCH_CHECK();
                const unsigned nb = blocks(rows, 256);
                hipLaunchKernelGGL(lu_subpanel_post, dim3(nb + 1), dim3(256), 0, s, A, lda, jj, rows, wi, vec, Wc,
                                   ipiv, j, j + w, (int)nb);
                MFG_LAUNCH_CHECK();
                const int64_t right = j + w - (jj + wi);  // columns of the panel right of the sub-panel
                const int below = rows - wi;              // > 0 whenever right > 0 (then wi == kP8)
                held = false;
                if (right > 0 && below > 0) {
                    const int wn = (int)std::min<int64_t>(kP8, right);
                    const int64_t threads = (int64_t)below * ((right + kP8 - 1) / kP8);
                    hipLaunchKernelGGL(lu_subpanel_update, dim3(blocks(threads, 256)), dim3(256), 0, s, A, lda, jj,
                                       below, j + w, Wc, copies[cur ^ 1], wn, (int)aligned);
                    MFG_LAUNCH_CHECK();
                    cur ^= 1;
                    held = true;
                }
            }
        } else {
            hipLaunchKernelGGL(lu_panel, dim3(1), dim3(kPanelThreads), 0, s, n, A, lda, j, w, ipiv, info);
            MFG_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(lu_laswp, dim3(blocks(n, 256)), dim3(256), 0, s, n, A, lda, j, w, ipiv);
        MFG_LAUNCH_CHECK();
        const int64_t rest = n - j - w;
        if (rest <= 0) continue;  // w == kNb from here on
        hipLaunchKernelGGL(lu_trsm, dim3(blocks(rest, 256)), dim3(256), 0, s, n, A, lda, j);
        MFG_LAUNCH_CHECK();
        // A22 -= L21 U12 on the matrix cores, in the factorisation's mode
        float* a22 = A + (j + w) * lda + j + w;
        const int st = mfg_gemm(rest, rest, w, A + (j + w) * lda + j, lda, A + j * lda + j + w, lda, a22, lda, -1.0f,
                                1.0f, mode, (void*)s);
        if (st != MFG_OK) return st;
    }
    return MFG_OK;
}

// The row permutation of the sequential swaps in ipiv (device), on the host.
static int permutation(int64_t n, const int32_t* ipiv, std::vector<int32_t>& perm, hipStream_t s) {
    std::vector<int32_t> piv((size_t)n);
    MFG_HIP_CHECK(hipMemcpyAsync(piv.data(), ipiv, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    MFG_HIP_CHECK(hipStreamSynchronize(s));
    perm.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t p = piv[(size_t)i];
        if (p < i || p >= n) return MFG_ERR_INVALID_ARG;  // not a pivot sequence of a factorisation
        std::swap(perm[(size_t)i], perm[(size_t)p]);
    }
    return MFG_OK;
}

// V = U^-1 L^-1 V (V: n x nrhs FP32, already permuted), FP32.
// Forward and backward substitution by blocks of kNb rows, in place in V
// (n x nrhs).  Y (n x nrhs, ldy) is scratch: each block step reads its
// right-hand sides from one of V and Y and writes its solution to the other
// (forward V -> Y, backward Y -> V), with the remaining rows updated in the
// same launch (lu_subst_step).  More right-hand sides than a grid dimension
// holds go block by block instead: the diagonal block (lu_trsv_block), then
// the rest of V by an FP32 mfg_gemm.
static int lu_substitute(int64_t n, int64_t nrhs, const float* LU, int64_t ldlu, float* V, int64_t ldv, float* Y,
                         int64_t ldy, hipStream_t s) {
    if (nrhs <= 65535) {
        const int vec = ldlu % 4 == 0 && reinterpret_cast<uintptr_t>(LU) % 16 == 0;
        for (int64_t b = 0; b < n; b += kNb) {  // forward, unit lower: V -> Y
            const int w = (int)std::min<int64_t>(kNb, n - b);
            const dim3 g(blocks(n - b - w, 256), (unsigned)nrhs);
            hipLaunchKernelGGL(lu_subst_step<true>, g, dim3(256), 0, s, LU, ldlu, n, b, w, V, ldv, Y, ldy, vec);
            MFG_LAUNCH_CHECK();
        }
        for (int64_t b = ((n - 1) / kNb) * kNb; b >= 0; b -= kNb) {  // backward, upper: Y -> V
            const int w = (int)std::min<int64_t>(kNb, n - b);
            const dim3 g(blocks(b, 256), (unsigned)nrhs);
            hipLaunchKernelGGL(lu_subst_step<false>, g, dim3(256), 0, s, LU, ldlu, n, b, w, Y, ldy, V, ldv, vec);
            MFG_LAUNCH_CHECK();
        }
        return MFG_OK;
    }
    const dim3 g((unsigned)nrhs);
    for (int64_t b = 0; b < n; b += kNb) {  // forward, unit lower
        const int w = (int)std::min<int64_t>(kNb, n - b);
        hipLaunchKernelGGL(lu_trsv_block<true>, g, dim3(kNb), 0, s, LU, ldlu, b, w, V, ldv);
        MFG_LAUNCH_CHECK();
        if (b + w < n) {
            const int st = mfg_gemm(n - b - w, nrhs, w, LU + (b + w) * ldlu + b, ldlu, V + b * ldv, ldv,
                                    V + (b + w) * ldv, ldv, -1.0f, 1.0f, MFG_F32, (void*)s);
            if (st != MFG_OK) return st;
        }
    }
    for (int64_t b = ((n - 1) / kNb) * kNb; b >= 0; b -= kNb) {  // backward, upper
        const int w = (int)std::min<int64_t>(kNb, n - b);
        hipLaunchKernelGGL(lu_trsv_block<false>, g, dim3(kNb), 0, s, LU, ldlu, b, w, V, ldv);
        MFG_LAUNCH_CHECK();
        if (b > 0) {
            const int st = mfg_gemm(b, nrhs, w, LU + b, ldlu, V + b * ldv, ldv, V, ldv, -1.0f, 1.0f, MFG_F32,
                                    (void*)s);
            if (st != MFG_OK) return st;
        }
    }
    return MFG_OK;
}

// X = (LU)^-1 P B with B, X n x nrhs FP32 (X may not alias B).  B is
// overwritten: once its rows are gathered into X it is the substitution's
// scratch.
static int lu_solve_impl(int64_t n, int64_t nrhs, const float* LU, int64_t ldlu, const int32_t* dperm, float* B,
                         int64_t ldb, float* X, int64_t ldx, hipStream_t s) {
    hipLaunchKernelGGL(gather_rows, dim3(blocks(n * nrhs, 256)), dim3(256), 0, s, n, nrhs, dperm, B, ldb, X, ldx);
    MFG_LAUNCH_CHECK();
    return lu_substitute(n, nrhs, LU, ldlu, X, ldx, B, ldb, s);
}

}  // namespace mfg

using namespace mfg;

namespace {

// Device buffers of one call, freed on every return path.
struct Buffers {
    std::vector<void*> ptrs;
    template <class T>
    int get(T** p, size_t count) {
        *p = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return MFG_ERR_NO_MEMORY;
        }
        ptrs.push_back(*p);
        return MFG_OK;
    }
    ~Buffers() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

int lu_factor_api(int64_t n, float* A, int64_t lda, int32_t* ipiv, int64_t* info, int mode, hipStream_t s) {
    if (n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && (!A || !ipiv)) || !factor_mode_ok(mode))
        return MFG_ERR_INVALID_ARG;
    if (n > INT32_MAX) return MFG_ERR_UNSUPPORTED;
    if (info) *info = 0;
    if (n == 0) return MFG_OK;
    Buffers buf;
    int32_t* dinfo = nullptr;
    float* W = nullptr;
    int st = buf.get(&dinfo, 1);
    if (st == MFG_OK) st = buf.get(&W, (size_t)lu_scratch_floats(n));
    if (st == MFG_OK) st = lu_factor_impl(n, A, lda, ipiv, dinfo, W, mode, s);
    if (st != MFG_OK) return st;
    int32_t h = 0;
    MFG_HIP_CHECK(hipMemcpyAsync(&h, dinfo, sizeof(h), hipMemcpyDeviceToHost, s));
    MFG_HIP_CHECK(hipStreamSynchronize(s));  // before dinfo is freed
    if (info) *info = h;
    return MFG_OK;
}

int lu_solve_api(int64_t n, int64_t nrhs, const float* LU, int64_t ldlu, const int32_t* ipiv, float* B, int64_t ldb,
                 hipStream_t s) {
    if (n < 0 || nrhs < 0 || ldlu < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, nrhs) ||
        (n > 0 && (!LU || !ipiv)) || (n > 0 && nrhs > 0 && !B))
        return MFG_ERR_INVALID_ARG;
    if (nrhs > INT32_MAX) return MFG_ERR_UNSUPPORTED;
    if (n == 0 || nrhs == 0) return MFG_OK;
    std::vector<int32_t> perm;
    int st = permutation(n, ipiv, perm, s);
    if (st != MFG_OK) return st;
    Buffers buf;
    int32_t* dperm = nullptr;
    float* tmp = nullptr;
    if ((st = buf.get(&dperm, (size_t)n)) != MFG_OK || (st = buf.get(&tmp, (size_t)(n * nrhs))) != MFG_OK) return st;
    MFG_HIP_CHECK(hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    if ((st = lu_solve_impl(n, nrhs, LU, ldlu, dperm, B, ldb, tmp, nrhs, s)) != MFG_OK) return st;
    MFG_HIP_CHECK(hipMemcpy2DAsync(B, (size_t)ldb * 4, tmp, (size_t)nrhs * 4, (size_t)nrhs * 4, (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
    MFG_HIP_CHECK(hipStreamSynchronize(s));  // before the buffers are freed
    return MFG_OK;
}

int solve_ir_api(int64_t n, int64_t nrhs, const double* A, int64_t lda, const double* B, int64_t ldb, double* X,
                 int64_t ldx, int mode, int max_iter, double tol, int* iters, double* berr, int64_t* info,
                 hipStream_t s) {
    if (n < 0 || nrhs < 0 || lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, nrhs) ||
        ldx < std::max<int64_t>(1, nrhs) || (n > 0 && !A) || (n > 0 && nrhs > 0 && (!B || !X)) ||
        !factor_mode_ok(mode) || max_iter < 0 || !(tol >= 0.0))
        return MFG_ERR_INVALID_ARG;
    if (n > INT32_MAX || nrhs > INT32_MAX) return MFG_ERR_UNSUPPORTED;
    if (iters) *iters = 0;
    if (berr) *berr = 0.0;
    if (info) *info = 0;
    if (n == 0 || nrhs == 0) return MFG_OK;
    Buffers buf;
    float *A32 = nullptr, *v = nullptr, *d = nullptr, *W = nullptr;
    double *R = nullptr, *rows = nullptr, *nrm = nullptr;
    int32_t *ipiv = nullptr, *dperm = nullptr, *dinfo = nullptr;
    int st;
    if ((st = buf.get(&A32, (size_t)(n * n))) != MFG_OK || (st = buf.get(&v, (size_t)(n * nrhs))) != MFG_OK ||
        (st = buf.get(&d, (size_t)(n * nrhs))) != MFG_OK || (st = buf.get(&R, (size_t)(n * nrhs))) != MFG_OK ||
        (st = buf.get(&rows, (size_t)n)) != MFG_OK || (st = buf.get(&nrm, (size_t)(3 * nrhs + 1))) != MFG_OK ||
        (st = buf.get(&ipiv, (size_t)n)) != MFG_OK || (st = buf.get(&dperm, (size_t)n)) != MFG_OK ||
        (st = buf.get(&dinfo, 1)) != MFG_OK || (st = buf.get(&W, (size_t)lu_scratch_floats(n))) != MFG_OK)
        return st;
    // the factorisation of the FP32 copy, in the given mode
    hipLaunchKernelGGL(f64_to_f32, dim3(blocks(n * n, 256)), dim3(256), 0, s, n, n, A, lda, A32, n);
    MFG_LAUNCH_CHECK();
    if ((st = lu_factor_impl(n, A32, n, ipiv, dinfo, W, mode, s)) != MFG_OK) return st;
    int32_t hinfo = 0;
    MFG_HIP_CHECK(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> perm;
    if ((st = permutation(n, ipiv, perm, s)) != MFG_OK) return st;  // synchronises
    if (info) *info = hinfo;
    if (hinfo != 0) {
        MFG_HIP_CHECK(hipStreamSynchronize(s));
        return MFG_OK;  // exactly singular factor: no solve (info says where)
    }
    MFG_HIP_CHECK(hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    // |A|_inf and |b_j|_inf, once
    hipLaunchKernelGGL(abs_row_sums, dim3(blocks(n, 4)), dim3(256), 0, s, n, A, lda, rows);
    MFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(col_abs_max, dim3(1), dim3(256), 0, s, n, (int64_t)1, rows, (int64_t)1, nrm + 3 * nrhs);
    MFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(col_abs_max, dim3((unsigned)nrhs), dim3(256), 0, s, n, nrhs, B, ldb, nrm + nrhs);
    MFG_LAUNCH_CHECK();
    // x0 from the factors
    hipLaunchKernelGGL(f64_to_f32, dim3(blocks(n * nrhs, 256)), dim3(256), 0, s, n, nrhs, B, ldb, v, nrhs);
    MFG_LAUNCH_CHECK();
    if ((st = lu_solve_impl(n, nrhs, A32, n, dperm, v, nrhs, d, nrhs, s)) != MFG_OK) return st;
    hipLaunchKernelGGL(accumulate_f64, dim3(blocks(n * nrhs, 256)), dim3(256), 0, s, n, nrhs, d, nrhs, X, ldx, 1);
    MFG_LAUNCH_CHECK();
    std::vector<double> h((size_t)(3 * nrhs + 1));
    double be = INFINITY;
    int it = 0;
    for (;; ++it) {
        // r = b - A x (FP64) and the backward error of x
        hipLaunchKernelGGL(residual_f64, dim3(blocks(n * nrhs, 4)), dim3(256), 0, s, n, nrhs, A, lda, X, ldx, B, ldb,
                           R, nrhs);
        MFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(col_abs_max, dim3((unsigned)nrhs), dim3(256), 0, s, n, nrhs, R, nrhs, nrm);
        MFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(col_abs_max, dim3((unsigned)nrhs), dim3(256), 0, s, n, nrhs, X, ldx, nrm + 2 * nrhs);
        MFG_LAUNCH_CHECK();
        MFG_HIP_CHECK(hipMemcpyAsync(h.data(), nrm, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        MFG_HIP_CHECK(hipStreamSynchronize(s));
        be = 0.0;
        const double anorm = h[(size_t)(3 * nrhs)];
        for (int64_t q = 0; q < nrhs; ++q) {
            const double den = anorm * h[(size_t)(2 * nrhs + q)] + h[(size_t)(nrhs + q)];
            const double e = den > 0.0 ? h[(size_t)q] / den : (h[(size_t)q] > 0.0 ? INFINITY : 0.0);
            be = std::max(be, e);
        }
        if (!(be > tol) || it >= max_iter) break;
        // correction: d = (LU)^-1 P r in FP32, x += d in FP64
        hipLaunchKernelGGL(f64_to_f32, dim3(blocks(n * nrhs, 256)), dim3(256), 0, s, n, nrhs, R, nrhs, v, nrhs);
        MFG_LAUNCH_CHECK();
        if ((st = lu_solve_impl(n, nrhs, A32, n, dperm, v, nrhs, d, nrhs, s)) != MFG_OK) return st;
        hipLaunchKernelGGL(accumulate_f64, dim3(blocks(n * nrhs, 256)), dim3(256), 0, s, n, nrhs, d, nrhs, X, ldx, 0);
        MFG_LAUNCH_CHECK();
    }
    if (iters) *iters = it;
    if (berr) *berr = be;
    return MFG_OK;
}

}  // namespace

#define MFG_SOLVE_GUARD(expr)                \
    try {                                    \
        return (expr);                       \
    } catch (const std::bad_alloc&) {        \
        return MFG_ERR_NO_MEMORY;            \
    } catch (...) {                          \
        return MFG_ERR_INTERNAL;             \
    }

extern "C" int mfg_lu_factor(int64_t n, float* A, int64_t lda, int32_t* ipiv, int64_t* info, int mode,
                             void* stream) {
    MFG_SOLVE_GUARD(lu_factor_api(n, A, lda, ipiv, info, mode, (hipStream_t)stream));
}

extern "C" int mfg_lu_solve(int64_t n, int64_t nrhs, const float* LU, int64_t ldlu, const int32_t* ipiv, float* B,
                            int64_t ldb, void* stream) {
    MFG_SOLVE_GUARD(lu_solve_api(n, nrhs, LU, ldlu, ipiv, B, ldb, (hipStream_t)stream));
}

extern "C" int mfg_solve_ir(int64_t n, int64_t nrhs, const double* A, int64_t lda, const double* B, int64_t ldb,
                            double* X, int64_t ldx, int mode, int max_iter, double tol, int* iters, double* berr,
                            int64_t* info, void* stream) {
    MFG_SOLVE_GUARD(solve_ir_api(n, nrhs, A, lda, B, ldb, X, ldx, mode, max_iter, tol, iters, berr, info,
                                 (hipStream_t)stream));
}
