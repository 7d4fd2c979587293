// batched.hip -- many small GEMMs (paper Sec. IV.B and Sec. VI: batched GEMM
// of many 16x16 problems, one warp per problem, 16 problems per block).
//
//   gemm16_batched_small : uniform strided batch with M, N <= 32.  Each
//     wavefront owns one problem at a time (one 32x32x16 MFMA per 16-deep K
//     chunk, rows/columns beyond M/N masked) and walks the batch with a
//     grid-wide stride, so the grid stays at a few waves per SIMD however
//     large the batch is.  Operands are read once: the batch is HBM-bound
//     (16^3: 2 KB and 8 Kflop per problem).
//   gemm16_batched_lds : the same per-problem arithmetic with whole-row
//     memory traffic when rows are 16-byte aligned: a K chunk of B (16 x 32)
//     arrives as one 16-byte load per lane into the wave's LDS slab and is
//     read back transposed (ds_read_b64_tr_b16), and the 32 x 32 result goes
//     through LDS so that C is read and written in 16-byte row pieces.
//   gemm16_grouped : thousands of GEMMs of different shapes in one
//     persistent launch.  The work list holds one entry per 32x32 output
//     tile of every problem (ordered by decreasing K, the tile's cost);
//     wavefronts take entries with a static grid stride.
// Both reuse the tile functions of the single GEMM, so each problem's result
// is bitwise identical to mfg_gemm on that problem alone.
#include <algorithm>

#include "tile16.h"

namespace mfg {

template <int KIND>
__global__ __launch_bounds__(256) void gemm16_batched_small(Gemm16Args p, int64_t count, int vecA) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < count; b += nwaves)
        simple_tile<KIND>(p, b, 0, 0, lane, vecA);
}

// s_waitcnt lgkmcnt(0): this wave's LDS accesses have completed.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4)); }

// B operand of the 32x32x16 MFMA from a row-major 16 x 32 slab: lane l gets
// column l % 32, rows 8 (l / 32) .. +7.  In each 16-lane group lane 4j + q
// points at row j, columns 4q .. 4q+3 of its half; the transposing read
// hands lane i column i of those four rows.
__device__ __forceinline__ u32x4 slab_read_b(const uint16_t* slab, int lane) {
    typedef short i16x4v __attribute__((ext_vector_type(4)));
    const int w = lane & 15, j = w >> 2, q = w & 3;
    const int c0 = ((lane >> 4) & 1) * 16, k0 = (lane >> 5) * 8;
    const int o1 = (k0 + j) * 32 + c0 + 4 * q, o2 = o1 + 4 * 32;
    i16x4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4v*)(slab + o1));
    i16x4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4v*)(slab + o2));
    u32x2 a = __builtin_bit_cast(u32x2, lo), b = __builtin_bit_cast(u32x2, hi);
    return u32x4{a[0], a[1], b[0], b[1]};
}

template <int KIND>
__global__ __launch_bounds__(256) void gemm16_batched_lds(Gemm16Args p, int64_t count, int vecC) {
    using T = KT<KIND>;
    constexpr int SLAB = 16 * 32;           // halfs per B plane slab
    constexpr int CROW = 33;                // floats per padded C row in LDS
    constexpr int WAVE_LDS = T::NPB * SLAB * 2 + 32 * CROW * 4;  // bytes
    __shared__ __attribute__((aligned(16))) unsigned char lds[4 * WAVE_LDS];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint16_t* slab = reinterpret_cast<uint16_t*>(lds + wid * WAVE_LDS);
    float* ct = reinterpret_cast<float*>(lds + wid * WAVE_LDS + T::NPB * SLAB * 2);
    const int r = lane & 31, g = lane >> 5;
    const int64_t M = p.M, N = p.N, K = p.K;
    const int krow = lane >> 2, c8 = (lane & 3) * 8;  // this lane's piece of a B chunk
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t b = (int64_t)blockIdx.x * 4 + wid; b < count; b += nwaves) {
        const uint16_t* Ap[2];
        const uint16_t* Bp[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            Ap[q] = (q < T::NPA) ? p.A[q] + b * p.sA : nullptr;
            Bp[q] = (q < T::NPB) ? p.B[q] + b * p.sB : nullptr;
        }
        f32x16 hi = {}, lo = {}, rr = {};
        for (int64_t k0 = 0; k0 < K; k0 += 16) {
            const int64_t kb = k0 + g * 8;
            u32x4 a[2] = {zero4(), zero4()}, bb[2] = {zero4(), zero4()};
#pragma unroll
            for (int q = 0; q < T::NPA; ++q) a[q] = load_row8(Ap[q], r < M, r * p.lda + kb, K - kb, true);
            const int64_t kr = k0 + krow;
#pragma unroll
            for (int q = 0; q < T::NPB; ++q) {
                u32x4 v;
                if (kr < K && c8 + 8 <= N) {
                    v = *reinterpret_cast<const u32x4*>(Bp[q] + kr * p.ldb + c8);
                } else {
                    uint16_t e[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) e[j] = (kr < K && c8 + j < N) ? Bp[q][kr * p.ldb + c8 + j] : (uint16_t)0;
                    v = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
                }
                *reinterpret_cast<u32x4*>(slab + q * SLAB + krow * 32 + c8) = v;
            }
            lds_wait();
#pragma unroll
            for (int q = 0; q < T::NPB; ++q) bb[q] = slab_read_b(slab + q * SLAB, lane);
            lds_wait();  // the slab is rewritten by the next chunk
            mma_step<KIND>(a, bb, hi, lo, rr);
        }
        // result -> LDS (row-major 32 x 32, padded), then whole row pieces to C
#pragma unroll
        for (int i = 0; i < 16; ++i) ct[mfma_out_row(i, lane) * CROW + r] = combine_at<KIND>(hi, lo, rr, i);
        lds_wait();
        float* C = p.C + b * p.sC;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int row = it * 8 + (lane >> 3), c4 = (lane & 7) * 4;
            if (row >= M) continue;
            const float* src = ct + row * CROW + c4;
            float* dst = C + row * p.ldc + c4;
            if (vecC && c4 + 4 <= N) {
                f32x4 v = {src[0], src[1], src[2], src[3]};
                if (p.beta == 0.0f) {
                    v = v * p.alpha;
                } else {
                    const f32x4 c = *reinterpret_cast<const f32x4*>(dst);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = __builtin_fmaf(p.alpha, v[e], p.beta * c[e]);
                }
                *reinterpret_cast<f32x4*>(dst) = v;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c4 + e < N)
                        dst[e] = (p.beta == 0.0f) ? p.alpha * src[e] : __builtin_fmaf(p.alpha, src[e], p.beta * dst[e]);
            }
        }
        lds_wait();  // the C tile is rewritten by the next problem
    }
}

int launch_batched_small(int kind, const Gemm16Args& a, int64_t count, bool vec_ok, int num_cu, hipStream_t s) {
    if (a.M > 32 || a.N > 32) return MFG_ERR_INTERNAL;
    const int64_t want = cdiv(count, 4);
    const int64_t cap = (int64_t)num_cu * 16;  // 16 workgroups (64 waves) per CU
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    if (grid == 0) return MFG_OK;
    const int v = vec_ok ? 1 : 0;
    if (vec_ok) {  // 16-byte aligned A and B rows: the LDS-staged kernel
        const int vc = (((uintptr_t)a.C % 16) == 0 && a.ldc % 4 == 0 && a.sC % 4 == 0) ? 1 : 0;
        switch (kind) {
            case K_F16: hipLaunchKernelGGL(gemm16_batched_lds<K_F16>, dim3(grid), dim3(256), 0, s, a, count, vc); break;
            case K_BF16: hipLaunchKernelGGL(gemm16_batched_lds<K_BF16>, dim3(grid), dim3(256), 0, s, a, count, vc); break;
            case K_REFINE_A:
                hipLaunchKernelGGL(gemm16_batched_lds<K_REFINE_A>, dim3(grid), dim3(256), 0, s, a, count, vc);
                break;
            case K_SPLIT3:
                hipLaunchKernelGGL(gemm16_batched_lds<K_SPLIT3>, dim3(grid), dim3(256), 0, s, a, count, vc);
                break;
            case K_SPLIT4:
                hipLaunchKernelGGL(gemm16_batched_lds<K_SPLIT4>, dim3(grid), dim3(256), 0, s, a, count, vc);
                break;
            default: return MFG_ERR_INVALID_ARG;
        }
        MFG_LAUNCH_CHECK();
        return MFG_OK;
    }
    switch (kind) {
        case K_F16: hipLaunchKernelGGL(gemm16_batched_small<K_F16>, dim3(grid), dim3(256), 0, s, a, count, v); break;
        case K_BF16: hipLaunchKernelGGL(gemm16_batched_small<K_BF16>, dim3(grid), dim3(256), 0, s, a, count, v); break;
        case K_REFINE_A:
            hipLaunchKernelGGL(gemm16_batched_small<K_REFINE_A>, dim3(grid), dim3(256), 0, s, a, count, v);
            break;
        case K_SPLIT3:
            hipLaunchKernelGGL(gemm16_batched_small<K_SPLIT3>, dim3(grid), dim3(256), 0, s, a, count, v);
            break;
        case K_SPLIT4:
            hipLaunchKernelGGL(gemm16_batched_small<K_SPLIT4>, dim3(grid), dim3(256), 0, s, a, count, v);
            break;
        default: return MFG_ERR_INVALID_ARG;
    }
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

// ------------------------------------------------------------------ grouped
// Every wavefront is an independent worker: it takes work items (one 32 x 32
// output tile of one problem) with a grid-wide stride.  Per 32-deep block of
// K it issues all global loads of the block first (A: one 16-byte row piece
// per lane and 16-deep chunk; B: one 16-byte row piece per lane of a 16 x 32
// chunk), then per chunk stages B in the wave's LDS slab, reads it back
// transposed and runs the 32x32x16 MFMA -- the same operands, in the same
// order, as the simple kernel on that tile.  Many independent waves per CU
// hide the memory latency of these HBM-bound problems.
constexpr int kGroupedWavesPerWG = 4;
constexpr int kGroupedChunks = 2;  // 16-deep K chunks whose loads are issued together
// 16 zero bytes in device memory: the load source of lanes with nothing to load
__device__ __attribute__((aligned(16))) const uint16_t kZero16[8] = {0, 0, 0, 0, 0, 0, 0, 0};
typedef __attribute__((address_space(1))) const uint16_t g_u16;
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;
typedef __attribute__((address_space(1))) float g_f32;
constexpr int kGroupedWGPerCU = 3;  // resident at 3 waves per SIMD (<= 168 VGPRs)

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gemm16_grouped(
    const GroupedDesc* descs, const GroupedWork* work, GroupedSplit split, float alpha, float beta) {
    __shared__ __attribute__((aligned(16))) uint16_t slabs[kGroupedWavesPerWG][16 * 32];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint16_t* slab = slabs[wid];
    const int r = lane & 31, g = lane >> 5;
    const int krow = lane >> 2, c8 = (lane & 3) * 8;
    // this XCD's range of the work list, shared by its workgroups
    const int xcd = blockIdx.x % kXcds;
    const int64_t nwaves = (int64_t)(gridDim.x / kXcds) * kGroupedWavesPerWG;
    const int64_t end = split.off[xcd + 1];
    // the wave's item index is uniform across its lanes (SGPRs)
    const int64_t first = split.off[xcd] + __builtin_amdgcn_readfirstlane((int)((blockIdx.x / kXcds) * kGroupedWavesPerWG + wid));
    for (int64_t it = first; it < end; it += nwaves) {
        const GroupedWork w = work[it];
        const GroupedDesc d = descs[w.prob];
        // The descriptor's pointers are device (global) memory.  Typed as such,
        // or every access is a flat one, which also counts against lgkmcnt
        // and so would wait behind (and be waited for by) the LDS traffic.
        const g_u16* gA = (const g_u16*)d.A;
        const g_u16* gB = (const g_u16*)d.B;
        g_f32* gC = (g_f32*)d.C;
        const int64_t m0 = (int64_t)w.tm * kGroupedTile, n0 = (int64_t)w.tn * kGroupedTile;
        const int64_t am = m0 + r;
        const bool vec = d.vec != 0;
        f32x16 hi = {}, lo = {}, rr = {};
        const int64_t bn = n0 + c8;
        // Loads of one block of kGroupedChunks 16-deep chunks: whole 16-byte
        // pieces first (all of them in flight together), then the ragged
        // pieces (K tail, N edge, unaligned rows) element by element.
        auto load_block = [&](int64_t kb0, u32x4 (&a)[kGroupedChunks], u32x4 (&b)[kGroupedChunks]) {
            bool ragged = false;
#pragma unroll
            for (int c = 0; c < kGroupedChunks; ++c) {
                const int64_t ka = kb0 + 16 * c + 8 * g, kr = kb0 + 16 * c + krow;
                const bool fa = vec && am < d.M && ka + 8 <= d.K;
                const bool fb = vec && kr < d.K && bn + 8 <= d.N;
                // unconditional loads (a lane with no whole piece reads 16 zero
                // bytes): no branch, so no wait at a join between the loads
                a[c] = *(const g_u32x4*)(fa ? gA + am * d.lda + ka : (const g_u16*)kZero16);
                b[c] = *(const g_u32x4*)(fb ? gB + kr * d.ldb + bn : (const g_u16*)kZero16);
                ragged |= (!fa && am < d.M && ka < d.K) || (!fb && kr < d.K && bn < d.N);
            }
            if (ragged) {
#pragma unroll
                for (int c = 0; c < kGroupedChunks; ++c) {
                    const int64_t ka = kb0 + 16 * c + 8 * g, kr = kb0 + 16 * c + krow;
                    if (!(vec && am < d.M && ka + 8 <= d.K) && am < d.M && ka < d.K) {
                        uint16_t e[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) e[j] = (ka + j < d.K) ? gA[am * d.lda + ka + j] : (uint16_t)0;
                        a[c] = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
                    }
                    if (!(vec && kr < d.K && bn + 8 <= d.N) && kr < d.K && bn < d.N) {
                        uint16_t e[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) e[j] = (bn + j < d.N) ? gB[kr * d.ldb + bn + j] : (uint16_t)0;
                        b[c] = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
                    }
                }
            }
        };
        // software pipeline over K blocks: block j+1's loads are in flight
        // while block j runs through the LDS slab and the MFMAs
        u32x4 ca[kGroupedChunks], cb[kGroupedChunks], na[kGroupedChunks], nb[kGroupedChunks];
        load_block(0, ca, cb);
        for (int64_t kb0 = 0; kb0 < d.K; kb0 += 16 * kGroupedChunks) {
            const bool more = kb0 + 16 * kGroupedChunks < d.K;
            if (more) load_block(kb0 + 16 * kGroupedChunks, na, nb);
#pragma unroll
            for (int c = 0; c < kGroupedChunks; ++c) {
                if (kb0 + 16 * c >= d.K) break;
                *reinterpret_cast<u32x4*>(slab + krow * 32 + c8) = cb[c];
                lds_wait();
                u32x4 aa[2] = {ca[c], zero4()}, bb[2] = {slab_read_b(slab, lane), zero4()};
                lds_wait();  // the slab is rewritten by the next chunk
                mma_step<KIND>(aa, bb, hi, lo, rr);
            }
            if (more) {
#pragma unroll
                for (int c = 0; c < kGroupedChunks; ++c) ca[c] = na[c], cb[c] = nb[c];
            }
        }
        store_blocks<1>(gC, d.ldc, d.M, d.N, m0, n0, lane, alpha, beta,
                        [&](int, int i) { return combine_at<KIND>(hi, lo, rr, i); });
    }
}

// Problems (or, for a problem above 1/16 of the total, bands of its tile
// rows) go to the XCD with the least work so far, largest first (LPT on
// flops); each XCD's items are then ordered by decreasing K, their cost.
void build_grouped_work(const GroupedDesc* descs, int64_t n, std::vector<GroupedWork>& work, GroupedSplit& split) {
    struct Unit {
        int64_t prob, tm0, tm1;
        double flops;
    };
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) total += 2.0 * (double)descs[i].M * (double)descs[i].N * (double)descs[i].K;
    const double cap = total / (2.0 * kXcds);
    std::vector<Unit> units;
    for (int64_t i = 0; i < n; ++i) {
        const GroupedDesc& d = descs[i];
        const int64_t tm = cdiv(d.M, kGroupedTile), tn = cdiv(d.N, kGroupedTile);
        if (tm == 0 || tn == 0) continue;
        const double f = 2.0 * (double)d.M * (double)d.N * (double)d.K;
        const int64_t parts = std::min<int64_t>(tm, cap > 0.0 ? std::max<int64_t>(1, (int64_t)(f / cap)) : 1);
        for (int64_t q = 0; q < parts; ++q) {
            const int64_t a = tm * q / parts, b = tm * (q + 1) / parts;
            units.push_back(Unit{i, a, b, f * (double)(b - a) / (double)tm});
        }
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.flops > y.flops; });
    std::vector<double> load(kXcds, 0.0);
    std::vector<std::vector<GroupedWork>> per(kXcds);
    for (const Unit& u : units) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += u.flops;
        const int64_t tn = cdiv(descs[u.prob].N, kGroupedTile);
        for (int64_t a = u.tm0; a < u.tm1; ++a)
            for (int64_t b = 0; b < tn; ++b) per[x].push_back(GroupedWork{(int32_t)u.prob, (int32_t)a, (int32_t)b, 0});
    }
    work.clear();
    split.off[0] = 0;
    for (int x = 0; x < kXcds; ++x) {
        std::stable_sort(per[x].begin(), per[x].end(), [&](const GroupedWork& p, const GroupedWork& q) {
            return descs[p.prob].K > descs[q.prob].K;
        });
        work.insert(work.end(), per[x].begin(), per[x].end());
        split.off[x + 1] = (int64_t)work.size();
    }
}

int grouped_grid(const GroupedSplit& split) {
    int64_t most = 0;  // the largest per-XCD range sets how many workgroups each XCD needs
    for (int x = 0; x < kXcds; ++x) most = std::max<int64_t>(most, split.off[x + 1] - split.off[x]);
    const int64_t per_xcd = std::max<int64_t>(
        1, std::min<int64_t>(cdiv(most, kGroupedWavesPerWG), (int64_t)device_cu_count() / kXcds * kGroupedWGPerCU));
    return (int)(per_xcd * kXcds);
}

int grouped_launch(int kind, const GroupedDesc* descs, const GroupedWork* work, const GroupedSplit& split, int grid,
                   float alpha, float beta, hipStream_t s) {
    if (kind != K_F16 && kind != K_BF16) return MFG_ERR_UNSUPPORTED;
    if (split.off[kXcds] == 0) return MFG_OK;
    if (grid % kXcds != 0 || grid <= 0) return MFG_ERR_INTERNAL;
    if (kind == K_F16)
        hipLaunchKernelGGL(gemm16_grouped<K_F16>, dim3(grid), dim3(256), 0, s, descs, work, split, alpha, beta);
    else
        hipLaunchKernelGGL(gemm16_grouped<K_BF16>, dim3(grid), dim3(256), 0, s, descs, work, split, alpha, beta);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

}  // namespace mfg
