// batched.hip -- many small GEMMs (paper Sec. IV.B and Sec. VI: batched GEMM
// of many 16x16 problems, one warp per problem, 16 problems per block).
//
//   gemm16_batched_small : uniform strided batch with M, N <= 32.  Each
//     wavefront owns one problem at a time (one 32x32x16 MFMA per 16-deep K
//     chunk, rows/columns beyond M/N masked) and walks the batch with a
//     grid-wide stride, so the grid stays at a few waves per SIMD however
//     large the batch is.  Operands are read once: the batch is HBM-bound
//     (16^3: 2 KB and 8 Kflop per problem).
//   gemm16_grouped : thousands of GEMMs of different shapes in one
//     persistent launch.  The work list holds one entry per 64x64 output
//     tile of every problem (ordered by decreasing K, the tile's cost);
//     workgroups take entries with a static grid stride.  Aligned problems
//     run the LDS-staged tile; others the per-wave global-memory tile.
// Both reuse the tile functions of the single GEMM, so each problem's result
// is bitwise identical to mfg_gemm on that problem alone.
#include "tile16.h"

namespace mfg {

template <int KIND>
__global__ __launch_bounds__(256) void gemm16_batched_small(Gemm16Args p, int64_t count, int vecA) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < count; b += nwaves)
        simple_tile<KIND>(p, b, 0, 0, lane, vecA);
}

int launch_batched_small(int kind, const Gemm16Args& a, int64_t count, bool vec_ok, int num_cu, hipStream_t s) {
    if (a.M > 32 || a.N > 32) return MFG_ERR_INTERNAL;
    const int64_t want = cdiv(count, 4);
    const int64_t cap = (int64_t)num_cu * 16;  // 16 workgroups (64 waves) per CU
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    if (grid == 0) return MFG_OK;
    const int v = vec_ok ? 1 : 0;
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
constexpr int kGroupTile = 64;
using GroupCfg = TileCfg<K_F16, 64, 64, 64, 2, 2>;

template <int KIND>
__global__ __launch_bounds__(256) void gemm16_grouped(const GroupedDesc* descs, const GroupedWork* work,
                                                      int64_t nwork, float alpha, float beta) {
    extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t i = blockIdx.x; i < nwork; i += gridDim.x) {
        const GroupedWork w = work[i];
        const GroupedDesc d = descs[w.prob];
        const int64_t m0 = (int64_t)w.tm * kGroupTile, n0 = (int64_t)w.tn * kGroupTile;
        if (d.vec) {
            const uint16_t* Ap[2] = {d.A, nullptr};
            const uint16_t* Bp[2] = {d.B, nullptr};
            tile_gemm<KIND, 64, 64, 64, 2, 2>(Ap, Bp, d.C, d.M, d.N, d.K, d.lda, d.ldb, d.ldc, alpha, beta, m0, n0,
                                              lds);
            __syncthreads();  // the next item overwrites the LDS tiles
        } else {
            Gemm16Args p{};
            p.M = d.M, p.N = d.N, p.K = d.K;
            p.A[0] = d.A, p.B[0] = d.B, p.C = d.C;
            p.lda = d.lda, p.ldb = d.ldb, p.ldc = d.ldc;
            p.alpha = alpha, p.beta = beta;
            simple_tile<KIND>(p, 0, m0 + 32 * (wid >> 1), n0 + 32 * (wid & 1), lane, 0);
        }
    }
}

int grouped_lds_bytes() { return GroupCfg::LDS_BYTES; }

int grouped_launch(int kind, const GroupedDesc* descs, const GroupedWork* work, int64_t nwork, int grid, float alpha,
                   float beta, hipStream_t s) {
    static bool attr_set[2] = {false, false};
    const int lds = GroupCfg::LDS_BYTES;
    if (kind == K_F16) {
        if (!attr_set[0]) {
            MFG_HIP_CHECK(hipFuncSetAttribute((const void*)gemm16_grouped<K_F16>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
            attr_set[0] = true;
        }
        if (nwork == 0) return MFG_OK;
        hipLaunchKernelGGL(gemm16_grouped<K_F16>, dim3(grid), dim3(256), lds, s, descs, work, nwork, alpha, beta);
    } else if (kind == K_BF16) {
        if (!attr_set[1]) {
            MFG_HIP_CHECK(hipFuncSetAttribute((const void*)gemm16_grouped<K_BF16>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
            attr_set[1] = true;
        }
        if (nwork == 0) return MFG_OK;
        hipLaunchKernelGGL(gemm16_grouped<K_BF16>, dim3(grid), dim3(256), lds, s, descs, work, nwork, alpha, beta);
    } else {
        return MFG_ERR_UNSUPPORTED;
    }
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

}  // namespace mfg
