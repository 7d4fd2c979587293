// gemm_f32.hip -- single-precision GEMM on the gfx950 matrix cores
// (v_mfma_f32_32x32x2_f32): the FP32 comparator of the half-precision modes
// (the paper's single-precision GEMM, Sec. VII.A and the error reference of
// Sec. VI).
//
// Accumulation order of an output element, shared by every kernel here: K
// is walked in blocks of 8; inside a block, four MFMAs j = 0..3 each add the
// products at k = kb + j (lane half 0) and k = kb + 4 + j (lane half 1).
#include "device.h"
#include "internal.h"
#include "runtime.h"

namespace mfg {

__device__ __forceinline__ f32x4 load_row4(const float* p, bool valid, int64_t off, int64_t remaining,
                                           bool vec) {
    if (!valid || remaining <= 0) return f32x4{0.f, 0.f, 0.f, 0.f};
    if (vec && remaining >= 4) return *reinterpret_cast<const f32x4*>(p + off);
    f32x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (j < remaining) ? p[off + j] : 0.0f;
    return v;
}

// One wavefront per 32x32 tile, operands from global memory.
__global__ __launch_bounds__(64) void gemmf32_simple(GemmF32Args p, int vecA) {
    const int lane = threadIdx.x;
    const int r = lane & 31, g = lane >> 5;
    const int64_t bz = blockIdx.z;
    const int64_t m0 = (int64_t)blockIdx.y * 32, n0 = (int64_t)blockIdx.x * 32;
    const float* A = p.A + bz * p.sA;
    const float* B = p.B + bz * p.sB;
    float* C = p.C + bz * p.sC;
    const int64_t am = m0 + r, bn = n0 + r;
    f32x16 acc = {};
    for (int64_t kb = 0; kb < p.K; kb += 8) {
        const int64_t k = kb + g * 4;
        f32x4 a = load_row4(A, am < p.M, am * p.lda + k, p.K - k, vecA != 0);
        f32x4 b;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (bn < p.N && k + j < p.K) ? B[(k + j) * p.ldb + bn] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = mma_32x32x2_f32(a[j], b[j], acc);
    }
    store_blocks<1>(C, p.ldc, p.M, p.N, m0, n0, lane, p.alpha, p.beta, [&](int, int i) { return acc[i]; });
}

__device__ __forceinline__ int xcd_remap_f32(int bid, int nblk) {
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = bid % 8, idx = bid / 8;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Tiled FP32 kernel: BM x BN tile, BK = 32 (eight 16-byte chunks per LDS
// row, XOR-swizzled), 2x2 wavefronts, LDS double buffer.  B is transposed
// through registers into B^T [BN][BK] (4 rows x 4 columns per thread).
template <int BM, int BN>
__global__ __launch_bounds__(256) void gemmf32_tiled(GemmF32Args p, int tiles_m, int tiles_n, int group_m) {
    constexpr int BK = 32, CPR = 8, NT = 256, WM = 2, WN = 2;
    constexpr int TMW = BM / WM, TNW = BN / WN, FM = TMW / 32, FN = TNW / 32;
    constexpr int A_PER_T = BM * CPR / NT;
    constexpr int B_UNITS = (BK / 4) * (BN / 4);
    constexpr int B_PER_T = B_UNITS / NT;
    constexpr int STAGE = (BM + BN) * BK;
    static_assert(B_UNITS % NT == 0 && (BM * CPR) % NT == 0, "tile/thread split");
    extern __shared__ __attribute__((aligned(16))) float ldsf[];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    int tm, tn;
    {
        const int lid = xcd_remap_f32(blockIdx.x, gridDim.x);
        const int group = group_m * tiles_n, gid = lid / group, first_m = gid * group_m;
        const int gm = min(tiles_m - first_m, group_m), in = lid - gid * group;
        tm = first_m + in % gm;
        tn = in / gm;
    }
    const int64_t bz = blockIdx.y;
    const float* A = p.A + bz * p.sA;
    const float* B = p.B + bz * p.sB;
    float* C = p.C + bz * p.sC;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int64_t M = p.M, N = p.N, K = p.K;
    const bool mn_interior = (m0 + BM <= M) && (n0 + BN <= N);

    f32x4 ra[A_PER_T];
    f32x4 rb[B_PER_T][4];
    auto gload = [&](int64_t k0) {
        const bool interior = mn_interior && (k0 + BK <= K);
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int id = tid + i * NT, row = id / CPR, c = id % CPR;
            const int64_t gm = m0 + row, gk = k0 + c * 4;
            ra[i] = interior ? *reinterpret_cast<const f32x4*>(A + gm * p.lda + gk)
                             : load_row4(A, gm < M, gm * p.lda + gk, K - gk, true);
        }
#pragma unroll
        for (int u = 0; u < B_PER_T; ++u) {
            const int uid = tid + u * NT;
            const int qn = uid % (BN / 4), gk_ = uid / (BN / 4);
            const int64_t gn = n0 + qn * 4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t gk = k0 + gk_ * 4 + i;
                rb[u][i] = interior ? *reinterpret_cast<const f32x4*>(B + gk * p.ldb + gn)
                                    : load_row4(B, gk < K, gk * p.ldb + gn, N - gn, true);
            }
        }
    };
    auto swrite = [&](int stage) {
        float* As = ldsf + stage * STAGE;
        float* Bs = As + BM * BK;
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int id = tid + i * NT, row = id / CPR, c = id % CPR;
            *reinterpret_cast<f32x4*>(As + row * BK + ((c ^ swz<CPR>(row)) * 4)) = ra[i];
        }
#pragma unroll
        for (int u = 0; u < B_PER_T; ++u) {
            const int uid = tid + u * NT;
            const int qn = uid % (BN / 4), gk_ = uid / (BN / 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = qn * 4 + j;
                f32x4 v = {rb[u][0][j], rb[u][1][j], rb[u][2][j], rb[u][3][j]};
                *reinterpret_cast<f32x4*>(Bs + n * BK + ((gk_ ^ swz<CPR>(n)) * 4)) = v;
            }
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

    auto compute = [&](int stage) {
        const float* As = ldsf + stage * STAGE;
        const float* Bs = As + BM * BK;
#pragma unroll
        for (int kk = 0; kk < BK / 8; ++kk) {
            const int c = kk * 2 + (lane >> 5);
            f32x4 af[FM], bf[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * TMW + fm * 32 + (lane & 31);
                af[fm] = *reinterpret_cast<const f32x4*>(As + row * BK + ((c ^ swz<CPR>(row)) * 4));
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int n = wn * TNW + fn * 32 + (lane & 31);
                bf[fn] = *reinterpret_cast<const f32x4*>(Bs + n * BK + ((c ^ swz<CPR>(n)) * 4));
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                    for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = mma_32x32x2_f32(af[fm][j], bf[fn][j], acc[fm][fn]);
        }
    };

    const int64_t KTN = cdiv(K, BK);
    if (KTN > 0) {
        gload(0);
        swrite(0);
        __syncthreads();
        for (int64_t kt = 0; kt < KTN; ++kt) {
            const int cur = (int)(kt & 1);
            if (kt + 1 < KTN) gload((kt + 1) * BK);
            compute(cur);
            if (kt + 1 < KTN) swrite(cur ^ 1);
            __syncthreads();
        }
    }
    store_tile<FM, FN>(C, p.ldc, M, N, m0 + wm * TMW, n0 + wn * TNW, lane, p.alpha, p.beta,
                       [&](int fm, int fn, int i) { return acc[fm][fn][i]; });
}

struct CfgF32 {
    const char* name;
    int bm, bn, group_m;
};
static const CfgF32 kCfgF32[] = {
    {"simple32", 0, 0, 0},
    {"t128x128k32w2x2g8", 128, 128, 8},
    {"t256x128k32w2x2g8", 256, 128, 8},
};

int num_configs_f32() { return (int)(sizeof(kCfgF32) / sizeof(kCfgF32[0])); }
const char* config_f32_name(int cfg) { return (cfg >= 0 && cfg < num_configs_f32()) ? kCfgF32[cfg].name : nullptr; }

template <int BM, int BN>
static int launch_f32_tiled(const GemmF32Args& a, int64_t batch, int group_m, hipStream_t s) {
    constexpr int lds = 2 * (BM + BN) * 32 * 4;
    auto kern = gemmf32_tiled<BM, BN>;
    static bool attr_set = false;
    if (!attr_set) {
        MFG_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        attr_set = true;
    }
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    hipLaunchKernelGGL(kern, dim3(tiles_m * tiles_n, (unsigned)batch), dim3(256), lds, s, a, tiles_m, tiles_n,
                       group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

bool config_f32_ok(int cfg, int64_t ldc, bool vec_ok) {
    if (cfg < 0 || cfg >= num_configs_f32()) return false;
    return cfg == 0 || (vec_ok && buffer_ldc_ok(ldc));
}

int launch_gemm_f32(int cfg, const GemmF32Args& a, int64_t batch, bool vec_ok, hipStream_t s) {
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    if (cfg < 0 || cfg >= num_configs_f32()) return MFG_ERR_INVALID_ARG;
    if (cfg != 0 && (!vec_ok || !buffer_ldc_ok(a.ldc))) return MFG_ERR_UNSUPPORTED;
    const CfgF32& c = kCfgF32[cfg];
    if (c.bm == 0) {
        dim3 grid((unsigned)cdiv(a.N, 32), (unsigned)cdiv(a.M, 32), (unsigned)batch);
        hipLaunchKernelGGL(gemmf32_simple, grid, dim3(64), 0, s, a, vec_ok ? 1 : 0);
        MFG_LAUNCH_CHECK();
        return MFG_OK;
    }
    if (c.bm == 128) return launch_f32_tiled<128, 128>(a, batch, c.group_m, s);
    if (c.bm == 256) return launch_f32_tiled<256, 128>(a, batch, c.group_m, s);
    return MFG_ERR_INTERNAL;
}

}  // namespace mfg
