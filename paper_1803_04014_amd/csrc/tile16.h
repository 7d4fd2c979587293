// tile16.h -- device code shared by the GEMM kernels on 16-bit operand planes
// (single, strided-batched and grouped launches).  Everything that decides
// the value of an output element -- the MFMA instruction, the order in which
// K chunks and products are accumulated, the epilogue -- lives here once, so
// all launch forms give bitwise-identical results for the same mode.
#pragma once

#include "device.h"
#include "internal.h"

namespace mfg {

template <int KIND>
struct KT {
    static constexpr bool BF = KIND == K_BF16 || KIND == K_BF16_SPLIT3;
    static constexpr int NPA = (KIND >= K_REFINE_A) ? 2 : 1;
    static constexpr int NPB = (KIND >= K_SPLIT3) ? 2 : 1;
    static constexpr bool LO = KIND >= K_REFINE_A;
    static constexpr bool RR = KIND == K_SPLIT4;
};

// One 16-deep K chunk of one 32x32 output tile, all products of the kind.
template <int KIND>
__device__ __forceinline__ void mma_step(const u32x4 (&a)[2], const u32x4 (&b)[2], f32x16& hi,
                                         f32x16& lo, f32x16& rr) {
    constexpr bool BF = KT<KIND>::BF;
    hi = mma_32x32x16<BF>(a[0], b[0], hi);
    if constexpr (KIND == K_REFINE_A) {
        lo = mma_32x32x16<BF>(a[1], b[0], lo);
    } else if constexpr (KIND == K_SPLIT3 || KIND == K_SPLIT4 || KIND == K_BF16_SPLIT3) {
        lo = mma_32x32x16<BF>(a[0], b[1], lo);
        lo = mma_32x32x16<BF>(a[1], b[0], lo);
        if constexpr (KIND == K_SPLIT4) rr = mma_32x32x16<BF>(a[1], b[1], rr);
    }
}

template <int KIND>
__device__ __forceinline__ float combine(float hi, float lo, float rr) {
    if constexpr (!KT<KIND>::LO) {
        return hi;
    } else {
        float l = lo;
        if constexpr (KT<KIND>::RR) l = __builtin_fmaf(rr, kResidInv, l);
        if constexpr (KIND == K_BF16_SPLIT3) return hi + l;  // unscaled residual planes
        return __builtin_fmaf(l, kResidInv, hi);
    }
}

// Value i of accumulator block (h, l, r) after combine (l, r unused, and
// never read, for kinds without them).
template <int KIND>
__device__ __forceinline__ float combine_at(const f32x16& h, const f32x16& l, const f32x16& r, int i) {
    float lv = 0.0f, rv = 0.0f;
    if constexpr (KT<KIND>::LO) lv = l[i];
    if constexpr (KT<KIND>::RR) rv = r[i];
    return combine<KIND>(h[i], lv, rv);
}


__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
    return (uint32_t)lo | ((uint32_t)hi << 16);
}

// Eight consecutive 16-bit values p[off .. off+7], zero beyond `remaining`
// or when !valid.  `vec` promises 16-byte alignment of p + off.
__device__ __forceinline__ u32x4 load_row8(const uint16_t* p, bool valid, int64_t off,
                                           int64_t remaining, bool vec) {
    if (!valid || remaining <= 0) return zero4();
    if (vec && remaining >= 8) return *reinterpret_cast<const u32x4*>(p + off);
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (j < remaining) ? p[off + j] : (uint16_t)0;
    return u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
}

// p[off + j*ld] for j = 0..7 (a column segment), zero beyond `remaining`.
__device__ __forceinline__ u32x4 load_col8(const uint16_t* p, bool valid, int64_t off, int64_t ld,
                                           int64_t remaining) {
    if (!valid || remaining <= 0) return zero4();
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (j < remaining) ? p[off + (int64_t)j * ld] : (uint16_t)0;
    return u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
}

// One 32x32 output tile at (m0, n0) of batch entry bz, computed by one
// wavefront straight from global memory.  `vecA` promises 16-byte aligned
// rows of A (lda % 8 == 0 and an aligned base).
template <int KIND>
__device__ __forceinline__ void simple_tile(const Gemm16Args& p, int64_t bz, int64_t m0, int64_t n0, int lane,
                                            int vecA) {
    using T = KT<KIND>;
    const int r = lane & 31, g = lane >> 5;
    const int64_t M = p.M, N = p.N, K = p.K;
    const uint16_t* Ap[2];
    const uint16_t* Bp[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        Ap[q] = (q < T::NPA) ? p.A[q] + bz * p.sA : nullptr;
        Bp[q] = (q < T::NPB) ? p.B[q] + bz * p.sB : nullptr;
    }
    float* C = p.C + bz * p.sC;
    const int64_t am = m0 + r, bn = n0 + r;
    f32x16 hi = {}, lo = {}, rr = {};
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        const int64_t kb = k0 + g * 8;
        u32x4 a[2] = {zero4(), zero4()}, b[2] = {zero4(), zero4()};
#pragma unroll
        for (int q = 0; q < T::NPA; ++q) a[q] = load_row8(Ap[q], am < M, am * p.lda + kb, K - kb, vecA != 0);
#pragma unroll
        for (int q = 0; q < T::NPB; ++q) b[q] = load_col8(Bp[q], bn < N, kb * p.ldb + bn, p.ldb, K - kb);
        mma_step<KIND>(a, b, hi, lo, rr);
    }
    store_blocks<1>(C, p.ldc, M, N, m0, n0, lane, p.alpha, p.beta,
                    [&](int, int i) { return combine_at<KIND>(hi, lo, rr, i); });
}

// Simple kernel: one wavefront per 32x32 output tile, operands straight from
// global memory (no LDS reuse).  Serves ragged and unaligned problems and
// tiny problems; blockIdx.z is the batch entry.
template <int KIND>
__global__ __launch_bounds__(64) void gemm16_simple(Gemm16Args p, int vecA) {
    simple_tile<KIND>(p, blockIdx.z, (int64_t)blockIdx.y * 32, (int64_t)blockIdx.x * 32, threadIdx.x, vecA);
}

// ---------------------------------------------------------------------------
// Tiled kernel: a workgroup of WM x WN wavefronts computes a BM x BN tile.
// Per BK-deep K step, A (BM x BK) and B (BK x BN) tiles of every plane are
// staged in LDS, double-buffered: the global loads of step k+1 are issued
// before the MFMAs of step k and written to the other LDS buffer after them.
//   - A is stored row-major [BM][BK] (K contiguous), 16-byte chunks XOR-
//     swizzled per row so that MFMA operand reads (32 rows, one chunk each)
//     are bank-conflict free.
//   - B arrives row-major (N contiguous) but the MFMA B operand wants eight
//     consecutive K values per lane, so each thread loads KU rows x 8
//     columns, transposes them in registers (v_perm_b32) and writes B^T
//     [BN][BK] with the same swizzle.
//   - Workgroups are renumbered so that each XCD (blocks are dealt to the 8
//     XCDs round-robin) works on a contiguous band of tiles, grouped GROUP_M
//     tile-rows high, which keeps the A and B panels of concurrently running
//     tiles in that XCD's L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int X = 8;
    const int per = nblk / X, rem = nblk % X;
    const int xcd = bid % X, idx = bid / X;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ void raster(int lid, int tiles_m, int tiles_n, int group_m, int& tm, int& tn) {
    const int group = group_m * tiles_n;
    const int gid = lid / group;
    const int first_m = gid * group_m;
    const int gm = min(tiles_m - first_m, group_m);
    const int in = lid - gid * group;
    tm = first_m + in % gm;
    tn = in / gm;
}

template <int KIND, int BM, int BN, int BK, int WM, int WN>
struct TileCfg {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int CPR = BK / 8;
    static constexpr int TMW = BM / WM, TNW = BN / WN;
    static constexpr int FM = TMW / 32, FN = TNW / 32;
    static constexpr int A_CH = BM * CPR;
    static constexpr int A_PER_T = A_CH / NT;
    static constexpr int KU_RAW = (BK * BN / 8) / NT;
    static constexpr int KU = KU_RAW >= 8 ? 8 : (KU_RAW >= 4 ? 4 : 2);
    static constexpr int B_UNITS = (BK / KU) * (BN / 8);
    static constexpr int B_PER_T = (B_UNITS + NT - 1) / NT;
    static constexpr int A_PLANE = BM * BK;
    static constexpr int B_PLANE = BN * BK;
    static constexpr int STAGE = KT<KIND>::NPA * A_PLANE + KT<KIND>::NPB * B_PLANE;
    static constexpr int LDS_BYTES = 2 * STAGE * 2;
    static_assert(A_CH % NT == 0, "A tile must split evenly over threads");
    static_assert(BK % 16 == 0 && (CPR == 4 || CPR == 8), "BK must be 32 or 64");
    static_assert(TMW % 32 == 0 && TNW % 32 == 0, "wave tile must be a multiple of 32");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
};

// One BM x BN output tile at (m0, n0) of a single GEMM whose planes are Ap /
// Bp (already offset to the right batch entry).  `lds` must hold
// TileCfg::LDS_BYTES.  Called by every workgroup thread.
template <int KIND, int BM, int BN, int BK, int WM, int WN>
__device__ __forceinline__ void tile_gemm(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2],
                                          float* C, int64_t M, int64_t N, int64_t K, int64_t lda,
                                          int64_t ldb, int64_t ldc, float alpha, float beta, int64_t m0,
                                          int64_t n0, uint16_t* lds) {
    using T = KT<KIND>;
    using G = TileCfg<KIND, BM, BN, BK, WM, WN>;
    constexpr int NT = G::NT, CPR = G::CPR, KU = G::KU;
    constexpr int FM = G::FM, FN = G::FN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const bool mn_interior = (m0 + BM <= M) && (n0 + BN <= N);

    u32x4 ra[T::NPA][G::A_PER_T];
    u32x4 rb[T::NPB][G::B_PER_T][KU];

    auto gload = [&](int64_t k0) {
        const bool interior = mn_interior && (k0 + BK <= K);
#pragma unroll
        for (int q = 0; q < T::NPA; ++q) {
#pragma unroll
            for (int i = 0; i < G::A_PER_T; ++i) {
                const int id = tid + i * NT;
                const int row = id / CPR, c = id % CPR;
                const int64_t gm = m0 + row, gk = k0 + c * 8;
                if (interior)
                    ra[q][i] = *reinterpret_cast<const u32x4*>(Ap[q] + gm * lda + gk);
                else
                    ra[q][i] = load_row8(Ap[q], gm < M, gm * lda + gk, K - gk, true);
            }
        }
#pragma unroll
        for (int q = 0; q < T::NPB; ++q) {
#pragma unroll
            for (int u = 0; u < G::B_PER_T; ++u) {
                const int uid = tid + u * NT;
                if (G::B_UNITS % NT == 0 || uid < G::B_UNITS) {
                    const int qn = uid % (BN / 8), gk_ = uid / (BN / 8);
                    const int64_t gn = n0 + qn * 8;
#pragma unroll
                    for (int i = 0; i < KU; ++i) {
                        const int64_t gk = k0 + gk_ * KU + i;
                        if (interior)
                            rb[q][u][i] = *reinterpret_cast<const u32x4*>(Bp[q] + gk * ldb + gn);
                        else
                            rb[q][u][i] = load_row8(Bp[q], gk < K, gk * ldb + gn, N - gn, true);
                    }
                }
            }
        }
    };

    auto swrite = [&](int stage) {
        uint16_t* base = lds + stage * G::STAGE;
#pragma unroll
        for (int q = 0; q < T::NPA; ++q) {
            uint16_t* As = base + q * G::A_PLANE;
#pragma unroll
            for (int i = 0; i < G::A_PER_T; ++i) {
                const int id = tid + i * NT;
                const int row = id / CPR, c = id % CPR;
                *reinterpret_cast<u32x4*>(As + row * BK + ((c ^ swz<CPR>(row)) * 8)) = ra[q][i];
            }
        }
#pragma unroll
        for (int q = 0; q < T::NPB; ++q) {
            uint16_t* Bs = base + T::NPA * G::A_PLANE + q * G::B_PLANE;
#pragma unroll
            for (int u = 0; u < G::B_PER_T; ++u) {
                const int uid = tid + u * NT;
                if (G::B_UNITS % NT == 0 || uid < G::B_UNITS) {
                    const int qn = uid % (BN / 8), gk_ = uid / (BN / 8);
                    const int kl = gk_ * KU;  // local k of this unit
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int w = j >> 1;
                        const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
                        uint32_t words[KU / 2];
#pragma unroll
                        for (int pp = 0; pp < KU / 2; ++pp)
                            words[pp] = __builtin_amdgcn_perm(rb[q][u][2 * pp + 1][w], rb[q][u][2 * pp][w], sel);
                        const int n = qn * 8 + j;
                        uint16_t* dst = Bs + n * BK + (((kl >> 3) ^ swz<CPR>(n)) * 8) + (kl & 7);
                        if constexpr (KU == 8)
                            *reinterpret_cast<u32x4*>(dst) = u32x4{words[0], words[1], words[2], words[3]};
                        else if constexpr (KU == 4)
                            *reinterpret_cast<u32x2*>(dst) = u32x2{words[0], words[1]};
                        else
                            *reinterpret_cast<uint32_t*>(dst) = words[0];
                    }
                }
            }
        }
    };

    f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            hi[i][j] = f32x16{};
            if constexpr (T::LO) lo[i][j] = f32x16{};
            if constexpr (T::RR) rr[i][j] = f32x16{};
        }

    auto compute = [&](int stage) {
        const uint16_t* base = lds + stage * G::STAGE;
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            const int c = kk * 2 + (lane >> 5);
            u32x4 af[FM][2], bf[FN][2];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * G::TMW + fm * 32 + (lane & 31);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (q < T::NPA)
                        af[fm][q] = *reinterpret_cast<const u32x4*>(base + q * G::A_PLANE + row * BK +
                                                                    ((c ^ swz<CPR>(row)) * 8));
                    else
                        af[fm][q] = zero4();
                }
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int n = wn * G::TNW + fn * 32 + (lane & 31);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (q < T::NPB)
                        bf[fn][q] = *reinterpret_cast<const u32x4*>(base + T::NPA * G::A_PLANE + q * G::B_PLANE +
                                                                    n * BK + ((c ^ swz<CPR>(n)) * 8));
                    else
                        bf[fn][q] = zero4();
                }
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) mma_step<KIND>(af[fm], bf[fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
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

    store_tile<FM, FN>(C, ldc, M, N, m0 + wm * G::TMW, n0 + wn * G::TNW, lane, alpha, beta,
                       [&](int fm, int fn, int i) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], i); });
}

template <int KIND, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm16_tiled(Gemm16Args p, int tiles_m, int tiles_n,
                                                             int group_m) {
    using T = KT<KIND>;
    extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
    int tm, tn;
    raster(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, group_m, tm, tn);
    const int64_t bz = blockIdx.y;
    const uint16_t* Ap[2];
    const uint16_t* Bp[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        Ap[q] = (q < T::NPA) ? p.A[q] + bz * p.sA : nullptr;
        Bp[q] = (q < T::NPB) ? p.B[q] + bz * p.sB : nullptr;
    }
    tile_gemm<KIND, BM, BN, BK, WM, WN>(Ap, Bp, p.C + bz * p.sC, p.M, p.N, p.K, p.lda, p.ldb, p.ldc,
                                        p.alpha, p.beta, (int64_t)tm * BM, (int64_t)tn * BN, lds);
}

}  // namespace mfg
