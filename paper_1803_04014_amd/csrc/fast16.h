// fast16.h -- the throughput kernel for 16-bit operand planes on gfx950.
//
// Same arithmetic as tile16.h (same MFMA, same K order, same epilogue, so
// results are bitwise identical), organised for the matrix cores:
//   - A (M x K, K contiguous) and B (K x N, N contiguous) tiles stream from
//     HBM into LDS in their natural row-major layout, 16 bytes per lane,
//     either straight into LDS (global_load_lds_dwordx4: no VGPR staging, no
//     ds_write) or through VGPRs (DMA = false).  A wavefront's load fills
//     1 KB of LDS contiguously, so the swizzle is applied by choosing which
//     global chunk each lane fetches.
//   - The MFMA A operand (eight K-consecutive values per lane) is one
//     ds_read_b128 per 32x32 sub-tile.  The B operand (eight K-consecutive
//     values of one column) comes from two ds_read_b64_tr_b16: in each group
//     of 16 lanes, lane 4j+q points at 4 columns of row j and lane i receives
//     column i of the 4 rows, i.e. the transpose happens in the LDS read.
//   - LDS swizzles (16-byte chunks): an A row of BK = 64 halfs stores chunk
//     c at c ^ ((r ^ (r >> 3)) & 7), a row of BK = 32 at
//     c ^ (((r >> 1) ^ (r >> 3)) & 3); B row k stores chunk c at c ^ F[k & 3]
//     with F = {0, 6, 12, 10}.  Both make the operand reads bank-conflict free for
//     a 32-bank (128 B) and a 64-bank (256 B) LDS.
//   - Two LDS stages.  A K step first reads all of its operand fragments
//     from LDS, then issues the loads of step t+1 into the other stage, then
//     runs its MFMAs while those loads are in flight; one barrier per step.
//     (Issuing the loads before the fragment reads would make the compiler
//     wait for them first: it cannot tell the two LDS stages apart.)
//   - M/N edges: rows/columns past the matrix are clamped to the last valid
//     one (their products only reach outputs that are not stored), so the
//     main loop has no branches.  K must be a multiple of BK.
#pragma once

#include "tile16.h"

namespace mfg {

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int swzB(int k) {
    // F = {0, 6, 12, 10} for k % 4 = 0, 1, 2, 3
    return (int)((0xA0C0600u >> ((k & 3) * 8)) & 0xFu);
}

template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK_ = 64>
struct FastCfg {
    static constexpr int BK = BK_;
    static constexpr int CPR = BK / 8;            // 16-byte chunks per A row
    static constexpr int A_ROWS_PER_INSTR = 512 / BK;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int NW = WM * WN;
    static constexpr int TMW = BM / WM, TNW = BN / WN;
    static constexpr int FM = TMW / 32, FN = TNW / 32;
    static constexpr int A_PLANE = BM * BK;  // halfs
    static constexpr int B_PLANE = BK * BN;
    static constexpr int NPA = KT<KIND>::NPA, NPB = KT<KIND>::NPB;
    static constexpr int STAGE = NPA * A_PLANE + NPB * B_PLANE;
    static constexpr int LDS_BYTES = 2 * STAGE * 2;
    // 1 KB (512 halfs) per wavefront load instruction
    static constexpr int A_INSTR = A_PLANE / 512 / NW;  // per wave, per plane
    static constexpr int B_INSTR = B_PLANE / 512 / NW;
    static constexpr int B_ROWS_PER_INSTR = 512 / BN;   // rows of B filled by one instruction
    static constexpr int B_CPR = BN / 8;                // 16-byte chunks per B row
    static_assert(A_PLANE % (512 * NW) == 0 && B_PLANE % (512 * NW) == 0, "tile must split into 1 KB loads");
    static_assert(BN == 128 || BN == 256, "B rows of 256 or 512 bytes");
    static_assert(BK == 32 || BK == 64, "BK of 32 or 64");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
};

// Staging registers of the VGPR path (unused when loads go straight to LDS).
template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK>
struct FastRegs {
    using G = FastCfg<KIND, BM, BN, WM, WN, DMA, BK>;
    u32x4 a[DMA ? 1 : G::NPA][DMA ? 1 : G::A_INSTR];
    u32x4 b[DMA ? 1 : G::NPB][DMA ? 1 : G::B_INSTR];
};

// Issue the loads of one K step (all planes) for LDS stage `dst`: straight
// into LDS (DMA) or into `regs`, written by fast_store after the MFMAs.
template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK>
__device__ __forceinline__ void fast_load(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2],
                                          int64_t lda, int64_t ldb, int64_t M, int64_t N, int64_t m0,
                                          int64_t n0, int64_t k0, uint16_t* dst, int wid, int lane,
                                          FastRegs<KIND, BM, BN, WM, WN, DMA, BK>& regs) {
    using G = FastCfg<KIND, BM, BN, WM, WN, DMA, BK>;
#pragma unroll
    for (int q = 0; q < G::NPA; ++q) {
        uint16_t* As = dst + q * G::A_PLANE;
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i) {
            const int blk = wid * G::A_INSTR + i;       // 1 KB block = 512/BK rows of BK halfs
            const int row = blk * G::A_ROWS_PER_INSTR + lane / G::CPR;
            const int c = (lane % G::CPR) ^ swz<G::CPR>(row);  // logical chunk stored at physical lane % CPR
            int64_t gm = m0 + row;
            gm = gm < M ? gm : M - 1;
            const uint16_t* src = Ap[q] + gm * lda + k0 + c * 8;
            uint16_t* d = As + blk * 512;
            if constexpr (DMA) {
                __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)d, 16, 0, 0);
            } else {
                regs.a[q][i] = *reinterpret_cast<const u32x4*>(src);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < G::NPB; ++q) {
        uint16_t* Bs = dst + G::NPA * G::A_PLANE + q * G::B_PLANE;
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i) {
            const int blk = wid * G::B_INSTR + i;
            const int krow = blk * G::B_ROWS_PER_INSTR + lane / G::B_CPR;
            const int c = (lane % G::B_CPR) ^ swzB(krow);
            int64_t gn = n0 + c * 8;
            gn = gn + 8 <= N ? gn : N - 8;
            const uint16_t* src = Bp[q] + (k0 + krow) * ldb + gn;
            uint16_t* d = Bs + blk * 512;
            if constexpr (DMA) {
                __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)d, 16, 0, 0);
            } else {
                regs.b[q][i] = *reinterpret_cast<const u32x4*>(src);
            }
        }
    }
}

// VGPR path: write the staged K step into LDS stage `dst` (same layout as DMA).
template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK>
__device__ __forceinline__ void fast_store(uint16_t* dst, int wid, int lane,
                                           const FastRegs<KIND, BM, BN, WM, WN, DMA, BK>& regs) {
    using G = FastCfg<KIND, BM, BN, WM, WN, DMA, BK>;
    if constexpr (!DMA) {
#pragma unroll
        for (int q = 0; q < G::NPA; ++q)
#pragma unroll
            for (int i = 0; i < G::A_INSTR; ++i)
                *reinterpret_cast<u32x4*>(dst + q * G::A_PLANE + (wid * G::A_INSTR + i) * 512 + lane * 8) = regs.a[q][i];
#pragma unroll
        for (int q = 0; q < G::NPB; ++q)
#pragma unroll
            for (int i = 0; i < G::B_INSTR; ++i)
                *reinterpret_cast<u32x4*>(dst + G::NPA * G::A_PLANE + q * G::B_PLANE + (wid * G::B_INSTR + i) * 512 +
                                          lane * 8) = regs.b[q][i];
    }
}

__device__ __forceinline__ void wait_vm0() {
    // s_waitcnt vmcnt(0): every global (and global->LDS) load of this wave done.
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// B operand of one 32x32x16 MFMA from a row-major B tile that starts
// `boff` halfs into the LDS array `st`: rows kb..kb+15 of columns nb..nb+31
// (lane l: column l % 32, rows kb + 8 (l/32) + 0..7).  Both reads are formed
// as one offset from the array base so the compiler can tell which array
// (pipeline stage) they touch.
template <int BN>
__device__ __forceinline__ u32x4 read_b_tr(const uint16_t* st, int boff, int kb, int nb, int lane) {
    const int w = lane & 15, j = w >> 2, q = w & 3;
    const int h = (lane >> 4) & 1, g = lane >> 5;
    const int n = nb + h * 16 + q * 4;
    const int c = n >> 3, off = n & 7;
    const int k1 = kb + g * 8 + j;  // k1 and k1 + 4 share k % 4
    const int o1 = boff + k1 * BN + ((c ^ swzB(k1)) << 3) + off;
    const int o2 = o1 + 4 * BN;
    i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4*)(st + o1));
    i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4*)(st + o2));
    u32x2 a = __builtin_bit_cast(u32x2, lo), b = __builtin_bit_cast(u32x2, hi);
    return u32x4{a[0], a[1], b[0], b[1]};
}

template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK_>
__device__ __forceinline__ void fast_tile(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2], float* C,
                                          int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb, int64_t ldc,
                                          float alpha, float beta, int64_t m0, int64_t n0, uint16_t* lds) {
    using T = KT<KIND>;
    using G = FastCfg<KIND, BM, BN, WM, WN, DMA, BK_>;
    constexpr int FM = G::FM, FN = G::FN, BK = G::BK, CPR = G::CPR;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;

    f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            hi[i][j] = f32x16{};
            if constexpr (T::LO) lo[i][j] = f32x16{};
            if constexpr (T::RR) rr[i][j] = f32x16{};
        }

    const int64_t KTN = K / BK;
    FastRegs<KIND, BM, BN, WM, WN, DMA, BK> regs;
    fast_load<KIND, BM, BN, WM, WN, DMA, BK>(Ap, Bp, lda, ldb, M, N, m0, n0, 0, lds, wid, lane, regs);
    fast_store<KIND, BM, BN, WM, WN, DMA, BK>(lds, wid, lane, regs);
    if constexpr (DMA) wait_vm0();
    __syncthreads();
    for (int64_t kt = 0; kt < KTN; ++kt) {
        const uint16_t* cur = lds + (kt & 1) * G::STAGE;
        // 1. every operand fragment of this K step, from LDS into VGPRs
        u32x4 af[BK / 16][FM][2], bf[BK / 16][FN][2];
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            const int c = kk * 2 + (lane >> 5);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * G::TMW + fm * 32 + (lane & 31);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    af[kk][fm][q] = (q < T::NPA) ? *reinterpret_cast<const u32x4*>(cur + q * G::A_PLANE + row * BK +
                                                                                   ((c ^ swz<CPR>(row)) * 8))
                                                 : zero4();
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    bf[kk][fn][q] = (q < T::NPB) ? read_b_tr<BN>(cur, T::NPA * G::A_PLANE + q * G::B_PLANE, kk * 16,
                                                                 wn * G::TNW + fn * 32, lane)
                                                 : zero4();
            }
        }
        // 2. the next K step's loads into the other stage (after the reads in
        //    program order, so no wait on them is needed before those reads)
        if (kt + 1 < KTN)
            fast_load<KIND, BM, BN, WM, WN, DMA, BK>(Ap, Bp, lda, ldb, M, N, m0, n0, (kt + 1) * BK,
                                                 lds + ((kt + 1) & 1) * G::STAGE, wid, lane, regs);
        // 3. the MFMAs, while those loads are in flight
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk)
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    mma_step<KIND>(af[kk][fm], bf[kk][fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
        // keep the MFMAs ahead of the wait for the next step's loads
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DMA) {
            wait_vm0();
        } else {
            if (kt + 1 < KTN) fast_store<KIND, BM, BN, WM, WN, DMA, BK>(lds + ((kt + 1) & 1) * G::STAGE, wid, lane, regs);
        }
        __syncthreads();
    }

    store_tile<FM, FN>(C, ldc, M, N, m0 + wm * G::TMW, n0 + wn * G::TNW, lane, alpha, beta,
                       [&](int fm, int fn, int i) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], i); });
}

template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK, int OCC = 1>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm16_fast(Gemm16Args p, int tiles_m, int tiles_n, int group_m) {
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
    fast_tile<KIND, BM, BN, WM, WN, DMA, BK>(Ap, Bp, p.C + bz * p.sC, p.M, p.N, p.K, p.lda, p.ldb, p.ldc, p.alpha,
                                         p.beta, (int64_t)tm * BM, (int64_t)tn * BN, lds);
}

}  // namespace mfg
