// pipe16.h -- multi-stage pipelined GEMM kernel for 16-bit operand planes.
//
// Same arithmetic and LDS layout as fast16.h (bitwise-identical results),
// with a deeper pipeline for the one-wavefront-per-SIMD regime of large
// tiles:
//   - S LDS stages of BK = 32, each its own __shared__ array.  Distinct
//     arrays let the compiler see that a read of stage s does not alias the
//     global->LDS loads still in flight into the other stages, so its own
//     wait insertion stays precise; loads run S-1 steps ahead.
//   - Operand fragments are double-buffered in VGPRs: while the MFMAs of
//     step t run, the fragments of step t+1 are read from LDS, interleaved
//     one read per MFMA (sched_group_barrier), so LDS latency hides under
//     the matrix cores.
//   - One barrier per step, a bare s_barrier (__syncthreads() would also
//     wait for the loads that must stay in flight).  At the top of step t:
//     wait for this wave's loads of step t+1 and its LDS reads, barrier
//     (everyone's loads landed; everyone's reads of step t's array, done
//     during step t-1, completed), then refill that array with step t+S.  Past the last step the refill fetches the last
//     step again (valid addresses, never read), so wait counts are fixed.
#pragma once

#include <type_traits>

#include "fast16.h"

namespace mfg {

template <int KIND, int BM, int BN, int WM, int WN, int S>
struct PipeCfg {
    static constexpr int BK = 32;
    static constexpr int NT = 64 * WM * WN, NW = WM * WN;
    static constexpr int TMW = BM / WM, TNW = BN / WN;
    static constexpr int FM = TMW / 32, FN = TNW / 32;
    static constexpr int NPA = KT<KIND>::NPA, NPB = KT<KIND>::NPB;
    static constexpr int A_PLANE = BM * BK, B_PLANE = BK * BN;  // halfs
    static constexpr int STAGE = NPA * A_PLANE + NPB * B_PLANE;
    static constexpr int LDS_BYTES = S * STAGE * 2;
    static constexpr int A_INSTR = A_PLANE / 512 / NW;  // 1 KB loads per wave per plane
    static constexpr int B_INSTR = B_PLANE / 512 / NW;
    static constexpr int LOADS = NPA * A_INSTR + NPB * B_INSTR;  // per wave per stage
    static constexpr int B_ROWS_PER_INSTR = 512 / BN, B_CPR = BN / 8;
    static constexpr int READS = 2 * (FM * NPA + 2 * FN * NPB);  // LDS reads per wave per step
    static constexpr int PRODUCTS = KIND == K_REFINE_A ? 2 : (KIND == K_SPLIT3 || KIND == K_BF16_SPLIT3) ? 3 : KIND == K_SPLIT4 ? 4 : 1;
    static constexpr int MFMAS = 2 * FM * FN * PRODUCTS;  // per wave per step
    static_assert(A_PLANE % (512 * NW) == 0 && B_PLANE % (512 * NW) == 0, "tile must split into 1 KB loads");
    static_assert(BN == 128 || BN == 256, "B rows of 256 or 512 bytes");
    static_assert(S == 4, "4 stages: the fragment double buffer alternates with the step parity only for an even unroll");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(LOADS * (S - 1) <= 63, "vmcnt range");
};

// Global -> LDS loads of one BK = 32 step into stage array `st`.  The A tile
// row has 4 chunks of 16 bytes (64 B); a 1 KB load fills 16 rows.  Chunk c of
// row r sits at c ^ ((r >> 1 ^ r >> 3) & 3): conflict-free A operand reads.
template <int KIND, int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void pipe_load(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2],
                                          int64_t lda, int64_t ldb, int64_t M, int64_t N, int64_t m0, int64_t n0,
                                          int64_t k0, uint16_t* st, int wid, int lane) {
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
#pragma unroll
    for (int q = 0; q < G::NPA; ++q) {
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i) {
            const int blk = wid * G::A_INSTR + i;  // 16 rows of 32 halfs
            const int row = blk * 16 + (lane >> 2);
            const int c = (lane & 3) ^ swz<4>(row);
            int64_t gm = m0 + row;
            gm = gm < M ? gm : M - 1;
            const int loff = q * G::A_PLANE + blk * 512;
            __builtin_amdgcn_global_load_lds((const void*)(Ap[q] + gm * lda + k0 + c * 8), (lds_void*)(st + loff), 16,
                                             0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < G::NPB; ++q) {
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i) {
            const int blk = wid * G::B_INSTR + i;
            const int krow = blk * G::B_ROWS_PER_INSTR + lane / G::B_CPR;
            const int c = (lane % G::B_CPR) ^ swzB(krow);
            int64_t gn = n0 + c * 8;
            gn = gn + 8 <= N ? gn : N - 8;
            const int loff = G::NPA * G::A_PLANE + q * G::B_PLANE + blk * 512;
            __builtin_amdgcn_global_load_lds((const void*)(Bp[q] + (k0 + krow) * ldb + gn), (lds_void*)(st + loff), 16,
                                             0, 0);
        }
    }
}

template <int KIND, int BM, int BN, int WM, int WN, int S>
struct PipeFrags {
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
    u32x4 a[2][G::FM][2];
    u32x4 b[2][G::FN][2];
};

template <int KIND, int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void pipe_read(const uint16_t* st, int wm, int wn, int lane,
                                          PipeFrags<KIND, BM, BN, WM, WN, S>& f) {
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
    using T = KT<KIND>;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const int c = kk * 2 + (lane >> 5);
#pragma unroll
        for (int fm = 0; fm < G::FM; ++fm) {
            const int row = wm * G::TMW + fm * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < 2; ++q)
                f.a[kk][fm][q] = (q < T::NPA) ? *reinterpret_cast<const u32x4*>(
                                                    st + (q * G::A_PLANE + row * 32 + ((c ^ swz<4>(row)) * 8)))
                                              : zero4();
        }
#pragma unroll
        for (int fn = 0; fn < G::FN; ++fn) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
                f.b[kk][fn][q] = (q < T::NPB) ? read_b_tr<BN>(st, G::NPA * G::A_PLANE + q * G::B_PLANE, kk * 16,
                                                              wn * G::TNW + fn * 32, lane)
                                              : zero4();
        }
    }
}

template <int KIND, int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void pipe_mma(const PipeFrags<KIND, BM, BN, WM, WN, S>& f,
                                         f32x16 (&hi)[PipeCfg<KIND, BM, BN, WM, WN, S>::FM][PipeCfg<KIND, BM, BN, WM, WN, S>::FN],
                                         f32x16 (&lo)[PipeCfg<KIND, BM, BN, WM, WN, S>::FM][PipeCfg<KIND, BM, BN, WM, WN, S>::FN],
                                         f32x16 (&rr)[PipeCfg<KIND, BM, BN, WM, WN, S>::FM][PipeCfg<KIND, BM, BN, WM, WN, S>::FN]) {
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int fm = 0; fm < G::FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < G::FN; ++fn) mma_step<KIND>(f.a[kk][fm], f.b[kk][fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
}

// s_waitcnt vmcnt(n) (gfx9 encoding: vmcnt bits [3:0] and [15:14]; expcnt
// and lgkmcnt left at their no-wait maxima).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// s_waitcnt lgkmcnt(0): this wave's LDS reads have returned their data.
__device__ __forceinline__ void wait_lgkm0() {
    __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4));
}

// Workgroup barrier without __syncthreads()'s release fence: that fence
// waits for every outstanding memory operation of the wave, including the
// global->LDS loads of later stages that must stay in flight.  The caller
// waits for exactly what the other wavefronts need first; the compiler-only
// fences keep LDS accesses on their side of the barrier.
__device__ __forceinline__ void bare_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Interleave: one LDS read after each MFMA until the reads run out.
template <int READS, int MFMAS>
__device__ __forceinline__ void pipe_interleave() {
#pragma unroll
    for (int i = 0; i < (READS < MFMAS ? READS : MFMAS); ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
    }
}

// Even interleave: the LDS reads spread over all MFMAs of the step (one read
// after MFMA i when floor((i+1) READS / MFMAS) grows), instead of one after
// each of the first READS MFMAs.
template <int READS, int MFMAS>
__device__ __forceinline__ void pipe_interleave_even() {
#pragma unroll
    for (int i = 0; i < MFMAS; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if ((i + 1) * READS / MFMAS > i * READS / MFMAS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
}

template <int READS, int LOADS, int MFMAS>
__device__ __forceinline__ void pipe_interleave_loads_even() {
#pragma unroll
    for (int i = 0; i < MFMAS; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if ((i + 1) * READS / MFMAS > i * READS / MFMAS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if ((i + 1) * LOADS / MFMAS > i * LOADS / MFMAS) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
}

// Interleave of the step that also issues the next stage's global->LDS
// loads: MFMA, LDS read, global load, ... while each kind lasts.  Issued in
// one burst, the loads back up in the texture-address unit and hold the
// wave (and with it its SIMD's matrix core) at issue.
template <int READS, int LOADS, int MFMAS>
__device__ __forceinline__ void pipe_interleave_loads() {
#pragma unroll
    for (int i = 0; i < MFMAS; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                 // one MFMA
        if (i < READS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
        if (i < LOADS) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one global load
    }
}

template <int KIND, int BM, int BN, int WM, int WN, int S>
__global__ __launch_bounds__(64 * WM * WN) void gemm16_pipe(Gemm16Args p, int tiles_m, int tiles_n, int group_m) {
    using T = KT<KIND>;
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
    constexpr int FM = G::FM, FN = G::FN, BK = G::BK;
    __shared__ __attribute__((aligned(16))) uint16_t st0[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint16_t st1[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint16_t st2[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint16_t st3[G::STAGE];

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
    float* C = p.C + bz * p.sC;
    const int64_t M = p.M, N = p.N, K = p.K, lda = p.lda, ldb = p.ldb;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int64_t KTN = K / BK;  // >= 1
    auto kclamp = [&](int64_t t) { return (t < KTN ? t : KTN - 1) * BK; };
    auto stage = [&](int s) -> uint16_t* { return s == 0 ? st0 : s == 1 ? st1 : s == 2 ? st2 : st3; };


    f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            hi[i][j] = f32x16{};
            if constexpr (T::LO) lo[i][j] = f32x16{};
            if constexpr (T::RR) rr[i][j] = f32x16{};
        }

    // prologue: steps 0 .. S-1 in flight; wait for step 0 and read its fragments
#pragma unroll
    for (int s = 0; s < S; ++s)
        pipe_load<KIND, BM, BN, WM, WN, S>(Ap, Bp, lda, ldb, M, N, m0, n0, kclamp(s), stage(s), wid, lane);
    PipeFrags<KIND, BM, BN, WM, WN, S> f[2];
    wait_vmcnt<G::LOADS * (S - 1)>();
    bare_barrier();
    pipe_read<KIND, BM, BN, WM, WN, S>(st0, wm, wn, lane, f[0]);

    // One step: wait + barrier, refill the freed array, read the next
    // step's fragments (always: past the end they are simply unused),
    // MFMAs of this step interleaved with those reads.
    auto step = [&](auto ucst, int64_t t) {
        constexpr int u = decltype(ucst)::value;
        wait_vmcnt<G::LOADS * (S - 2)>();  // this wave's loads of step t+1 landed
        wait_lgkm0();                      // this wave's reads of step t's array returned
        bare_barrier();
        pipe_load<KIND, BM, BN, WM, WN, S>(Ap, Bp, lda, ldb, M, N, m0, n0, kclamp(t + S), stage(u), wid, lane);
        pipe_read<KIND, BM, BN, WM, WN, S>(stage((u + 1) % S), wm, wn, lane, f[(u + 1) & 1]);
        pipe_mma<KIND, BM, BN, WM, WN, S>(f[u & 1], hi, lo, rr);
        pipe_interleave<G::READS, G::MFMAS>();
        __builtin_amdgcn_sched_barrier(0);
    };
    // main loop over whole groups of S steps (stage arrays named statically, no branches)
    const int64_t KFULL = KTN - KTN % S;
    for (int64_t t0 = 0; t0 < KFULL; t0 += S) {
        step(std::integral_constant<int, 0>{}, t0);
        step(std::integral_constant<int, 1>{}, t0 + 1);
        step(std::integral_constant<int, 2>{}, t0 + 2);
        step(std::integral_constant<int, 3>{}, t0 + 3);
    }
    // remaining KTN % S steps
    if (KFULL < KTN) step(std::integral_constant<int, 0>{}, KFULL);
    if (KFULL + 1 < KTN) step(std::integral_constant<int, 1>{}, KFULL + 1);
    if (KFULL + 2 < KTN) step(std::integral_constant<int, 2>{}, KFULL + 2);

    wait_vmcnt<0>();  // no global->LDS load may outlive the workgroup's LDS
    store_tile<FM, FN>(C, p.ldc, M, N, m0 + wm * G::TMW, n0 + wn * G::TNW, lane, p.alpha, p.beta,
                       [&](int fm, int fn, int i) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], i); });
}


// ---------------------------------------------------------------------------
// gemm16_pipe64: the same pipeline with LDS stages 64 wide in K.
//
// An A tile row of a BK = 32 stage is 64 bytes, half of a 128-byte cache line,
// so every A line is requested twice and the load path moves ~40% fewer bytes
// per clock than with whole lines (measured on MI355X: ~16 vs ~27 TB/s of
// L2 -> LDS streaming).  Here a stage holds K = 64 (A rows of 128 bytes, the
// BK = 64 swizzle of fast16.h), while the operand fragments stay double-
// buffered at 32-wide half steps, which keeps the register budget of a
// 256 x 256 tile (256 accumulators + 2 x 64 fragment VGPRs):
// KK = 2: fragment steps of 32 (two per stage); KK = 1: of 16 (four per
// stage), which halves the fragment registers (measured slower for the
// tiles in the menus, so they all use KK = 2):
//   fragment steps but the last:  read the next step's fragments into the
//                                 other buffer, MFMAs on this one;
//   the last:                     wait for stage T+1's loads and this wave's
//                                 LDS reads, barrier, refill stage T's array
//                                 with step T+S, read T+1's first fragments,
//                                 MFMAs.
// Loads run S-1 stage steps ahead; one barrier per stage step.
template <int KIND, int BM, int BN, int WM, int WN, int S, int KK = 2>
struct Pipe64Cfg {
    static constexpr int BK = 64;
    static constexpr int KSUB = 4 / KK;  // fragment steps per stage (KK 16-deep chunks each)
    static constexpr int NT = 64 * WM * WN, NW = WM * WN;
    static constexpr int TMW = BM / WM, TNW = BN / WN;
    static constexpr int FM = TMW / 32, FN = TNW / 32;
    static constexpr int NPA = KT<KIND>::NPA, NPB = KT<KIND>::NPB;
    static constexpr int A_PLANE = BM * BK, B_PLANE = BK * BN;  // halfs
    static constexpr int STAGE = NPA * A_PLANE + NPB * B_PLANE;
    static constexpr int LDS_BYTES = S * STAGE * 2;
    static constexpr int A_INSTR = A_PLANE / 512 / NW;
    static constexpr int B_INSTR = B_PLANE / 512 / NW;
    static constexpr int LOADS = NPA * A_INSTR + NPB * B_INSTR;  // per wave per stage
    static constexpr int B_ROWS_PER_INSTR = 512 / BN, B_CPR = BN / 8;
    static constexpr int READS = KK * (FM * NPA + 2 * FN * NPB);  // LDS reads per wave per fragment step
    static constexpr int PRODUCTS = KIND == K_REFINE_A ? 2 : (KIND == K_SPLIT3 || KIND == K_BF16_SPLIT3) ? 3 : KIND == K_SPLIT4 ? 4 : 1;
    static constexpr int MFMAS = KK * FM * FN * PRODUCTS;  // per wave per fragment step
    static_assert(A_PLANE % (512 * NW) == 0 && B_PLANE % (512 * NW) == 0, "tile must split into 1 KB loads");
    static_assert(BN == 128 || BN == 256, "B rows of 256 or 512 bytes");
    static_assert(S == 2 || S == 3, "2 or 3 stages");
    static_assert(KK == 1 || KK == 2, "fragment steps of 16 or 32");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(LOADS * (S - 1) <= 63, "vmcnt range");
};

// Global -> LDS loads of one 64-wide stage into array `st`: A rows of 8
// chunks (a 1 KB load fills 8 rows; chunk c of row r at c ^ swz<8>(r)), B
// rows as in fast16.h.
template <int KIND, int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void pipe64_load(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2],
                                            int64_t lda, int64_t ldb, int64_t M, int64_t N, int64_t m0, int64_t n0,
                                            int64_t k0, uint16_t* st, int wid, int lane) {
    using G = Pipe64Cfg<KIND, BM, BN, WM, WN, S>;
#pragma unroll
    for (int q = 0; q < G::NPA; ++q) {
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i) {
            const int blk = wid * G::A_INSTR + i;  // 8 rows of 64 halfs
            const int row = blk * 8 + (lane >> 3);
            const int c = (lane & 7) ^ swz<8>(row);
            int64_t gm = m0 + row;
            gm = gm < M ? gm : M - 1;
            const int loff = q * G::A_PLANE + blk * 512;
            __builtin_amdgcn_global_load_lds((const void*)(Ap[q] + gm * lda + k0 + c * 8), (lds_void*)(st + loff), 16,
                                             0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < G::NPB; ++q) {
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i) {
            const int blk = wid * G::B_INSTR + i;
            const int krow = blk * G::B_ROWS_PER_INSTR + lane / G::B_CPR;
            const int c = (lane % G::B_CPR) ^ swzB(krow);
            int64_t gn = n0 + c * 8;
            gn = gn + 8 <= N ? gn : N - 8;
            const int loff = G::NPA * G::A_PLANE + q * G::B_PLANE + blk * 512;
            __builtin_amdgcn_global_load_lds((const void*)(Bp[q] + (k0 + krow) * ldb + gn), (lds_void*)(st + loff), 16,
                                             0, 0);
        }
    }
}

// The same loads with their addressing split into a per-lane part fixed for
// the whole K loop and a per-stage part that is the same in every lane.  Each
// lane's byte offset from the tile's corner (A: row m0, column 0 of the stage;
// B: row 0 of the stage, column n0), with the row clamps and the swizzled
// chunk of pipe64_load, is computed once (32 bits: the caller guarantees
// BM * lda and BK * ldb below 2^30 elements); a stage adds its K offset to
// the corner in scalar registers, and the LDS destinations come from the
// wavefront index made visibly uniform, so a load costs one address add
// instead of a 64-bit multiply per lane.  Same sources, same LDS layout and
// the same instruction order as pipe64_load.
template <int KIND, int BM, int BN, int WM, int WN, int S>
struct P64Loader {
    using G = Pipe64Cfg<KIND, BM, BN, WM, WN, S>;
    const char* a[2];  // tile corner of each A plane, row m0 (same in every lane)
    const char* b[2];  // of each B plane, column n0
    int64_t ldb2;      // B row pitch in bytes
    int wid;           // this wavefront's index (scalar)
    uint32_t offa[G::A_INSTR];
    uint32_t offb[G::B_INSTR];

    __device__ __forceinline__ void init(const uint16_t* const (&Ap)[2], const uint16_t* const (&Bp)[2], int64_t lda,
                                         int64_t ldb, int64_t M, int64_t N, int64_t m0, int64_t n0, int wid_, int lane) {
        wid = __builtin_amdgcn_readfirstlane(wid_);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            a[q] = (const char*)uniform64((int64_t)(Ap[q] ? Ap[q] + m0 * lda : nullptr));
            b[q] = (const char*)uniform64((int64_t)(Bp[q] ? Bp[q] + n0 : nullptr));
        }
        ldb2 = uniform64(ldb * 2);
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i) {
            const int row = (wid * G::A_INSTR + i) * 8 + (lane >> 3);
            const int c = (lane & 7) ^ swz<8>(row);
            const int64_t gm = m0 + row < M ? m0 + row : M - 1;
            offa[i] = (uint32_t)(((gm - m0) * lda + c * 8) * 2);
        }
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i) {
            const int krow = (wid * G::B_INSTR + i) * G::B_ROWS_PER_INSTR + lane / G::B_CPR;
            const int c = (lane % G::B_CPR) ^ swzB(krow);
            const int64_t gn = n0 + c * 8 + 8 <= N ? n0 + c * 8 : N - 8;
            offb[i] = (uint32_t)((krow * ldb + (gn - n0)) * 2);
        }
    }

    // The loads of the stage starting at column (A) / row (B) k0 into `st`.
    __device__ __forceinline__ void load(int64_t k0, uint16_t* st) const {
        const int64_t ka = uniform64(k0 * 2), kb = uniform64(k0 * ldb2);
#pragma unroll
        for (int q = 0; q < G::NPA; ++q)
#pragma unroll
            for (int i = 0; i < G::A_INSTR; ++i)
                __builtin_amdgcn_global_load_lds((const void*)(a[q] + ka + offa[i]),
                                                 (lds_void*)(st + q * G::A_PLANE + (wid * G::A_INSTR + i) * 512), 16,
                                                 0, 0);
#pragma unroll
        for (int q = 0; q < G::NPB; ++q)
#pragma unroll
            for (int i = 0; i < G::B_INSTR; ++i)
                __builtin_amdgcn_global_load_lds(
                    (const void*)(b[q] + kb + offb[i]),
                    (lds_void*)(st + G::NPA * G::A_PLANE + q * G::B_PLANE + (wid * G::B_INSTR + i) * 512), 16, 0, 0);
    }
};

// Operand fragments of one fragment step: KK 16-deep chunks.
template <int FM, int FN, int KK>
struct P64Frags {
    u32x4 a[KK][FM][2];
    u32x4 b[KK][FN][2];
};

// Fragments of fragment step h (chunks KK h .. KK h + KK - 1 of the 64-wide
// stage in `st`).
template <int KIND, int BM, int BN, int WM, int WN, int S, int KK>
__device__ __forceinline__ void pipe64_read(const uint16_t* st, int h, int wm, int wn, int lane,
                                            P64Frags<Pipe64Cfg<KIND, BM, BN, WM, WN, S, KK>::FM,
                                                     Pipe64Cfg<KIND, BM, BN, WM, WN, S, KK>::FN, KK>& f) {
    using G = Pipe64Cfg<KIND, BM, BN, WM, WN, S, KK>;
    using T = KT<KIND>;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
        const int ch = h * KK + kk;             // 16-deep chunk of the stage
        const int c = ch * 2 + (lane >> 5);      // 16-byte chunk of the 64-wide row
#pragma unroll
        for (int fm = 0; fm < G::FM; ++fm) {
            const int row = wm * G::TMW + fm * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < 2; ++q)
                f.a[kk][fm][q] = (q < T::NPA) ? *reinterpret_cast<const u32x4*>(
                                                    st + (q * G::A_PLANE + row * 64 + ((c ^ swz<8>(row)) * 8)))
                                              : zero4();
        }
#pragma unroll
        for (int fn = 0; fn < G::FN; ++fn) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
                f.b[kk][fn][q] = (q < T::NPB) ? read_b_tr<BN>(st, G::NPA * G::A_PLANE + q * G::B_PLANE, ch * 16,
                                                              wn * G::TNW + fn * 32, lane)
                                              : zero4();
        }
    }
}

template <int KIND, int BM, int BN, int WM, int WN, int S, int KK, bool EVEN = false>
__global__ __launch_bounds__(64 * WM * WN) void gemm16_pipe64(Gemm16Args p, int tiles_m, int tiles_n, int group_m) {
    using T = KT<KIND>;
    using G = Pipe64Cfg<KIND, BM, BN, WM, WN, S, KK>;
    constexpr int FM = G::FM, FN = G::FN, BK = G::BK, KSUB = G::KSUB;
    using F = P64Frags<FM, FN, KK>;
    __shared__ __attribute__((aligned(16))) uint16_t st0[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint16_t st1[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint16_t st2[S == 3 ? G::STAGE : 8];

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
    float* C = p.C + bz * p.sC;
    const int64_t M = p.M, N = p.N, K = p.K, lda = p.lda, ldb = p.ldb;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int64_t KTN = uniform64(K / BK);  // >= 1
    auto kclamp = [&](int64_t t) { return (t < KTN ? t : KTN - 1) * BK; };
    auto stage = [&](int s) -> uint16_t* { return s == 0 ? st0 : s == 1 ? st1 : st2; };

    f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            hi[i][j] = f32x16{};
            if constexpr (T::LO) lo[i][j] = f32x16{};
            if constexpr (T::RR) rr[i][j] = f32x16{};
        }

    P64Loader<KIND, BM, BN, WM, WN, S> ld;
    ld.init(Ap, Bp, lda, ldb, M, N, m0, n0, wid, lane);

    // prologue: stages 0 .. S-1 in flight; wait for stage 0, read its first fragments
#pragma unroll
    for (int s = 0; s < S; ++s) ld.load(kclamp(s), stage(s));
    F f[2];
    wait_vmcnt<G::LOADS * (S - 1)>();
    bare_barrier();
    pipe64_read<KIND, BM, BN, WM, WN, S, KK>(st0, 0, wm, wn, lane, f[0]);

    auto mma = [&](const F& fr) {
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    mma_step<KIND>(fr.a[kk][fm], fr.b[kk][fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
    };
    // One stage step T (u = T % S, a compile-time constant inside the
    // unrolled loop): KSUB fragment steps; each reads the next step's
    // fragments while its MFMAs run.  Before the last one, whose read
    // crosses into stage T+1: wait for that stage's loads (this wave) and
    // for this wave's reads of stage T, barrier, refill stage T's array with
    // step T+S.  KSUB is even, so fragment step h always uses f[h & 1].
    auto step = [&](auto ucst, int64_t t) {
        constexpr int u = decltype(ucst)::value;
#pragma unroll
        for (int h = 0; h < KSUB; ++h) {
            if (h == KSUB - 1) {
                wait_vmcnt<G::LOADS * (S - 2)>();
                wait_lgkm0();
                bare_barrier();
                ld.load(kclamp(t + S), stage(u));
                pipe64_read<KIND, BM, BN, WM, WN, S, KK>(stage((u + 1) % S), 0, wm, wn, lane, f[(h + 1) & 1]);
                mma(f[h & 1]);
                if constexpr (EVEN) pipe_interleave_loads_even<G::READS, G::LOADS, G::MFMAS>();
                else pipe_interleave_loads<G::READS, G::LOADS, G::MFMAS>();
            } else {
                pipe64_read<KIND, BM, BN, WM, WN, S, KK>(stage(u), h + 1, wm, wn, lane, f[(h + 1) & 1]);
                mma(f[h & 1]);
                if constexpr (EVEN) pipe_interleave_even<G::READS, G::MFMAS>();
                else pipe_interleave<G::READS, G::MFMAS>();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    const int64_t KFULL = KTN - KTN % S;
    for (int64_t t0 = 0; t0 < KFULL; t0 += S) {
        step(std::integral_constant<int, 0>{}, t0);
        step(std::integral_constant<int, 1>{}, t0 + 1);
        if constexpr (S == 3) step(std::integral_constant<int, 2>{}, t0 + 2);
    }
    if (KFULL < KTN) step(std::integral_constant<int, 0>{}, KFULL);
    if constexpr (S == 3)
        if (KFULL + 1 < KTN) step(std::integral_constant<int, 1>{}, KFULL + 1);

    wait_vmcnt<0>();  // no global->LDS load may outlive the workgroup's LDS
    store_tile<FM, FN>(C, p.ldc, M, N, m0 + wm * G::TMW, n0 + wn * G::TNW, lane, p.alpha, p.beta,
                       [&](int fm, int fn, int i) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], i); });
}

}  // namespace mfg
