// gemm_f8.hip -- FP8-E4M3 GEMM with per-128x128-tile power-of-two scales on
// the gfx950 matrix cores (v_mfma_scale_f32_32x32x64_f8f6f4).
//
// A tile scale is 2^E with E in [-127, 127], so it is passed to the MFMA as
// its E8M0 block-scale code E + 127 and applied in hardware:
//   acc += (2^Ea * qA) (2^Eb * qB)  over each 64-deep K chunk.
// A 64-deep chunk never straddles a 128-wide K tile and a 32-row / 32-column
// output block never straddles a 128 tile, so one scale per operand applies
// to the whole instruction.  Accumulation order: K chunks 0, 64, 128, ...
#include <type_traits>

#include "device.h"
#include "internal.h"
#include "pipe16.h"
#include "runtime.h"

namespace mfg {

// E8M0 code of a power-of-two FP32 scale 2^E (E in [-127, 127]): the biased
// exponent field; 2^-127 is the FP32 subnormal with field 0, code 0.
__device__ __forceinline__ int e8m0_code(float s) {
    return (int)((__builtin_bit_cast(uint32_t, s) >> 23) & 0xFFu);
}

// One wavefront per 32x32 output tile; operands from global memory.  Lane
// (r, g) supplies the 32 codes k = k0 + 32 g + 0..31 of A row r and of B
// column r.
__global__ __launch_bounds__(64) void gemmf8_simple(GemmF8Args p, int vecA) {
    const int lane = threadIdx.x;
    const int r = lane & 31, g = lane >> 5;
    const int64_t m0 = (int64_t)blockIdx.y * 32, n0 = (int64_t)blockIdx.x * 32;
    const int64_t am = m0 + r, bn = n0 + r;
    const int64_t ktiles = cdiv(p.K, MFG_FP8_TILE), ntiles = cdiv(p.N, MFG_FP8_TILE);
    const int64_t mt = m0 / MFG_FP8_TILE, nt = n0 / MFG_FP8_TILE;
    f32x16 acc = {};
    for (int64_t k0 = 0; k0 < p.K; k0 += 64) {
        const int64_t kb = k0 + g * 32;
        const int64_t kt = k0 / MFG_FP8_TILE;
        union {
            i32x8 v;
            uint8_t b[32];
            u32x4 q[2];
        } a, b;
        if (am < p.M && vecA && kb + 32 <= p.K) {
            a.q[0] = *reinterpret_cast<const u32x4*>(p.A + am * p.lda + kb);
            a.q[1] = *reinterpret_cast<const u32x4*>(p.A + am * p.lda + kb + 16);
        } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) a.b[j] = (am < p.M && kb + j < p.K) ? p.A[am * p.lda + kb + j] : (uint8_t)0;
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) b.b[j] = (bn < p.N && kb + j < p.K) ? p.B[(kb + j) * p.ldb + bn] : (uint8_t)0;
        const int sa = e8m0_code(p.sa[mt * ktiles + kt]);
        const int sb = e8m0_code(p.sb[kt * ntiles + nt]);
        acc = mma_32x32x64_e4m3(a.v, b.v, acc, sa, sb);
    }
    store_blocks<1>(p.C, p.ldc, p.M, p.N, m0, n0, lane, p.alpha, p.beta, [&](int, int i) { return acc[i]; });
}

// ---------------------------------------------------------------------------
// gemmf8_pipe: the tiled FP8 kernel.  A (M x K) and Bt = B^T (N x K) are both
// K-contiguous code matrices, so both operands load and read the same way:
// LDS stages of 128 K (rows of 128 bytes = one cache line, chunk c of row r
// at c ^ swz<8>(r), conflict-free), a lane's 32 codes are two ds_read_b128.
// Each output still accumulates K chunks 0, 64, 128, ... with the same lane
// data and the same scale codes as gemmf8_simple, so results are bitwise
// identical.  Pipeline as gemm16_pipe64: S stages in distinct __shared__
// arrays, fragments double-buffered per 64-deep half step, one barrier per
// stage, loads S-1 stages ahead.  K must be a multiple of 128; M / N edges
// clamp rows (and tile-scale indices) to the last valid one.
template <int BM, int BN, int WM, int WN, int S>
struct F8Cfg {
    static constexpr int BK = 128;  // bytes = codes
    static constexpr int NT = 64 * WM * WN, NW = WM * WN;
    static constexpr int TMW = BM / WM, TNW = BN / WN;
    static constexpr int FM = TMW / 32, FN = TNW / 32;
    static constexpr int A_PLANE = BM * BK, B_PLANE = BN * BK;  // bytes
    static constexpr int STAGE = A_PLANE + B_PLANE;
    static constexpr int A_INSTR = A_PLANE / 1024 / NW, B_INSTR = B_PLANE / 1024 / NW;
    static constexpr int LOADS = A_INSTR + B_INSTR;
    static constexpr int READS = 2 * (FM + FN);  // per wave per half step
    static constexpr int MFMAS = FM * FN;        // per wave per half step
    static_assert(A_PLANE % (1024 * NW) == 0 && B_PLANE % (1024 * NW) == 0, "tile must split into 1 KB loads");
    static_assert(TMW <= 128 && TNW <= 128 && 128 % TMW == 0 && 128 % TNW == 0, "a wave's rows lie in one scale tile");
    static_assert(S * STAGE <= 160 * 1024, "LDS budget");
    static_assert(LOADS * (S - 1) <= 63, "vmcnt range");
};

template <int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void f8_load(const uint8_t* A, const uint8_t* Bt, int64_t lda, int64_t ldbt, int64_t M,
                                        int64_t N, int64_t m0, int64_t n0, int64_t k0, uint8_t* st, int wid,
                                        int lane) {
    using G = F8Cfg<BM, BN, WM, WN, S>;
    const int rr = lane >> 3;                 // 8 rows of 128 bytes per 1 KB load
#pragma unroll
    for (int i = 0; i < G::A_INSTR; ++i) {
        const int blk = wid * G::A_INSTR + i;
        const int row = blk * 8 + rr;
        const int c = (lane & 7) ^ swz<8>(row);
        int64_t gm = m0 + row;
        gm = gm < M ? gm : M - 1;
        __builtin_amdgcn_global_load_lds((const void*)(A + gm * lda + k0 + c * 16), (lds_void*)(st + blk * 1024), 16,
                                         0, 0);
    }
#pragma unroll
    for (int i = 0; i < G::B_INSTR; ++i) {
        const int blk = wid * G::B_INSTR + i;
        const int row = blk * 8 + rr;
        const int c = (lane & 7) ^ swz<8>(row);
        int64_t gn = n0 + row;
        gn = gn < N ? gn : N - 1;
        __builtin_amdgcn_global_load_lds((const void*)(Bt + gn * ldbt + k0 + c * 16),
                                         (lds_void*)(st + G::A_PLANE + blk * 1024), 16, 0, 0);
    }
}

// f8_load with the addressing of P64Loader: each lane's byte offset from the
// tile's corner (A row m0, Bt row n0) fixed for the K loop, the stage's K
// offset and the LDS destinations in scalar registers.  Same sources, LDS
// layout and instruction order as f8_load.
template <int BM, int BN, int WM, int WN, int S>
struct F8Loader {
    using G = F8Cfg<BM, BN, WM, WN, S>;
    const uint8_t* a;
    const uint8_t* b;
    int wid;
    uint32_t offa[G::A_INSTR], offb[G::B_INSTR];

    __device__ __forceinline__ void init(const uint8_t* A, const uint8_t* Bt, int64_t lda, int64_t ldbt, int64_t M,
                                         int64_t N, int64_t m0, int64_t n0, int wid_, int lane) {
        wid = __builtin_amdgcn_readfirstlane(wid_);
        a = (const uint8_t*)uniform64((int64_t)(A + m0 * lda));
        b = (const uint8_t*)uniform64((int64_t)(Bt + n0 * ldbt));
        const int rr = lane >> 3;
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i) {
            const int row = (wid * G::A_INSTR + i) * 8 + rr;
            const int c = (lane & 7) ^ swz<8>(row);
            const int64_t gm = m0 + row < M ? m0 + row : M - 1;
            offa[i] = (uint32_t)((gm - m0) * lda + c * 16);
        }
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i) {
            const int row = (wid * G::B_INSTR + i) * 8 + rr;
            const int c = (lane & 7) ^ swz<8>(row);
            const int64_t gn = n0 + row < N ? n0 + row : N - 1;
            offb[i] = (uint32_t)((gn - n0) * ldbt + c * 16);
        }
    }

    __device__ __forceinline__ void load(int64_t k0, uint8_t* st) const {
        const int64_t k = uniform64(k0);
#pragma unroll
        for (int i = 0; i < G::A_INSTR; ++i)
            __builtin_amdgcn_global_load_lds((const void*)(a + k + offa[i]),
                                             (lds_void*)(st + (wid * G::A_INSTR + i) * 1024), 16, 0, 0);
#pragma unroll
        for (int i = 0; i < G::B_INSTR; ++i)
            __builtin_amdgcn_global_load_lds((const void*)(b + k + offb[i]),
                                             (lds_void*)(st + G::A_PLANE + (wid * G::B_INSTR + i) * 1024), 16, 0, 0);
    }
};

template <int FM, int FN>
struct F8Frags {
    i32x8 a[FM];
    i32x8 b[FN];
};

// Lane (r, g) of a 32-row block: the 32 codes at K offset 64 h + 32 g of row r.
__device__ __forceinline__ i32x8 f8_read_row(const uint8_t* st, int off, int row, int h, int lane) {
    const int c0 = h * 4 + (lane >> 5) * 2;  // first of the lane's two 16-byte chunks
    const u32x4 lo = *reinterpret_cast<const u32x4*>(st + off + row * 128 + ((c0 ^ swz<8>(row)) << 4));
    const u32x4 hi = *reinterpret_cast<const u32x4*>(st + off + row * 128 + (((c0 + 1) ^ swz<8>(row)) << 4));
    return i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
}

template <int BM, int BN, int WM, int WN, int S>
__device__ __forceinline__ void f8_read(const uint8_t* st, int h, int wm, int wn, int lane,
                                        F8Frags<F8Cfg<BM, BN, WM, WN, S>::FM, F8Cfg<BM, BN, WM, WN, S>::FN>& f) {
    using G = F8Cfg<BM, BN, WM, WN, S>;
#pragma unroll
    for (int fm = 0; fm < G::FM; ++fm) f.a[fm] = f8_read_row(st, 0, wm * G::TMW + fm * 32 + (lane & 31), h, lane);
#pragma unroll
    for (int fn = 0; fn < G::FN; ++fn)
        f.b[fn] = f8_read_row(st, G::A_PLANE, wn * G::TNW + fn * 32 + (lane & 31), h, lane);
}

template <int BM, int BN, int WM, int WN, int S, bool EVEN = false>
__global__ __launch_bounds__(64 * WM * WN) void gemmf8_pipe(GemmF8Args p, int tiles_m, int tiles_n, int group_m) {
    using G = F8Cfg<BM, BN, WM, WN, S>;
    constexpr int FM = G::FM, FN = G::FN, BK = G::BK;
    using F = F8Frags<FM, FN>;
    __shared__ __attribute__((aligned(16))) uint8_t st0[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint8_t st1[G::STAGE];
    __shared__ __attribute__((aligned(16))) uint8_t st2[S == 3 ? G::STAGE : 16];

    int tm, tn;
    raster(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, group_m, tm, tn);
    const int64_t M = p.M, N = p.N, K = p.K;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int64_t KTN = uniform64(K / BK);  // >= 1
    auto kclamp = [&](int64_t t) { return (t < KTN ? t : KTN - 1) * BK; };
    auto stage = [&](int s) -> uint8_t* { return s == 0 ? st0 : s == 1 ? st1 : st2; };
    // this wave's scale tiles (rows clamped like the operand rows)
    const int64_t ktiles = cdiv(K, MFG_FP8_TILE), ntiles = cdiv(N, MFG_FP8_TILE), mtiles = cdiv(M, MFG_FP8_TILE);
    int64_t mt = (m0 + wm * G::TMW) / MFG_FP8_TILE, nt = (n0 + wn * G::TNW) / MFG_FP8_TILE;
    mt = mt < mtiles ? mt : mtiles - 1;
    nt = nt < ntiles ? nt : ntiles - 1;
    const float* sa_row = p.sa + mt * ktiles;
    const float* sb_col = p.sb + nt;
    // Stage t's scale values (one 128-wide scale tile per stage).  A step
    // loads the next stage's values at its start and turns them into codes
    // only at its end, behind a scheduling barrier: extracted at once, the
    // codes made the wait for those loads (vmcnt 0) also wait for the stage
    // loads in flight, at every stage.
    auto scale_vals = [&](int64_t t, float& va, float& vb) {
        const int64_t kt = t < KTN ? t : KTN - 1;
        va = sa_row[kt];
        vb = sb_col[kt * ntiles];
    };
    auto scale_codes = [&](int64_t t, int& ca, int& cb) {
        float va, vb;
        scale_vals(t, va, vb);
        ca = e8m0_code(va);
        cb = e8m0_code(vb);
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

    F8Loader<BM, BN, WM, WN, S> ld;
    ld.init(p.A, p.Bt, p.lda, p.ldbt, M, N, m0, n0, wid, lane);
#pragma unroll
    for (int s = 0; s < S; ++s) ld.load(kclamp(s), stage(s));
    int ca, cb;
    float va, vb;
    scale_codes(0, ca, cb);
    F f[2];
    wait_vmcnt<G::LOADS * (S - 1)>();
    bare_barrier();
    f8_read<BM, BN, WM, WN, S>(st0, 0, wm, wn, lane, f[0]);

    auto mma = [&](const F& fr, int sa, int sb) {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = mma_32x32x64_e4m3(fr.a[fm], fr.b[fn], acc[fm][fn], sa, sb);
    };
    auto step = [&](auto ucst, int64_t t) {
        constexpr int u = decltype(ucst)::value;
        scale_vals(t + 1, va, vb);  // next stage's scale values, early
        f8_read<BM, BN, WM, WN, S>(stage(u), 1, wm, wn, lane, f[1]);
        mma(f[0], ca, cb);
        if constexpr (EVEN) pipe_interleave_even<G::READS, G::MFMAS>();
        else pipe_interleave<G::READS, G::MFMAS>();
        __builtin_amdgcn_sched_barrier(0);
        wait_vmcnt<G::LOADS * (S - 2)>();
        wait_lgkm0();
        bare_barrier();
        ld.load(kclamp(t + S), stage(u));
        f8_read<BM, BN, WM, WN, S>(stage((u + 1) % S), 0, wm, wn, lane, f[0]);
        mma(f[1], ca, cb);
        // the stage's global->LDS loads spread over the MFMAs as well: issued in
        // one burst they back up in the texture-address unit and hold the wave
        if constexpr (EVEN) pipe_interleave_loads_even<G::READS, G::LOADS, G::MFMAS>();
        else pipe_interleave_loads<G::READS, G::LOADS, G::MFMAS>();
        __builtin_amdgcn_sched_barrier(0);
        ca = e8m0_code(va), cb = e8m0_code(vb);
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

    wait_vmcnt<0>();
    store_tile<FM, FN>(p.C, p.ldc, M, N, m0 + wm * G::TMW, n0 + wn * G::TNW, lane, p.alpha, p.beta,
                       [&](int fm, int fn, int i) { return acc[fm][fn][i]; });
}

struct CfgF8 {
    const char* name;
    int bm, bn, wm, wn, s, group_m;
};
static const CfgF8 kCfgF8[] = {
    {"simple32", 0, 0, 0, 0, 0, 0},
    {"p256x256k128s2w2x2g8", 256, 256, 2, 2, 2, 8},
    {"p128x128k128s3w2x2g8", 128, 128, 2, 2, 3, 8},
    {"p256x128k128s2w2x2g8", 256, 128, 2, 2, 2, 8},
    {"p256x256k128s2w2x2g8e", 256, 256, 2, 2, 2, 8},
};
constexpr int kNumF8 = (int)(sizeof(kCfgF8) / sizeof(kCfgF8[0]));

template <int BM, int BN, int WM, int WN, int S, bool EVEN = false>
static int launch_f8_pipe(const GemmF8Args& a, int group_m, hipStream_t s) {
    using G = F8Cfg<BM, BN, WM, WN, S>;
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    hipLaunchKernelGGL((gemmf8_pipe<BM, BN, WM, WN, S, EVEN>), dim3(tiles_m * tiles_n), dim3(G::NT), 0, s, a,
                       tiles_m, tiles_n, group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

int num_configs_f8() { return kNumF8; }
const char* config_f8_name(int cfg) { return (cfg >= 0 && cfg < kNumF8) ? kCfgF8[cfg].name : nullptr; }
bool f8_config_needs_bt(int cfg) { return cfg > 0 && cfg < kNumF8; }
bool config_f8_ok(int cfg, int64_t M, int64_t N, int64_t K, int64_t ldc, bool vec_ok) {
    if (cfg < 0 || cfg >= kNumF8) return false;
    if (cfg == 0) return true;
    return vec_ok && K % 128 == 0 && M >= 1 && N >= 1 && buffer_ldc_ok(ldc);
}

// The tiled kernels need K % 128 == 0, 16-byte aligned rows of A and Bt.
int launch_gemm_f8(int cfg, const GemmF8Args& a, bool vec_ok, hipStream_t s) {
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    if (cfg < 0 || cfg >= kNumF8) return MFG_ERR_INVALID_ARG;
    if (cfg == 0) {
        dim3 grid((unsigned)cdiv(a.N, 32), (unsigned)cdiv(a.M, 32), 1);
        hipLaunchKernelGGL(gemmf8_simple, grid, dim3(64), 0, s, a, vec_ok ? 1 : 0);
        MFG_LAUNCH_CHECK();
        return MFG_OK;
    }
    const bool bt_ok = a.Bt != nullptr && ((uintptr_t)a.Bt % 16) == 0 && a.ldbt % 16 == 0;
    if (!vec_ok || !bt_ok || a.K % 128 != 0 || a.M < 1 || a.N < 1 || !buffer_ldc_ok(a.ldc)) return MFG_ERR_UNSUPPORTED;
    const CfgF8& c = kCfgF8[cfg];
    if (cfg == 4) return launch_f8_pipe<256, 256, 2, 2, 2, true>(a, c.group_m, s);
    if (c.bm == 256 && c.bn == 256) return launch_f8_pipe<256, 256, 2, 2, 2>(a, c.group_m, s);
    if (c.bm == 128 && c.bn == 128) return launch_f8_pipe<128, 128, 2, 2, 3>(a, c.group_m, s);
    if (c.bm == 256 && c.bn == 128) return launch_f8_pipe<256, 128, 2, 2, 2>(a, c.group_m, s);
    return MFG_ERR_INTERNAL;
}

}  // namespace mfg
