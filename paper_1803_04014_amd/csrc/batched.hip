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
//     persistent launch.  The work list holds one self-contained record per
//     32x32 output tile of every problem (ordered by decreasing K, the
//     tile's cost); wavefronts take records with a static grid stride and
//     prefetch records and operand blocks across item boundaries.
// Both reuse the tile functions of the single GEMM, so each problem's result
// is bitwise identical to mfg_gemm on that problem alone.
#include <algorithm>
#include <type_traits>

#include "runtime.h"
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

// PAIR (M, N <= 16): two problems share one 32x32x16 MFMA -- problem 2j in
// rows and columns 0..15, problem 2j + 1 in 16..31 (A rows stacked, B
// columns side by side); the diagonal blocks of the product are the two
// results and the off-diagonal blocks are discarded.  Every element is the
// same dot product, in the same order, as the one-problem MFMA.
template <int KIND, bool PAIR>
__global__ __launch_bounds__(256) void gemm16_batched_lds(Gemm16Args p, int64_t count, int vecC) {
    using T = KT<KIND>;
    constexpr int SLAB = 16 * 32;           // halfs per B plane slab
    constexpr int CROW = 33;                // floats per padded C row in LDS
    constexpr int WAVE_LDS = T::NPB * SLAB * 2 + 32 * CROW * 4;  // bytes
    constexpr int PER = PAIR ? 2 : 1;        // problems per wavefront step
    __shared__ __attribute__((aligned(16))) unsigned char lds[4 * WAVE_LDS];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint16_t* slab = reinterpret_cast<uint16_t*>(lds + wid * WAVE_LDS);
    float* ct = reinterpret_cast<float*>(lds + wid * WAVE_LDS + T::NPB * SLAB * 2);
    const int r = lane & 31, g = lane >> 5;
    const int64_t M = p.M, N = p.N, K = p.K;
    const int krow = lane >> 2, c8 = (lane & 3) * 8;  // this lane's piece of a B chunk
    // PAIR: A row r belongs to problem r / 16 (row r % 16), B columns c8 ..
    // c8 + 7 to problem c8 / 16 (columns c8 % 16 ..)
    const int pa = PAIR ? (r >> 4) : 0, ar = PAIR ? (r & 15) : r;
    const int pb = PAIR ? (c8 >> 4) : 0, bc = PAIR ? (c8 & 15) : c8;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t b0 = ((int64_t)blockIdx.x * 4 + wid) * PER; b0 < count; b0 += nwaves * PER) {
        const bool has_a = b0 + pa < count, has_b = b0 + pb < count;
        const uint16_t* Ap[2];
        const uint16_t* Bp[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            Ap[q] = (q < T::NPA) ? p.A[q] + (b0 + pa) * p.sA : nullptr;
            Bp[q] = (q < T::NPB) ? p.B[q] + (b0 + pb) * p.sB : nullptr;
        }
        f32x16 hi = {}, lo = {}, rr = {};
        for (int64_t k0 = 0; k0 < K; k0 += 16) {
            const int64_t kb = k0 + g * 8;
            u32x4 a[2] = {zero4(), zero4()}, bb[2] = {zero4(), zero4()};
#pragma unroll
            for (int q = 0; q < T::NPA; ++q) a[q] = load_row8(Ap[q], has_a && ar < M, ar * p.lda + kb, K - kb, true);
            const int64_t kr = k0 + krow;
#pragma unroll
            for (int q = 0; q < T::NPB; ++q) {
                u32x4 v;
                if (has_b && kr < K && bc + 8 <= N) {
                    v = *reinterpret_cast<const u32x4*>(Bp[q] + kr * p.ldb + bc);
                } else {
                    uint16_t e[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        e[j] = (has_b && kr < K && bc + j < N) ? Bp[q][kr * p.ldb + bc + j] : (uint16_t)0;
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
#pragma unroll
        for (int it = 0; it < (PAIR ? 2 : 4); ++it) {
            // PAIR: pass `it` stores problem b0 + it, rows lane / 4, columns 4 (lane % 4) ..
            const int row = PAIR ? (lane >> 2) : it * 8 + (lane >> 3), c4 = PAIR ? (lane & 3) * 4 : (lane & 7) * 4;
            const int64_t bq = PAIR ? b0 + it : b0;
            if (row >= M || bq >= count) continue;
            const float* src = ct + (PAIR ? (16 * it + row) * CROW + 16 * it + c4 : row * CROW + c4);
            float* dst = p.C + bq * p.sC + row * p.ldc + c4;
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
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    if (a.M > 32 || a.N > 32) return MFG_ERR_INTERNAL;
    const int64_t want = cdiv(count, 4);
    const int64_t cap = (int64_t)num_cu * 16;  // 16 workgroups (64 waves) per CU
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    if (grid == 0) return MFG_OK;
    const int v = vec_ok ? 1 : 0;
    if (vec_ok) {  // 16-byte aligned A and B rows: the LDS-staged kernel
        const int vc = (((uintptr_t)a.C % 16) == 0 && a.ldc % 4 == 0 && a.sC % 4 == 0) ? 1 : 0;
        const bool pair = a.M <= 16 && a.N <= 16;  // two problems per MFMA
        const unsigned g2 = pair ? (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 8), cap)) : grid;
#define MFG_BATCHED_LDS(KIND_)                                                                                     \
    if (pair)                                                                                                       \
        hipLaunchKernelGGL((gemm16_batched_lds<KIND_, true>), dim3(g2), dim3(256), 0, s, a, count, vc);          \
    else                                                                                                            \
        hipLaunchKernelGGL((gemm16_batched_lds<KIND_, false>), dim3(grid), dim3(256), 0, s, a, count, vc);
        switch (kind) {
            case K_F16: MFG_BATCHED_LDS(K_F16) break;
            case K_BF16: MFG_BATCHED_LDS(K_BF16) break;
            case K_REFINE_A: MFG_BATCHED_LDS(K_REFINE_A) break;
            case K_SPLIT3: MFG_BATCHED_LDS(K_SPLIT3) break;
            case K_SPLIT4: MFG_BATCHED_LDS(K_SPLIT4) break;
            case K_BF16_SPLIT3: MFG_BATCHED_LDS(K_BF16_SPLIT3) break;
            default: return MFG_ERR_INVALID_ARG;
        }
#undef MFG_BATCHED_LDS
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
        case K_BF16_SPLIT3:
            hipLaunchKernelGGL(gemm16_batched_small<K_BF16_SPLIT3>, dim3(grid), dim3(256), 0, s, a, count, v);
            break;
        default: return MFG_ERR_INVALID_ARG;
    }
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

// ------------------------------------------------------------------ grouped
// Each workgroup (four wavefronts) takes work items -- one square output
// tile of one problem (F16 / BF16: 128, measured 13% faster than 64 on 4096
// uneven problems, with two workgroups per CU instead of three; the refined
// kinds: 64) --
// with a stride over its XCD's range of the work list; wavefront (wm, wn)
// computes the quarter (wm, wn).  The work
// list is denormalised: each record carries the tile's operand pointers,
// leading dimensions and extent (one 64-byte scalar load).
//
// The items' 64-deep K blocks form one stream per workgroup.  Block s + 2 is
// loaded into registers (16-byte pieces, TT / 32 of A and of B per lane and
// plane: whole 128-byte rows of the A and B tiles) while block s is
// multiplied, and block s + 1 is written into the LDS buffer of its parity
// after it -- across item boundaries, so a short item's loads overlap its
// predecessor's MFMAs and C stores.  One barrier per block.  (A third
// register set, loads three blocks ahead, measured no faster on the
// 4096-problem set: the kernel is bound by the memory system's mixed
// read/write throughput, not by the latency of its loads.)  A rows sit in LDS as 8 XOR-swizzled 16-byte pieces; B
// as 16 x 32 slabs read back transposed.  Every wavefront runs the 32x32x16
// MFMA on 16-deep chunks in K order from zero, with zeros beyond K: the
// operands and order of the simple kernel on that tile.
constexpr int kGroupedBK = 64;  // K per block: 128-byte A and B rows
// Extent of the operand buffer resources and the offset of pieces outside
// an item (at the extent: the load returns zeros).  Piece offsets are below
// TT * kOperandLdLimit * 2 <= 2^30.
constexpr uint32_t kGroupedOob = 0x7FFFFFF0u;
static_assert(128 * kOperandLdLimit * 2 < (int64_t)kGroupedOob, "piece offsets below the out-of-range offset");
// 16 zero bytes in device memory: the load source of lanes with nothing to load
typedef __attribute__((address_space(1))) const uint16_t g_u16;
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;
typedef __attribute__((address_space(1))) const uint32_t g_u32;
typedef __attribute__((address_space(1))) float g_f32;
// Tile classes of the grouped kernel: output tiles of TT x TT (one
// workgroup, four wavefronts of TT/2 x TT/2), TT = 128 or 64, chosen per
// problem (size bucket) when a plan is built.  LDS per workgroup is
// 256 * TT * (planes of A + planes of B) bytes; occupancy (workgroups per CU):
//   TT = 128: F16 / BF16 64 KB, two per CU (<= 256 VGPRs); the refined kinds
//             128 KB, one (latency-bound: measured 2.9x the F16 time for
//             SPLIT3 on mixed sizes, kept as a class for the tuner);
//   TT = 64:  F16 / BF16 32 KB, four per CU (<= 128 VGPRs); REFINE_A 48 KB,
//             three (<= 168 VGPRs); SPLIT3 / SPLIT4 / BF16_SPLIT3 64 KB, two.
template <int KIND, int TT>
constexpr int grouped_wg_per_cu() {
    constexpr int planes = KT<KIND>::NPA + KT<KIND>::NPB;
    if constexpr (TT == 128) return planes == 2 ? 2 : 1;
    return planes == 2 ? 4 : planes == 3 ? 3 : 2;
}
static_assert(kGroupedTile == 128 && kGroupedTileRefined == 64, "default classes: 128 (F16, BF16), 64 (refined)");

// One work record in scalar registers.
struct GItem {
    const g_u16* A;
    const g_u16* B;
    g_f32* C;
    int64_t lda, ldb, ldc;
    int rows, cols, K, vec;
};

// Work records are read with scalar loads (through the constant address
// space: the list is not written while the kernel runs).  They land in
// SGPRs and are counted by lgkmcnt, apart from the operand loads' vmcnt, so
// reading the next record never waits for operand blocks still in flight.
typedef __attribute__((address_space(4))) const GroupedWork c_work;
typedef __attribute__((address_space(4))) const int64_t c_i64;
__device__ __forceinline__ GItem load_item(const c_work* w, int64_t i) {
    const c_work& r = w[i];
    GItem t;
    t.A = (const g_u16*)r.A;
    t.B = (const g_u16*)r.B;
    t.C = (g_f32*)r.C;
    t.lda = r.lda, t.ldb = r.ldb, t.ldc = r.ldc;
    t.rows = r.rows, t.cols = r.cols, t.K = r.K, t.vec = r.vec;
    return t;
}

__device__ __forceinline__ int grouped_blocks(int K) { return max(1, (K + kGroupedBK - 1) / kGroupedBK); }

// Workgroup barrier after this wave's LDS accesses completed (global stores
// and loads stay in flight).
__device__ __forceinline__ void grouped_barrier() {
    lds_wait();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// `planes` (refined kinds only): per work item, the element offsets of the
// residual planes of A and B from their head planes.
template <int KIND, bool VEC, int TT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(grouped_wg_per_cu<KIND, TT>()))) void gemm16_grouped(
    const GroupedWork* work, const int64_t* planes, GroupedSplit split, float alpha, float beta) {
    static_assert(TT == 64 || TT == 128, "tile classes of 64 and 128");
    constexpr int TH = TT / 2;  // workgroup tile, wavefront tile
    constexpr int FM = TH / 32, FN = TH / 32;       // 32 x 32 MFMA blocks per wavefront
    constexpr int PA = TT / 32, PB = TT / 32;       // 16-byte pieces per thread and block: A, B
    constexpr int BPR = TT / 8;                     // pieces per B row
    constexpr int NA = KT<KIND>::NPA, NB = KT<KIND>::NPB;  // operand planes (head, residual)
    constexpr int NR = 2;  // register sets: blocks s + 1 and s + 2 in flight while block s is multiplied
    const int64_t* off = split.off[VEC ? 0 : 1];
    // per plane and buffer: A TT rows x 64, B 4 chunks x TT/32 column slabs x (16 x 32)
    __shared__ __attribute__((aligned(16))) uint16_t As[NA][2][TT * 64];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[NB][2][4][TT / 32][16 * 32];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6), wm = wid >> 1, wn = wid & 1;
    const int xcd = blockIdx.x % kXcds;
    const int64_t stride = gridDim.x / kXcds;
    const int64_t first = off[xcd] + blockIdx.x / kXcds, end = off[xcd + 1];
    if (first >= end) return;
    const int64_t count = (end - first + stride - 1) / stride;  // items of this workgroup
    const c_work* cw = (const c_work*)work;
    auto item_at = [&](int64_t i) { return load_item(cw, first + i * stride); };

    // This thread's pieces of each operand block (piece p = tid + 256 j: A row
    // p / 8, K columns 8 (p % 8) ..; B K row p / BPR, columns 8 (p % BPR) ..).
    // Aligned items (the VEC list: vec records only) load every piece that
    // starts inside the operand as a whole 16-byte piece: with 16-byte
    // aligned rows and ld a multiple of 8 the piece lies in the same aligned
    // 16 bytes as its first element, inside the row's ld extent (and never
    // across a page).  A's elements at or beyond K are then zeroed in
    // registers; B's columns at or beyond the tile's width only reach
    // discarded outputs.  Pieces wholly outside the item (A rows beyond the
    // tile, B rows or A columns at or beyond K, B columns beyond the tile)
    // are zero and cost no memory traffic: every lane issues its buffer load
    // (one resource per plane from the block's first column of A / first
    // row of B), those lanes with an offset past the resource's end, which
    // the hardware answers with zeros.  The loads are thus issued
    // unconditionally, the same number every block, so the compiler's wait
    // before a block's LDS store counts the block loaded after it and lets
    // it stay in flight (with loads behind branches it has to assume none
    // were issued and waits for all).  Offsets stay below 2^31: the VEC list
    // holds only lda, ldb < kOperandLdLimit.
    // Unaligned items load element by element.
    // Residual planes sit at element offsets pa (A) and pb (B) from the head
    // planes of the item being loaded (refined kinds; read with the item).
    int64_t pa = 0, pb = 0;
    auto load_block = [&](const GItem& t, int kb0, u32x4 (&a)[NA][PA], u32x4 (&b)[NB][PB], int (&nv)[PA]) {
        if constexpr (VEC) {
            const uint32_t lda32 = (uint32_t)t.lda, ldb32 = (uint32_t)t.ldb;
            uint32_t oa[PA], ob[PB];
#pragma unroll
            for (int j = 0; j < PA; ++j) {
                const int p = tid + 256 * j, row = p >> 3, ka = kb0 + 8 * (p & 7);
                const bool fa = row < t.rows && ka < t.K;
                oa[j] = fa ? ((uint32_t)row * lda32 + (uint32_t)(8 * (p & 7))) * 2u : kGroupedOob;
                nv[j] = t.K - ka;  // valid elements of the A piece (masked when it is stored)
            }
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int p = tid + 256 * j, kr = p / BPR, cb = 8 * (p % BPR);
                const bool fb = kb0 + kr < t.K && cb < t.cols;
                ob[j] = fb ? ((uint32_t)kr * ldb32 + (uint32_t)cb) * 2u : kGroupedOob;
            }
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                const __amdgpu_buffer_rsrc_t rs =
                    buffer_rsrc((const void*)(t.A + (q ? pa : 0) + kb0), kGroupedOob);
#pragma unroll
                for (int j = 0; j < PA; ++j) a[q][j] = __builtin_amdgcn_raw_buffer_load_b128(rs, oa[j], 0, 0);
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const __amdgpu_buffer_rsrc_t rs =
                    buffer_rsrc((const void*)(t.B + (q ? pb : 0) + (int64_t)kb0 * t.ldb), kGroupedOob);
#pragma unroll
                for (int j = 0; j < PB; ++j) b[q][j] = __builtin_amdgcn_raw_buffer_load_b128(rs, ob[j], 0, 0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < PA; ++j) {
                const int p = tid + 256 * j, row = p >> 3, ka = kb0 + 8 * (p & 7);
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    const g_u16* src = t.A + (q ? pa : 0);
                    uint16_t e[8];
#pragma unroll
                    for (int x = 0; x < 8; ++x)
                        e[x] = (row < t.rows && ka + x < t.K) ? src[row * t.lda + ka + x] : (uint16_t)0;
                    a[q][j] = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
                }
                nv[j] = 8;
            }
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int p = tid + 256 * j, kr = kb0 + p / BPR, cb = 8 * (p % BPR);
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const g_u16* src = t.B + (q ? pb : 0);
                    uint16_t f[8];
#pragma unroll
                    for (int x = 0; x < 8; ++x)
                        f[x] = (kr < t.K && cb + x < t.cols) ? src[kr * t.ldb + cb + x] : (uint16_t)0;
                    b[q][j] = u32x4{pack2(f[0], f[1]), pack2(f[2], f[3]), pack2(f[4], f[5]), pack2(f[6], f[7])};
                }
            }
        }
    };
    auto store_block = [&](int buf, const u32x4 (&a)[NA][PA], const u32x4 (&b)[NB][PB], const int (&nv)[PA]) {
#pragma unroll
        for (int j = 0; j < PA; ++j) {
            const int p = tid + 256 * j, row = p >> 3, c = p & 7;
            uint32_t m[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) m[d] = (2 * d < nv[j] ? 0xFFFFu : 0u) | (2 * d + 1 < nv[j] ? 0xFFFF0000u : 0u);
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                u32x4 am = a[q][j];
#pragma unroll
                for (int d = 0; d < 4; ++d) am[d] &= m[d];
                *reinterpret_cast<u32x4*>(&As[q][buf][row * 64 + ((c ^ swz<8>(row)) * 8)]) = am;
            }
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            // B row kr of the block: chunk kr / 16, slab row kr % 16, column
            // slab c / 4, columns 8 (c % 4) .. +7 of the slab
            const int p = tid + 256 * j, kr = p / BPR, c = p % BPR;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                *reinterpret_cast<u32x4*>(&Bs[q][buf][kr >> 4][c >> 2][(kr & 15) * 32 + 8 * (c & 3)]) = b[q][j];
        }
    };
    auto item_planes = [&](int64_t i) {  // residual-plane offsets of this workgroup's item i
        if constexpr (NA > 1 || NB > 1) {
            const int64_t it = first + i * stride;
            const c_i64* pl = (const c_i64*)planes;
            pa = pl[2 * it], pb = pl[2 * it + 1];
        }
    };

    // cursors: the computed block (item ci, block cb) and the loaded one,
    // NR blocks ahead (item li, block lb); both advance through the stream
    int64_t ci = 0, li = 0;
    int cbk = 0, lbk = 0;
    GItem cur = item_at(0), ld = cur;
    item_planes(0);
    auto advance_load = [&]() {
        if (++lbk >= grouped_blocks(ld.K)) {
            lbk = 0;
            if (++li < count) {
                ld = item_at(li);
                item_planes(li);
            } else {  // past the stream: an empty item (every piece reads zeros)
                ld.rows = ld.cols = ld.K = 0;
                li = count;
            }
        }
    };
    u32x4 ra[NR][NA][PA], rb[NR][NB][PB];  // register sets of the blocks in flight
    int rn[NR][PA];
    // prologue: block 0 into LDS buffer 0, blocks 1 .. NR - 1 into registers
    load_block(ld, 0, ra[0], rb[0], rn[0]);
    store_block(0, ra[0], rb[0], rn[0]);
    advance_load();
#pragma unroll
    for (int r = 1; r < NR; ++r) {
        load_block(ld, lbk * kGroupedBK, ra[r], rb[r], rn[r]);
        advance_load();
    }
    grouped_barrier();

    f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
    auto clear = [&]() {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) hi[i][j] = f32x16{}, lo[i][j] = f32x16{}, rr[i][j] = f32x16{};
    };
    clear();
    // one block s of the stream; BUF: its LDS buffer (s % 2), SET: the
    // register set it arrived in (s % NR).  Returns true after the last
    // item's last block.
    auto step = [&](auto bufc, auto setc) -> bool {
        constexpr int buf = decltype(bufc)::value, set = decltype(setc)::value, nset = (set + 1) % NR;
        // loads of block s + NR into the register set block s used (kept
        // ahead of everything below: the compiler would otherwise sink them)
        load_block(ld, lbk * kGroupedBK, ra[set], rb[set], rn[set]);
        asm volatile("" ::: "memory");  // the IR passes would otherwise sink the buffer loads to their use
        __builtin_amdgcn_sched_barrier(0);
        const int kb0 = cbk * kGroupedBK;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (kb0 + 16 * c >= cur.K) break;
            u32x4 aa[FM][2], bb[FN][2];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int row = wm * TH + fm * 32 + (lane & 31), piece = 2 * c + (lane >> 5);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    aa[fm][q] = q < NA ? *reinterpret_cast<const u32x4*>(
                                             &As[q < NA ? q : 0][buf][row * 64 + ((piece ^ swz<8>(row)) * 8)])
                                       : zero4();
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    bb[fn][q] = q < NB ? slab_read_b(Bs[q < NB ? q : 0][buf][c][wn * FN + fn], lane) : zero4();
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) mma_step<KIND>(aa[fm], bb[fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
        }
        // block s + 1 (loaded during block s + 1 - NR) into the other buffer
        store_block(buf ^ 1, ra[nset], rb[nset], rn[nset]);
        advance_load();
        bool done = false;
        if (cbk + 1 >= grouped_blocks(cur.K)) {  // the item's last block: its C, then the next item
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int r0 = wm * TH + fm * 32;
                if (r0 >= cur.rows || wn * TH >= cur.cols) continue;  // this wavefront's blocks lie outside C
                g_f32* cq = cur.C + (int64_t)r0 * cur.ldc + wn * TH;
                auto val = [&](int fn, int e) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], e); };
                // the VEC list holds only ldc < kBufferLdcLimit: no 64-bit path
                // (whose C reads may stay unconsumed on masked lanes)
                if constexpr (VEC) {
                    store_blocks_buf<FN>(cq, cur.ldc, cur.rows - r0, cur.cols - wn * TH, 0, 0, lane, alpha, beta, val);
                } else {
#pragma unroll
                    for (int fn = 0; fn < FN; ++fn)
                        store_blocks<1>(cq + fn * 32, cur.ldc, cur.rows - r0, cur.cols - wn * TH - fn * 32, 0, 0, lane,
                                        alpha, beta, [&](int, int e) { return val(fn, e); });
                }
            }
            clear();
            cbk = 0;
            if (++ci >= count) {
                done = true;
            } else {
                cur = item_at(ci);
            }
        } else {
            ++cbk;
        }
        if (done) return true;
        grouped_barrier();
        return false;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    for (;;) {
        if (step(I0{}, I0{})) break;
        if (step(I1{}, I1{})) break;
    }
}

// Problems (or, for a problem above 1/16 of the total, bands of its tile
// rows) go to the XCD with the least work so far, largest first (LPT on
// flops); each XCD's items are then ordered by decreasing K, their cost, and
// written out as self-contained records.
void build_grouped_work(const GroupedDesc* descs, int64_t n, std::vector<GroupedWork>& work, GroupedSplit& split,
                        std::vector<int64_t>* planes, int tile) {
    struct Unit {
        int64_t prob, tm0, tm1;
        double flops;
    };
    struct Tile {
        int32_t prob, tm, tn;
    };
    work.clear();
    if (planes) planes->clear();
    for (int list = 0; list < 2; ++list) {  // 0: aligned problems, ldc and operand ld within the 32-bit offset bounds; 1: the rest
        auto in_list = [&](const GroupedDesc& d) {
            return (d.vec != 0 && buffer_ldc_ok(d.ldc) && operand_ld_ok(d.lda, d.ldb)) == (list == 0);
        };
        double total = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (in_list(descs[i])) total += 2.0 * (double)descs[i].M * (double)descs[i].N * (double)descs[i].K;
        const double cap = total / (2.0 * kXcds);
        std::vector<Unit> units;
        for (int64_t i = 0; i < n; ++i) {
            const GroupedDesc& d = descs[i];
            const int64_t tm = cdiv(d.M, tile), tn = cdiv(d.N, tile);
            if (!in_list(d) || tm == 0 || tn == 0) continue;
            const double f = 2.0 * (double)d.M * (double)d.N * (double)d.K;
            const int64_t parts = std::min<int64_t>(tm, cap > 0.0 ? std::max<int64_t>(1, (int64_t)(f / cap)) : 1);
            for (int64_t q = 0; q < parts; ++q) {
                const int64_t a = tm * q / parts, b = tm * (q + 1) / parts;
                units.push_back(Unit{i, a, b, f * (double)(b - a) / (double)tm});
            }
        }
        std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.flops > y.flops; });
        std::vector<double> load(kXcds, 0.0);
        std::vector<std::vector<Tile>> per(kXcds);
        for (const Unit& u : units) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[x] += u.flops;
            const int64_t tn = cdiv(descs[u.prob].N, tile);
            for (int64_t a = u.tm0; a < u.tm1; ++a)
                for (int64_t b = 0; b < tn; ++b) per[x].push_back(Tile{(int32_t)u.prob, (int32_t)a, (int32_t)b});
        }
        split.off[list][0] = (int64_t)work.size();
        for (int x = 0; x < kXcds; ++x) {
            std::stable_sort(per[x].begin(), per[x].end(),
                             [&](const Tile& p, const Tile& q) { return descs[p.prob].K > descs[q.prob].K; });
            for (const Tile& t : per[x]) {
                const GroupedDesc& d = descs[t.prob];
                const int64_t m0 = (int64_t)t.tm * tile, n0 = (int64_t)t.tn * tile;
                GroupedWork w;
                w.A = d.A + m0 * d.lda;
                w.B = d.B + n0;
                w.C = d.C + m0 * d.ldc + n0;
                w.lda = d.lda, w.ldb = d.ldb, w.ldc = d.ldc;
                w.rows = (int32_t)std::min<int64_t>(tile, d.M - m0);
                w.cols = (int32_t)std::min<int64_t>(tile, d.N - n0);
                w.K = (int32_t)d.K, w.vec = d.vec;
                work.push_back(w);
                if (planes) planes->push_back(d.pa), planes->push_back(d.pb);
            }
            split.off[list][x + 1] = (int64_t)work.size();
        }
    }
}

template <int TT>
static int wg_per_cu_tt(int kind) {
    switch (kind) {
        case K_REFINE_A: return grouped_wg_per_cu<K_REFINE_A, TT>();
        case K_SPLIT3: return grouped_wg_per_cu<K_SPLIT3, TT>();
        case K_SPLIT4: return grouped_wg_per_cu<K_SPLIT4, TT>();
        case K_BF16_SPLIT3: return grouped_wg_per_cu<K_BF16_SPLIT3, TT>();
        case K_BF16: return grouped_wg_per_cu<K_BF16, TT>();
        default: return grouped_wg_per_cu<K_F16, TT>();
    }
}

int grouped_grid(const GroupedSplit& split, int list, int kind, int tile) {
    int64_t most = 0;  // the largest per-XCD range sets how many workgroups each XCD needs
    for (int x = 0; x < kXcds; ++x) most = std::max<int64_t>(most, split.off[list][x + 1] - split.off[list][x]);
    const int per_cu = tile == 128 ? wg_per_cu_tt<128>(kind) : wg_per_cu_tt<64>(kind);
    const int64_t per_xcd = std::max<int64_t>(1, std::min<int64_t>(most, (int64_t)device_cu_count() / kXcds * per_cu));
    return (int)(per_xcd * kXcds);
}

template <int KIND, int TT>
static void launch_grouped_kind(int list, dim3 grid, const GroupedWork* work, const int64_t* planes,
                                const GroupedSplit& split, float alpha, float beta, hipStream_t s) {
    if (list == 0)
        hipLaunchKernelGGL((gemm16_grouped<KIND, true, TT>), grid, dim3(256), 0, s, work, planes, split, alpha, beta);
    else
        hipLaunchKernelGGL((gemm16_grouped<KIND, false, TT>), grid, dim3(256), 0, s, work, planes, split, alpha, beta);
}

template <int TT>
static void launch_grouped_tt(int kind, int list, dim3 grid, const GroupedWork* work, const int64_t* planes,
                              const GroupedSplit& split, float alpha, float beta, hipStream_t s) {
    switch (kind) {
        case K_F16: launch_grouped_kind<K_F16, TT>(list, grid, work, planes, split, alpha, beta, s); break;
        case K_BF16: launch_grouped_kind<K_BF16, TT>(list, grid, work, planes, split, alpha, beta, s); break;
        case K_REFINE_A: launch_grouped_kind<K_REFINE_A, TT>(list, grid, work, planes, split, alpha, beta, s); break;
        case K_SPLIT3: launch_grouped_kind<K_SPLIT3, TT>(list, grid, work, planes, split, alpha, beta, s); break;
        case K_BF16_SPLIT3: launch_grouped_kind<K_BF16_SPLIT3, TT>(list, grid, work, planes, split, alpha, beta, s); break;
        default:
            if constexpr (TT == 64) launch_grouped_kind<K_SPLIT4, TT>(list, grid, work, planes, split, alpha, beta, s);
            break;
    }
}

// SPLIT4 at 128 (three accumulator blocks of 64 x 64 per wavefront) spills:
// it has the 64 class only.
bool grouped_tile_ok(int kind, int tile) { return tile == 64 || (tile == 128 && kind != K_SPLIT4); }

int grouped_tiles(int kind, int* tiles) {
    tiles[0] = grouped_tile(kind);
    if (kind == K_SPLIT4) return 1;
    tiles[1] = tiles[0] == 128 ? 64 : 128;
    return 2;
}

int grouped_launch(int kind, int tile, const GroupedWork* work, const int64_t* planes, const GroupedSplit& split,
                   float alpha, float beta, hipStream_t s) {
    if (kind < K_F16 || kind > K_BF16_SPLIT3 || !grouped_tile_ok(kind, tile)) return MFG_ERR_UNSUPPORTED;
    if (kind >= K_REFINE_A && !planes) return MFG_ERR_INTERNAL;  // the refined kinds read residual planes
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    for (int list = 0; list < 2; ++list) {
        if (split.off[list][kXcds] == split.off[list][0]) continue;  // empty list
        const dim3 grid((unsigned)grouped_grid(split, list, kind, tile));
        if (tile == 128)
            launch_grouped_tt<128>(kind, list, grid, work, planes, split, alpha, beta, s);
        else
            launch_grouped_tt<64>(kind, list, grid, work, planes, split, alpha, beta, s);
        MFG_LAUNCH_CHECK();
    }
    return MFG_OK;
}

}  // namespace mfg
