// MFMA contraction of the TensCol step on gfx950:
//   G = A . S_cat  (+ P . S_cat when the penalty is active),
// with S_cat = [S_1 ... S_D] (n x D*k, stored transposed as S^T [D*k][n_pad])
// and P the penalty operand built by the group-concentration kernel.
//
// A and S are 0/1, so A.S is exact in fp32, bf16, fp8 and fp4 operands with FP32
// accumulation; between the two passes each block gathers (A.S_d)[i, c_d(i)]
// into 2 f_color(S_d) (the gradient's first term is the TabuCol gamma matrix,
// whose entry at the vertex's own colour counts its conflicts).
//
// Layout: 4 waves as 2 (rows) x 2 (columns), or 8 as 4 x 2 for 256-row tiles; block
// tile BM x BN with BN = 32 * NTW; each wave owns (BM/WM) x (16 NTW) as 16x16 MFMA
// subtiles.
// Both operands are K-contiguous; a K-stage moves 128 bytes of every operand
// row straight from global memory into LDS (global_load_lds, 16 bytes per
// lane, no registers on the way) through two or three stage buffers, and the
// fragments of the next stage are read while the MFMAs of the current one run
// (see gemm_sweep).  Within a 128-byte LDS row the
// 16-byte chunk c of row r sits in slot c ^ ((r / 2) mod 8): a fragment read
// covers 16 consecutive rows at one chunk, and with 64 four-byte banks the bank
// of (row, slot) depends on (row mod 2, slot), so those 16 reads land in 16
// different bank groups.
//
// Mode 0 stores G as [D][n][k] fp32 for the separate update kernel.
// Mode 1 (fused): column tiles hold whole members; the accumulators go through
// LDS and each (member, vertex) row gets softmax, straight-through gradient,
// update, smoothing and the next iteration's argmax in the same kernel.
#include "tcol_internal.h"
#include "tcol_launch.h"

#include <math.h>

namespace tcol {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// one MFMA step on a 16x16 output subtile for each operand format
__device__ inline f32x4 mfma_fp8(const i32x8& a, const i32x8& b, const f32x4& c) {
    // operand formats 0/0 = fp8 e4m3; zero scale arguments select the unscaled instruction
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}
__device__ inline f32x4 mfma_fp4(const i32x8& a, const i32x8& b, const f32x4& c) {
    // operand formats 4/4 = fp4 e2m1 (the low four registers of each operand)
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 4, 4, 0, 0, 0, 0);
}
__device__ inline f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_f32(float a, float b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 16-row MFMA subtiles per wave of a BM-row tile (4 waves of BM/2 rows, or 8 of 64 rows at BM = 256)
constexpr int tile_mt(int bm) { return bm == 256 ? 4 : bm / 32; }
constexpr int tile_threads(int bm) { return bm == 256 ? 512 : 256; }

template <int BM, int NTW>
struct Tile {
    static constexpr int BN = 32 * NTW;
    // 256-row tiles run 8 waves (4 x 2, 64 x 64 each, two per SIMD); the others 4 (2 x 2)
    static constexpr int WAVES = BM == 256 ? 8 : 4;
    static constexpr int THREADS = 64 * WAVES;
    static_assert(THREADS == tile_threads(BM), "threads per block");
    static constexpr int WM = WAVES / 2;                     // waves along the rows
    static constexpr int RW = BM / WM;                       // rows per wave
    static constexpr int MT = RW / 16;                       // 16-row subtiles per wave
    static_assert(MT == tile_mt(BM), "subtiles per wave");
    static constexpr int STAGE = (BM + BN) * kStageRowBytes; // bytes per LDS stage
    static constexpr int GROUPS = (BM + BN) / (8 * WAVES);   // 8-row load groups per wave per stage
    static_assert((BM + BN) % (8 * WAVES) == 0, "load split");
    // LDS stage buffers: three, unless only two keep a 4-wave block within 80 KB (two
    // blocks, i.e. two waves per SIMD, per CU); an 8-wave block takes two
    static constexpr int NB = WAVES == 8 ? 2
                              : ((3 * STAGE <= 80 * 1024) ? 3 : ((2 * STAGE <= 80 * 1024) ? 2 : 3));
    // compiled for two waves per SIMD (at most 256 registers per lane)
    static constexpr bool TWO_PER_SIMD = WAVES == 8 || 2 * NB * STAGE <= 160 * 1024;
    // after the K-sweep the stage buffers hold the gather: the colours of the tile's
    // rows for its members, then the per-member conflict counters
    static constexpr int CT_BYTES = ((BN + 2) * BM * 2 + 15) / 16 * 16;
    static_assert(CT_BYTES + 4 * (BN + 2) <= NB * STAGE, "gather fits the stage buffers");
};

// Fragments of one LDS stage for one wave (chunk c of row r sits at slot c ^ ((r >> 1) & 7)).
// A stage is one K-step of the 16x16x128 fp8 MFMA (32 bytes per lane: chunks 2q and
// 2q+1) or two K-steps of 16 bytes per lane (chunk 4 ks + q) for fp4 (16x16x128),
// bf16 (16x16x32) and fp32 (four 16x16x4); A and B use the same chunks, so every
// format sums the plain product.
template <int PREC, int BM, int NTW>
struct StageFrags {
    static constexpr int MT = Tile<BM, NTW>::MT;
    static constexpr int SUB = PREC == kPrecFP8 ? 1 : 2;   // K-steps per stage
    static constexpr int W = PREC == kPrecFP8 ? 2 : 1;     // 16-byte chunks per fragment
    uint4 a[SUB][MT][W], b[SUB][NTW][W];
};

template <int PREC, int BM, int NTW>
__device__ __forceinline__ void stage_read(StageFrags<PREC, BM, NTW>& F, const uint8_t* L, int lane, int wm, int wn) {
    using Fr = StageFrags<PREC, BM, NTW>;
    const int ra = wm * Tile<BM, NTW>::RW + (lane & 15);
    const int rb = BM + wn * (NTW * 16) + (lane & 15);
    const int q = lane >> 4;
    const int swz = (lane & 15) >> 1;  // = (row >> 1) & 7 for every row this lane reads
#pragma unroll
    for (int ks = 0; ks < Fr::SUB; ++ks) {
#pragma unroll
        for (int w = 0; w < Fr::W; ++w) {
            const int o = ((Fr::W == 2 ? 2 * q + w : ks * 4 + q) ^ swz) * 16;
#pragma unroll
            for (int mt = 0; mt < Fr::MT; ++mt) F.a[ks][mt][w] = *(const uint4*)(L + (ra + mt * 16) * kStageRowBytes + o);
        }
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
            for (int w = 0; w < Fr::W; ++w) {
                const int o = ((Fr::W == 2 ? 2 * q + w : ks * 4 + q) ^ swz) * 16;
                F.b[ks][nt][w] = *(const uint4*)(L + (rb + nt * 16) * kStageRowBytes + o);
            }
    }
}

// One K-step (16-byte chunk ks*4 + q of every row) of a two-K-step stage, for the
// staggered sweep below: the same chunks as stage_read's K-step ks.
template <int PREC, int BM, int NTW>
struct KStepFrags {
    uint4 a[Tile<BM, NTW>::MT], b[NTW];
};

template <int PREC, int BM, int NTW>
__device__ __forceinline__ void kstep_read(KStepFrags<PREC, BM, NTW>& F, const uint8_t* L, int ks, int lane, int wm,
                                           int wn) {
    const int ra = wm * Tile<BM, NTW>::RW + (lane & 15);
    const int rb = BM + wn * (NTW * 16) + (lane & 15);
    const int o = ((ks * 4 + (lane >> 4)) ^ ((lane & 15) >> 1)) * 16;
#pragma unroll
    for (int mt = 0; mt < Tile<BM, NTW>::MT; ++mt) F.a[mt] = *(const uint4*)(L + (ra + mt * 16) * kStageRowBytes + o);
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) F.b[nt] = *(const uint4*)(L + (rb + nt * 16) * kStageRowBytes + o);
}

template <int PREC, int BM, int NTW>
__device__ __forceinline__ void kstep_mma(f32x4 (&acc)[tile_mt(BM)][NTW], const KStepFrags<PREC, BM, NTW>& F) {
    static_assert(PREC == kPrecFP4 || PREC == kPrecBF16, "fp4 and bf16 stages hold two K-steps");
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
        for (int mt = 0; mt < Tile<BM, NTW>::MT; ++mt) {
            const uint4 a0 = F.a[mt], b0 = F.b[nt];
            if constexpr (PREC == kPrecFP4) {
                const i32x8 a{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, 0, 0, 0, 0};
                const i32x8 b{(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, 0, 0, 0, 0};
                acc[mt][nt] = mfma_fp4(a, b, acc[mt][nt]);
            } else {
                acc[mt][nt] = mfma_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0), acc[mt][nt]);
            }
        }
}

template <int PREC, int BM, int NTW>
__device__ __forceinline__ void stage_mma(f32x4 (&acc)[tile_mt(BM)][NTW], const StageFrags<PREC, BM, NTW>& F) {
    using Fr = StageFrags<PREC, BM, NTW>;
#pragma unroll
    for (int ks = 0; ks < Fr::SUB; ++ks)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
            for (int mt = 0; mt < Fr::MT; ++mt) {
                const uint4 a0 = F.a[ks][mt][0], b0 = F.b[ks][nt][0];
                if constexpr (PREC == kPrecFP8) {
                    const uint4 a1 = F.a[ks][mt][Fr::W - 1], b1 = F.b[ks][nt][Fr::W - 1];
                    const i32x8 a{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
                    const i32x8 b{(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
                    acc[mt][nt] = mfma_fp8(a, b, acc[mt][nt]);
                } else if constexpr (PREC == kPrecFP4) {
                    const i32x8 a{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, 0, 0, 0, 0};
                    const i32x8 b{(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, 0, 0, 0, 0};
                    acc[mt][nt] = mfma_fp4(a, b, acc[mt][nt]);
                } else if constexpr (PREC == kPrecBF16) {
                    acc[mt][nt] = mfma_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0), acc[mt][nt]);
                } else {
                    const float4 a = __builtin_bit_cast(float4, a0), b = __builtin_bit_cast(float4, b0);
                    acc[mt][nt] = mfma_f32(a.x, b.x, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a.y, b.y, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a.z, b.z, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a.w, b.w, acc[mt][nt]);
                }
            }
}

typedef const __attribute__((address_space(1))) void* gbl_ptr;
typedef __attribute__((address_space(3))) void* lds_ptr;

// Issue the direct-to-LDS loads of one K-stage.  Wave w moves the 8-row groups
// w, w+4, ...; lane L of a group writes LDS bytes [16L, 16L+16) of the group, i.e.
// row L/8, slot L%8, which receives global chunk (L%8) ^ ((row >> 1) & 7).
template <int BM, int NTW>
__device__ __forceinline__ void stage_load(const uint8_t* __restrict__ Arow, const uint8_t* __restrict__ Brow,
                                           size_t ld, int s, uint8_t* buf, int lane, int wave) {
    using T = Tile<BM, NTW>;
    const int rsub = lane >> 3, slot = lane & 7;
#pragma unroll
    for (int gi = 0; gi < T::GROUPS; ++gi) {
        const int grp = wave + T::WAVES * gi;
        const int r = grp * 8 + rsub;
        const int c = slot ^ ((r >> 1) & 7);
        const uint8_t* src = (r < BM ? Arow + (size_t)r * ld : Brow + (size_t)(r - BM) * ld) +
                             (size_t)s * kStageRowBytes + c * 16;
        __builtin_amdgcn_global_load_lds((gbl_ptr)src, (lds_ptr)(buf + grp * 8 * kStageRowBytes), 16, 0, 0);
    }
}

// s_waitcnt vmcnt(N) (N <= 63) with expcnt / lgkmcnt left alone: at most N of this
// wave's vector memory operations, including the ones that write LDS, are in flight
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}


// Workgroup barrier without the memory fence of __syncthreads(): that fence would
// make every wave drain all its loads, including the prefetches of later stages.
// Visibility of the LDS stages is ordered explicitly by wait_vm before it.  The
// barrier itself waits for this wave's LDS reads (lgkmcnt 0): the compiler may
// issue the fragment reads of a stage before the barrier and consume them after
// it, and once every wave has passed, the next stage's direct-to-LDS loads may
// overwrite that buffer.
__device__ __forceinline__ void stage_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));   // lgkmcnt(0), others untouched
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One K-sweep: acc += Arows[m0.., :] . Brows[n0.., :]^T over `nstages` stages
// of 128 bytes.  Arow / Brow point at the first row of the tile; ld in bytes.
// Two pipelines: global -> LDS runs NB stages ahead through the NB stage buffers,
// and LDS -> registers one stage ahead through two fragment sets, so the fragment
// reads of stage s+1 proceed while the MFMAs of stage s run.  At the top of
// iteration s every wave has finished reading stage s, so its buffer takes the
// loads of stage s+NB.  Large tiles, whose two fragment sets would spill, keep one:
// in fp4 and bf16 (two K-steps per stage) they put the barrier between the K-steps.
template <int PREC, int BM, int NTW>
__device__ __forceinline__ void gemm_sweep(f32x4 (&acc)[tile_mt(BM)][NTW], const uint8_t* __restrict__ Arow,
                                           const uint8_t* __restrict__ Brow, size_t ld, int nstages,
                                           uint8_t* lds) {
    using T = Tile<BM, NTW>;
    using Fr = StageFrags<PREC, BM, NTW>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    if constexpr (Fr::SUB * (Fr::MT + NTW) * Fr::W * 4 > 64 && Fr::SUB == 2 && PREC != kPrecFP32) {
        // fp4 and bf16 tiles whose stage fragments would not fit twice in registers (two
        // K-steps per stage): the barrier falls between the K-steps.  The second K-step's fragments
        // are read before it and its MFMAs run after it, while the next stage's first
        // K-step is read; the buffer freed at the barrier takes the loads of stage s+NB
        // at once, so a load has a whole stage of MFMAs to land.  Two K-step sets hold
        // as many registers as one stage set.
        constexpr int NB = T::NB;
        using KF = KStepFrags<PREC, BM, NTW>;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            stage_load<BM, NTW>(Arow, Brow, ld, min(b, nstages - 1), lds + b * T::STAGE, lane, wave);
        wait_vm<(NB - 1) * T::GROUPS>();   // stage 0 has landed
        stage_barrier();
        KF Fa, Fb;
        kstep_read<PREC, BM, NTW>(Fa, lds, 0, lane, wm, wn);
        int cur = 0;
        for (int s = 0; s < nstages; ++s) {
            kstep_read<PREC, BM, NTW>(Fb, lds + cur * T::STAGE, 1, lane, wm, wn);
            __builtin_amdgcn_sched_barrier(0);
            kstep_mma<PREC, BM, NTW>(acc, Fa);
            wait_vm<(NB - 2) * T::GROUPS>();   // stage s+1 has landed (later ones may be in flight)
            stage_barrier();                   // ... for every wave, and no wave reads stage s any more
            // past the end, the last stage again into the freed buffer; nobody reads it
            stage_load<BM, NTW>(Arow, Brow, ld, min(s + NB, nstages - 1), lds + cur * T::STAGE, lane, wave);
            cur = cur == NB - 1 ? 0 : cur + 1;
            if (s + 1 < nstages) kstep_read<PREC, BM, NTW>(Fa, lds + cur * T::STAGE, 0, lane, wm, wn);
            __builtin_amdgcn_sched_barrier(0);
            kstep_mma<PREC, BM, NTW>(acc, Fb);
        }
        return;
    } else if constexpr (Fr::SUB * (Fr::MT + NTW) * Fr::W * 4 > 64) {
        // fp8 and fp32 tiles whose fragments would not fit twice in registers: one
        // fragment set, the global -> LDS loads NB - 1 stages ahead (fp32, whose K-step is
        // four MFMAs, ran 8 % slower at C5 in the staggered form)
        constexpr int NB = T::NB;
#pragma unroll
        for (int b = 0; b < NB - 1; ++b)
            stage_load<BM, NTW>(Arow, Brow, ld, min(b, nstages - 1), lds + b * T::STAGE, lane, wave);
        wait_vm<(NB - 2) * T::GROUPS>();   // stage 0 has landed
        stage_barrier();
        int cur = 0;
        for (int s = 0; s < nstages; ++s) {
            const int nxt = cur == 0 ? NB - 1 : cur - 1;   // (s + NB - 1) mod NB
            stage_load<BM, NTW>(Arow, Brow, ld, min(s + NB - 1, nstages - 1), lds + nxt * T::STAGE, lane, wave);
            Fr F;
            stage_read<PREC, BM, NTW>(F, lds + cur * T::STAGE, lane, wm, wn);
            __builtin_amdgcn_sched_barrier(0);
            stage_mma<PREC, BM, NTW>(acc, F);
            wait_vm<(NB - 2) * T::GROUPS>();  // stage s+1 has landed
            stage_barrier();
            cur = cur == NB - 1 ? 0 : cur + 1;
        }
        return;
    }
    // stages past the end reload the last one into a free buffer; nobody reads it
    constexpr int NB = T::NB;
#pragma unroll
    for (int b = 0; b < NB; ++b) stage_load<BM, NTW>(Arow, Brow, ld, min(b, nstages - 1), lds + b * T::STAGE, lane, wave);
    wait_vm<(NB - 1) * T::GROUPS>();   // stage 0 has landed
    stage_barrier();
    Fr F0, F1;
    stage_read<PREC, BM, NTW>(F0, lds, lane, wm, wn);
    int cur = 0;                   // buffer of stage s
    for (int s = 0; s < nstages; s += 2) {
        // ---- stage s (fragments in F0)
        wait_vm<(NB - 2) * T::GROUPS>();   // stage s+1 has landed (later ones may be in flight)
        stage_barrier();           // ... for every wave, and every wave has stage s in registers
        stage_load<BM, NTW>(Arow, Brow, ld, min(s + NB, nstages - 1), lds + cur * T::STAGE, lane, wave);
        cur = cur == NB - 1 ? 0 : cur + 1;
        if (s + 1 < nstages) stage_read<PREC, BM, NTW>(F1, lds + cur * T::STAGE, lane, wm, wn);
        __builtin_amdgcn_sched_barrier(0);
        stage_mma<PREC, BM, NTW>(acc, F0);
        if (s + 1 >= nstages) break;
        // ---- stage s+1 (fragments in F1)
        wait_vm<(NB - 2) * T::GROUPS>();
        stage_barrier();
        stage_load<BM, NTW>(Arow, Brow, ld, min(s + 1 + NB, nstages - 1), lds + cur * T::STAGE, lane, wave);
        cur = cur == NB - 1 ? 0 : cur + 1;
        if (s + 2 < nstages) stage_read<PREC, BM, NTW>(F0, lds + cur * T::STAGE, lane, wm, wn);
        __builtin_amdgcn_sched_barrier(0);
        stage_mma<PREC, BM, NTW>(acc, F1);
    }
}

// ---- penalty pass of the fp4 mode: P (bf16) against S^T straight from the fp4 operand ----
//
// A K-stage covers 64 K-values: 128 bytes of each P row (as in the sweep above) and 32
// bytes of each S^T row in fp4, whose 0/1 nibbles (1.0 = 0x2) become bf16 in registers
// when the MFMAs need them.  They become 2.0 rather than 1.0: bf16 2.0 is 0x4000, a
// single byte, so one shift-and-mask and one byte permute make each pair; the operand
// P of an fp4 graph is stored halved (exact in bf16), so the products are unchanged.  This avoids a bf16 copy of S and quarters the S bytes
// staged and read from LDS, so three stage buffers fit where the fp4 A.S sweep keeps
// two.  The S rows move with 4-byte direct-to-LDS loads (a load writes 4 bytes per lane,
// 256 per wave: 8 rows of 32 bytes); word w of row r sits at slot w ^ (((r >> 3) & 1) << 2),
// so a fragment read (16 consecutive rows, one word each) touches 16 different banks
// pairs.
template <int BM, int NTW>
struct PenTile {
    using T = Tile<BM, NTW>;
    static constexpr int BN = T::BN;
    static constexpr int BROW = 32;                              // fp4 bytes of S per row per stage
    static constexpr int A_BYTES = BM * kStageRowBytes;
    static constexpr int STAGE = A_BYTES + BN * BROW;
    static constexpr int AG = BM / (8 * T::WAVES);               // 16-byte-lane loads of P per wave per stage
    static constexpr int BG = BN * BROW / (256 * T::WAVES);      // 4-byte-lane loads of S per wave per stage
    static_assert(BM % (8 * T::WAVES) == 0 && (BN * BROW) % (256 * T::WAVES) == 0, "penalty load split");
    static constexpr int NB = 3 * STAGE <= T::NB * T::STAGE ? 3 : 2;   // within the block's stage buffers
    static_assert(NB * STAGE <= T::NB * T::STAGE, "penalty stages fit");
};

template <int BM, int NTW>
struct PenFrags {
    uint4 a[2][tile_mt(BM)];     // P: 16 bytes (8 bf16) per lane per K-step
    uint32_t b[2][NTW];          // S: 4 bytes (8 fp4) per lane per K-step
};

// eight fp4 nibbles equal to 0 or 0x2 (0.0 or 1.0), the lowest first, as eight bf16
// equal to 0.0 or 2.0: even nibbles' flag bit moved to bit 6 of their byte (0x40, the
// high byte of bf16 2.0), odd nibbles' likewise, then each output word takes
// [0, even byte j, 0, odd byte j]
__device__ __forceinline__ bf16x8 fp4_01_to_bf16x2(uint32_t x) {
    const uint32_t e = (x << 5) & 0x40404040u;    // nibbles 0, 2, 4, 6
    const uint32_t o = (x << 1) & 0x40404040u;    // nibbles 1, 3, 5, 7
    // v_perm_b32 byte selectors: 0-3 pick bytes of the second source, 4-7 of the first,
    // 0x0C gives 0x00
    uint4 r;
    r.x = __builtin_amdgcn_perm(o, e, 0x040C000Cu);
    r.y = __builtin_amdgcn_perm(o, e, 0x050C010Cu);
    r.z = __builtin_amdgcn_perm(o, e, 0x060C020Cu);
    r.w = __builtin_amdgcn_perm(o, e, 0x070C030Cu);
    return __builtin_bit_cast(bf16x8, r);
}

template <int BM, int NTW>
__device__ __forceinline__ void pen_read(PenFrags<BM, NTW>& F, const uint8_t* L, int lane, int wm, int wn) {
    using T = Tile<BM, NTW>;
    using P = PenTile<BM, NTW>;
    const int ra = wm * T::RW + (lane & 15);
    const int rb = wn * (NTW * 16) + (lane & 15);
    const int q = lane >> 4;
    const int swz = (lane & 15) >> 1;                 // P rows: (row >> 1) & 7
    const int swb = ((lane & 15) >> 3) << 2;          // S rows: ((row >> 3) & 1) << 2
    const uint8_t* LB = L + P::A_BYTES;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int o = ((ks * 4 + q) ^ swz) * 16;
#pragma unroll
        for (int mt = 0; mt < T::MT; ++mt) F.a[ks][mt] = *(const uint4*)(L + (ra + mt * 16) * kStageRowBytes + o);
        const int ob = ((ks * 4 + q) ^ swb) * 4;
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) F.b[ks][nt] = *(const uint32_t*)(LB + (rb + nt * 16) * P::BROW + ob);
    }
}

template <int BM, int NTW>
__device__ __forceinline__ void pen_mma(f32x4 (&acc)[tile_mt(BM)][NTW], const PenFrags<BM, NTW>& F) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
            const bf16x8 b = fp4_01_to_bf16x2(F.b[ks][nt]);
#pragma unroll
            for (int mt = 0; mt < tile_mt(BM); ++mt)
                acc[mt][nt] = mfma_bf16(__builtin_bit_cast(bf16x8, F.a[ks][mt]), b, acc[mt][nt]);
        }
}

// P rows: as stage_load (8-row groups of 128 bytes, 16 bytes per lane); S rows: 8-row
// groups of 32 bytes, 4 bytes per lane (lane L: row L / 8, slot L % 8, which receives
// global word (L % 8) ^ (((row >> 3) & 1) << 2))
template <int BM, int NTW>
__device__ __forceinline__ void pen_load(const uint8_t* __restrict__ Prow, const uint8_t* __restrict__ Srow,
                                         size_t ldp, size_t lds_, int s, uint8_t* buf, int lane, int wave) {
    using T = Tile<BM, NTW>;
    using P = PenTile<BM, NTW>;
    {
        const int rsub = lane >> 3, slot = lane & 7;
#pragma unroll
        for (int gi = 0; gi < P::AG; ++gi) {
            const int grp = wave + T::WAVES * gi;
            const int r = grp * 8 + rsub;
            const int c = slot ^ ((r >> 1) & 7);
            const uint8_t* src = Prow + (size_t)r * ldp + (size_t)s * kStageRowBytes + c * 16;
            __builtin_amdgcn_global_load_lds((gbl_ptr)src, (lds_ptr)(buf + grp * 8 * kStageRowBytes), 16, 0, 0);
        }
    }
    {
        uint8_t* bb = buf + P::A_BYTES;
        const int rsub = lane >> 3, slot = lane & 7;
#pragma unroll
        for (int gi = 0; gi < P::BG; ++gi) {
            const int grp = wave + T::WAVES * gi;
            const int r = grp * 8 + rsub;
            const int w = slot ^ (((r >> 3) & 1) << 2);
            const uint8_t* src = Srow + (size_t)r * lds_ + (size_t)s * P::BROW + w * 4;
            __builtin_amdgcn_global_load_lds((gbl_ptr)src, (lds_ptr)(bb + grp * 8 * P::BROW), 4, 0, 0);
        }
    }
}

// acc += Prows . (S^T rows)^T over `nstages` stages of 64 K-values; the same two
// pipelines as gemm_sweep's pipelined form (loads NB stages ahead, fragments one ahead).
template <int BM, int NTW>
__device__ __forceinline__ void pen_sweep(f32x4 (&acc)[tile_mt(BM)][NTW], const uint8_t* __restrict__ Prow,
                                          const uint8_t* __restrict__ Srow, size_t ldp, size_t lds_, int nstages,
                                          uint8_t* lds) {
    using P = PenTile<BM, NTW>;
    constexpr int NB = P::NB, PER = P::AG + P::BG;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int b = 0; b < NB; ++b) pen_load<BM, NTW>(Prow, Srow, ldp, lds_, min(b, nstages - 1), lds + b * P::STAGE, lane, wave);
    wait_vm<(NB - 1) * PER>();   // stage 0 has landed
    stage_barrier();
    PenFrags<BM, NTW> F0, F1;
    pen_read<BM, NTW>(F0, lds, lane, wm, wn);
    int cur = 0;
    for (int s = 0; s < nstages; s += 2) {
        wait_vm<(NB - 2) * PER>();   // stage s+1 has landed
        stage_barrier();
        pen_load<BM, NTW>(Prow, Srow, ldp, lds_, min(s + NB, nstages - 1), lds + cur * P::STAGE, lane, wave);
        cur = cur == NB - 1 ? 0 : cur + 1;
        if (s + 1 < nstages) pen_read<BM, NTW>(F1, lds + cur * P::STAGE, lane, wm, wn);
        __builtin_amdgcn_sched_barrier(0);
        pen_mma<BM, NTW>(acc, F0);
        if (s + 1 >= nstages) break;
        wait_vm<(NB - 2) * PER>();
        stage_barrier();
        pen_load<BM, NTW>(Prow, Srow, ldp, lds_, min(s + 1 + NB, nstages - 1), lds + cur * P::STAGE, lane, wave);
        cur = cur == NB - 1 ? 0 : cur + 1;
        if (s + 2 < nstages) pen_read<BM, NTW>(F0, lds + cur * P::STAGE, lane, wm, wn);
        __builtin_amdgcn_sched_barrier(0);
        pen_mma<BM, NTW>(acc, F1);
    }
}

// XCD-aware order: hardware deals block b to XCD b mod 8, so give each XCD a
// contiguous range of tiles (neighbouring tiles share operand panels in its L2)
__device__ inline int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

// Block -> tile of a batch of graphs (G > 1): the tiles, in decreasing cost, are dealt to the
// XCDs in chunks of 16 consecutive tiles (in the main 4 row tiles by 4 column tiles of one graph), so every
// XCD starts on the longest tiles and the short ones fill the end; a single graph keeps
// xcd_remap's contiguous range per XCD
__device__ inline int batch_remap(int b, int nb, int G) {
    if (G == 1) return xcd_remap(b, nb);
    constexpr int C = 16;
    const int full = nb / (8 * C) * (8 * C);
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return ((i / C) * 8 + x) * C + (i % C);
}

// tile `local` of one graph's contraction -> (row tile, column tile)
template <int MODE>
__device__ inline void local_tile(const GraphDev& d, int local, int& tm, int& tn) {
    const int TM = d.gm_tm[MODE], TN = d.gm_tn[MODE];
    // groups of 4 row tiles sweep the column tiles together (measured faster than
    // groups of 8, which cut the L2 misses by a third but not the time)
    constexpr int GM = 4;
    const int per_group = GM * TN;
    const int grp = local / per_group;
    const int rows_in = min(GM, TM - grp * GM);
    const int w = local - grp * per_group;
    tm = grp * GM + w % rows_in;
    tn = w / rows_in;
}

template <int MODE>
__device__ inline void decode_tile(const GraphDev* gd, int G, int tile, int& g, int& tm, int& tn) {
    // the graphs' tile ranges follow one another in decreasing tile cost (K = n_pad), not in
    // graph order, so the longest tiles of a batch are dispatched first
    g = 0;
    for (int x = 0; x < G; ++x) {
        const int b = gd[x].gm_begin[MODE];
        if (tile >= b && tile < b + gd[x].gm_tm[MODE] * gd[x].gm_tn[MODE]) {
            g = x;
            break;
        }
    }
    local_tile<MODE>(gd[g], tile - gd[g].gm_begin[MODE], tm, tn);
}

// One block tile (row tile tm, column tile tn) of graph g's contraction.
template <int PREC, int BM, int NTW, int MODE>
__device__ __forceinline__ void gemm_tile(const GraphDev* __restrict__ gd, int g, int tm, int tn, int honor_stop,
                                          int passes, int cstage) {
    using T = Tile<BM, NTW>;
    constexpr int MT = T::MT;
    constexpr int BN = T::BN;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    int* f2l = (int*)(lds + T::CT_BYTES);            // BN + 2 gather counters (after the colours)

    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const int pS = st->pS;
    const float tf = (float)st->t;
    const bool pen = (d.lambda * tf != 0.0f) || (d.mu * tf != 0.0f);
    // a graph takes either the dense operand pass or, in the iterations where its graph
    // state asks for them, the sparse penalty rows (written to G before the fused
    // epilogue, added to G after the fast path's store); the plain path
    // (passes bit 3) always takes the dense pass
    const bool sparse_pen = pen && d.psparse && !st->pdense && !(passes & 8);
    // passes bit 4: no penalty pass (the form the launch takes in iterations without one)
    const bool dense_pen = pen && !sparse_pen && !(passes & 16);
    // partitioning: the fitness term is -A.S, and with the operand built over D - Mt the
    // penalty product is negated as well
    const float sgn = prob_partition(d.problem) ? -1.0f : 1.0f;

    // graph fields in registers: reading them through gd after a store or an
    // atomic would reload them, one dependent round trip per use
    const int n = d.n, k = d.k, cs = d.cs;
    const int16_t* __restrict__ colr = d.c[pS];
    float* __restrict__ Gg = d.G;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = tm * BM;
    // column range of the tile in the flattened (member, colour) space
    int n0, ncol_end, d0 = 0;
    if (MODE == 1) {
        d0 = tn * d.gm_mpb;
        n0 = d0 * d.k;
        ncol_end = min(d.ncols, n0 + d.gm_mpb * d.k);
    } else {
        n0 = tn * BN;
        ncol_end = min(d.ncols, n0 + BN);
    }

    f32x4 acc[MT][NTW];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    const size_t ld = op_row_bytes(PREC, d.n_pad);
    const int nst = (int)(ld / kStageRowBytes);

    // per-lane columns: member and colour of each 16-column subtile
    int cm[NTW], cl[NTW];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        const int col = n0 + wn * (NTW * 16) + nt * 16 + (lane & 15);
        if (col < ncol_end) {
            cm[nt] = col / d.k;
            cl[nt] = col - cm[nt] * d.k;
        } else {
            cm[nt] = -1;
            cl[nt] = -1;
        }
    }
    const int dfirst = n0 / d.k;

    if (passes & 1) {
        // gather 2 f_color: sum over rows i of (A.S_d)[i, c_d(i)].  Skipped (passes bit 6) in
        // iterations whose penalty the sparse rows take, which read those entries of G anyway
        // and gather them there, and never done with passes bit 7 (timing).  The colours of the
        // tile's rows for its members go to LDS first (the stage buffers are free once every
        // wave is past the barrier), in coalesced loads
        const bool gather = !(passes & 128) && !((passes & 64) && sparse_pen);
        gemm_sweep<PREC, BM, NTW>(acc, (const uint8_t*)d.Aop + (size_t)m0 * ld,
                                  (const uint8_t*)d.Sop[pS] + (size_t)n0 * ld, ld, nst, lds);
        if (gather) {
            const int dlast = (ncol_end - 1) / k;
            const int nm = dlast - dfirst + 1;
            int16_t* ct = (int16_t*)lds;   // [nm][BM]
            // multicolouring: each selected colour of a vertex in turn (slot sl of the selection)
            const int CM = d.cmax;
            for (int sl = 0; sl < CM; ++sl) {
                __syncthreads();
                const int16_t* __restrict__ src = CM > 1 ? d.sel + (size_t)sl * cs : colr;
                const size_t rs = (size_t)CM * cs;   // row stride of a member
                for (int e = tid; e < nm * BM; e += T::THREADS) {
                    const int dm = e / BM, r = e - dm * BM;
                    ct[e] = m0 + r < n ? src[(size_t)(dfirst + dm) * rs + m0 + r] : (int16_t)-1;
                }
                // per element, through LDS counters of the tile's members
                if (sl == 0)
                    for (int e = tid; e < nm; e += T::THREADS) f2l[e] = 0;
                __syncthreads();
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ri = wm * T::RW + mt * 16 + (lane >> 4) * 4 + r;
#pragma unroll
                        for (int nt = 0; nt < NTW; ++nt) {
                            if (cm[nt] >= 0 && ct[(cm[nt] - dfirst) * BM + ri] == cl[nt])
                                atomicAdd(&f2l[cm[nt] - dfirst], (int)acc[mt][nt][r]);
                        }
                    }
            }
            __syncthreads();
            for (int e = tid; e < nm; e += T::THREADS)
                if (f2l[e]) atomicAdd(&d.f2[dfirst + e], f2l[e]);
        }
    }
    if ((passes & 2) && dense_pen) {
        __syncthreads();
        if constexpr (PREC == kPrecFP4) {
            // bf16 P against the fp4 S^T operand itself
            const size_t ld2 = (size_t)d.n_pad * 2;
            pen_sweep<BM, NTW>(acc, (const uint8_t*)d.Pop + (size_t)m0 * ld2,
                               (const uint8_t*)d.Sop[pS] + (size_t)n0 * ld, ld2, ld, d.n_pad / 64, lds);
        } else if constexpr (PREC == kPrecFP8) {
            const size_t ld2 = (size_t)d.n_pad * 2;
            gemm_sweep<kPrecBF16, BM, NTW>(acc, (const uint8_t*)d.Pop + (size_t)m0 * ld2,
                                           (const uint8_t*)d.Sp2[pS] + (size_t)n0 * ld2, ld2,
                                           d.n_pad * 2 / kStageRowBytes, lds);
        } else {
            gemm_sweep<PREC, BM, NTW>(acc, (const uint8_t*)d.Pop + (size_t)m0 * ld,
                                      (const uint8_t*)d.Sop[pS] + (size_t)n0 * ld, ld, nst, lds);
        }
    }
    if (!(passes & 4)) return;
    if constexpr (MODE == 0) {
        if (sparse_pen && d.pfuse && (passes & 32)) {
            // the sparse-rows launch takes this iteration's penalty and row update: it reads the
            // A.S counts (integers below n <= 32768) as uint16, half the bytes of fp32
            uint16_t* __restrict__ G16 = (uint16_t*)Gg;
            if ((k & 7) == 0) {
                // k a multiple of 8: column tiles start at multiples of 32 and members at multiples
                // of 8, so every 8-column piece of a tile row lies in one member's row.  The tile
                // goes through LDS (the stage buffers are free once every wave has read its last
                // fragments) and leaves in 16-byte stores along the rows, instead of 2-byte
                // stores that touch four rows at once
                constexpr int L16 = BN + 8;   // uint16 per LDS row (rows four apart on other banks)
                static_assert(BM * L16 * 2 <= T::NB * T::STAGE, "count tile fits the stage buffers");
                uint16_t* T16 = (uint16_t*)lds;
                __syncthreads();
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = wm * T::RW + mt * 16 + (lane >> 4) * 4 + r;
                            const int col = wn * (NTW * 16) + nt * 16 + (lane & 15);
                            T16[row * L16 + col] = (uint16_t)acc[mt][nt][r];
                        }
                __syncthreads();
                constexpr int CPR = BN / 8;   // 16-byte pieces per tile row
                for (int e = tid; e < BM * CPR; e += T::THREADS) {
                    const int row = e / CPR, ch = e - row * CPR;
                    const int i = m0 + row, col = n0 + ch * 8;
                    if (i < n && col < ncol_end) {
                        const int dm = col / k, l = col - dm * k;
                        *(uint4*)(G16 + ((size_t)dm * n + i) * k + l) = *(const uint4*)(T16 + row * L16 + ch * 8);
                    }
                }
                return;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * T::RW + mt * 16 + (lane >> 4) * 4 + r;
                    if (i < n) {
#pragma unroll
                        for (int nt = 0; nt < NTW; ++nt)
                            if (cm[nt] >= 0) G16[((size_t)cm[nt] * n + i) * k + cl[nt]] = (uint16_t)acc[mt][nt][r];
                    }
                }
            return;
        }
        // G[d][i][l] = acc (sparse penalty rows, when present, are added afterwards)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * T::RW + mt * 16 + (lane >> 4) * 4 + r;
                if (i < n) {
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
                        if (cm[nt] >= 0) Gg[((size_t)cm[nt] * n + i) * k + cl[nt]] = sgn * acc[mt][nt][r];
                }
            }
    } else {
        // ---- fused epilogue: the tile's gradient rows go through LDS, at most 128 rows at a time ----
        constexpr int EPI = BM < 128 ? BM : 128;
        constexpr int LDG = BN + 4;
        float* Gt = (float*)lds;
        const int nmem = min(d.gm_mpb, d.D - d0);
        const int g16 = tid >> 4, l16 = tid & 15;
        const long long t = st->t;
        const float nut = prob_added(d.problem) ? d.nu * (float)t : 0.0f;
        const int prob = d.problem;
        const bool smooth = d.nb_iter > 0 && ((t + 1) % d.nb_iter) == 0;
        const int pW = st->pW;
        const float* __restrict__ Wc = d.W[pW];
        float* __restrict__ Wn = d.W[pW ^ 1];
        int16_t* __restrict__ cn = d.c[pS ^ 1];
        const int32_t* __restrict__ Vp = d.V[pS];
        const float eta = d.eta, rho = d.rho;
        const int c1 = d.c1, c2 = d.c2;
#pragma unroll 1
        for (int h = 0; h < BM / EPI; ++h) {
            __syncthreads();
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * T::RW + mt * 16 + (lane >> 4) * 4 + r;
                        const int col = wn * (NTW * 16) + nt * 16 + (lane & 15);
                        if (row / EPI == h) Gt[(row - h * EPI) * LDG + col] = acc[mt][nt][r];
                    }
            __syncthreads();
            // rows (member, vertex): softmax along k, straight-through gradient, update,
            // smoothing, and the argmax colouring of the updated weights
            for (int rr = g16; rr < EPI * nmem; rr += T::THREADS / 16) {
                const int r = rr % EPI, dm = rr / EPI;
                const int i = m0 + h * EPI + r;
                if (i >= n) continue;
                const int dd = d0 + dm;
                const size_t rowoff = ((size_t)dd * n + i) * k;
                const float* w = Wc + rowoff;
                float* wo = Wn + rowoff;
                const float* gr = Gt + r * LDG + dm * k;
                const float* g1 = Gg + rowoff;      // sparse penalty rows
                const int32_t* V = Vp + (size_t)dd * k;
                float mx = -INFINITY;
                for (int l = l16; l < k; l += 16) mx = fmaxf(mx, w[l]);
                mx = row16_max(mx);
                float z = 0.0f, q = 0.0f;
                for (int l = l16; l < k; l += 16) {
                    const float e = exp_soft(w[l] - mx);
                    float gv = sgn * gr[l];
                    if (sparse_pen) gv += g1[l];
                    if (nut != 0.0f) gv += nut * added_grad(prob, V[l], l, c1, c2);
                    z += e;
                    q += e * gv;
                }
                z = row16_sum(z);
                q = row16_sum(q);
                const float rz = 1.0f / z;
                const float rq = q * rz;
                float best = -INFINITY;
                int bi = 0x7FFFFFFF, bad = 0;
                for (int l = l16; l < k; l += 16) {
                    const float e = exp_soft(w[l] - mx) * rz;
                    float gv = sgn * gr[l];
                    if (sparse_pen) gv += g1[l];
                    if (nut != 0.0f) gv += nut * added_grad(prob, V[l], l, c1, c2);
                    float nw = w[l] - eta * (e * (gv - rq));
                    if (smooth) nw = nw / rho;
                    wo[l] = nw;
                    if ((__float_as_uint(nw) & 0x7F800000u) == 0x7F800000u) bad = 1;
                    if (nw > best) { best = nw; bi = l; }
                }
                // the argmax over the row: the largest value, then the lowest colour holding it
                const int bo = f32_ord(best);
                const int bmax = row16_max_i(bo);
                bi = row16_min_i(bo == bmax ? bi : 0x7FFFFFFF);
                bad = row16_max_i(bad);
                if (l16 == 0) {
                    if (bad || bi >= k) {
                        bi = 0;
                        atomicExch(&st->next_bad, 1);
                    }
                    cn[(size_t)dd * cs + i] = (int16_t)bi;
                }
            }
        }
    }
}

template <int PREC, int BM, int NTW, int MODE>
__device__ __forceinline__ void gemm_body(const GraphDev* __restrict__ gd, int G, int total_tiles, int honor_stop,
                                          int passes, int cstage) {
    const int tile = batch_remap(blockIdx.x, total_tiles, G);
    int g, tm, tn;
    decode_tile<MODE>(gd, G, tile, g, tm, tn);
    gemm_tile<PREC, BM, NTW, MODE>(gd, g, tm, tn, honor_stop, passes, cstage);
}

// ------------------------------------------------------------- dispatch ------

constexpr int kMaxLds = 160 * 1024;

template <int BM, int NTW, int MODE>
static size_t lds_bytes(int cstage) {
    using T = Tile<BM, NTW>;
    const size_t sweep = T::NB * T::STAGE;
    if (MODE == 0) return sweep;
    const size_t epi = (size_t)(BM < 128 ? BM : 128) * (T::BN + 4) * sizeof(float) + (size_t)cstage;
    return sweep > epi ? sweep : epi;
}

// The contraction kernel.  Tiles that run two waves per SIMD (a second 4-wave block
// per CU, or one 8-wave block) are compiled for at most 256 registers per lane, so
// that the second wave can actually be resident.
template <int PREC, int BM, int NTW, int MODE>
__global__ __launch_bounds__(tile_threads(BM)) void k_gemm(const GraphDev* __restrict__ gd, int G,
                                                                 int total_tiles, int honor_stop, int passes,
                                                                 int cstage) {
    gemm_body<PREC, BM, NTW, MODE>(gd, G, total_tiles, honor_stop, passes, cstage);
}
template <int PREC, int BM, int NTW, int MODE>
__global__ __launch_bounds__(tile_threads(BM)) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_x2(
    const GraphDev* __restrict__ gd, int G, int total_tiles, int honor_stop, int passes, int cstage) {
    gemm_body<PREC, BM, NTW, MODE>(gd, G, total_tiles, honor_stop, passes, cstage);
}
template <int BM, int NTW, int MODE>
constexpr bool two_per_simd() {
    return MODE == 0 && Tile<BM, NTW>::TWO_PER_SIMD;
}

template <int PREC, int BM, int NTW, int MODE>
static hipError_t prep_one() {
    const void* f;
    if constexpr (two_per_simd<BM, NTW, MODE>())
        f = (const void*)k_gemm_x2<PREC, BM, NTW, MODE>;
    else
        f = (const void*)k_gemm<PREC, BM, NTW, MODE>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
}

template <int PREC, int BM, int NTW, int MODE>
static hipError_t launch_one(const GraphDev* gd, int G, int total_tiles, int honor_stop, int passes, int cstage,
                             hipStream_t s) {
    const size_t shm = lds_bytes<BM, NTW, MODE>(cstage);
    if (shm > (size_t)kMaxLds) return hipErrorInvalidValue;
    constexpr int threads = Tile<BM, NTW>::THREADS;
    if constexpr (two_per_simd<BM, NTW, MODE>())
        k_gemm_x2<PREC, BM, NTW, MODE><<<dim3(total_tiles), dim3(threads), shm, s>>>(gd, G, total_tiles, honor_stop,
                                                                                    passes, cstage);
    else
        k_gemm<PREC, BM, NTW, MODE><<<dim3(total_tiles), dim3(threads), shm, s>>>(gd, G, total_tiles, honor_stop,
                                                                                 passes, cstage);
    return hipGetLastError();
}

// instantiated tile shapes: (BM, NTW)
#define TCOL_GEMM_SHAPES(X, PREC, MODE) \
    X(PREC, 64, 2, MODE) X(PREC, 64, 4, MODE) X(PREC, 128, 4, MODE) X(PREC, 128, 6, MODE) X(PREC, 128, 8, MODE) \
    X(PREC, 64, 9, MODE) X(PREC, 128, 9, MODE) X(PREC, 256, 4, MODE) X(PREC, 256, 6, MODE)

#define TCOL_GEMM_CASE(PREC, BM, NTW, MODE)                                                             \
    if (s.prec == PREC && s.bm == BM && s.ntw == NTW && s.mode == MODE) {                               \
        if (op == 0) return hipSuccess;                                                                 \
        if (op == 1) return prep_one<PREC, BM, NTW, MODE>();                                             \
        if (op == 3) { *lds_out = lds_bytes<BM, NTW, MODE>(cstage); return hipSuccess; }                 \
        return launch_one<PREC, BM, NTW, MODE>(gd, G, total_tiles, honor_stop, passes, cstage, st);     \
    }

static hipError_t gemm_dispatch(int op, const GemmShape& s, const GraphDev* gd, int G, int total_tiles,
                                int honor_stop, int passes, int cstage, hipStream_t st, size_t* lds_out) {
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP32, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecBF16, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP8, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP4, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP32, 1)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecBF16, 1)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP8, 1)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP4, 1)
    return hipErrorInvalidValue;
}

bool gemm_supported(const GemmShape& s) {
    return gemm_dispatch(0, s, nullptr, 0, 0, 0, 0, 0, nullptr, nullptr) == hipSuccess;
}
hipError_t gemm_prepare(const GemmShape& s) { return gemm_dispatch(1, s, nullptr, 0, 0, 0, 0, 0, nullptr, nullptr); }
hipError_t launch_gemm(const GemmShape& s, const GraphDev* gd, int G, int total_tiles, int honor_stop, int passes,
                       int cstage, hipStream_t st) {
    if (total_tiles <= 0) return hipSuccess;
    return gemm_dispatch(2, s, gd, G, total_tiles, honor_stop, passes, cstage, st, nullptr);
}
size_t gemm_lds_bytes(const GemmShape& s, int cstage) {
    size_t b = 0;
    if (gemm_dispatch(3, s, nullptr, 0, 0, 0, 0, cstage, nullptr, &b) != hipSuccess) return 0;
    return b;
}
int gemm_bn(int ntw) { return 32 * ntw; }

}  // namespace tcol
