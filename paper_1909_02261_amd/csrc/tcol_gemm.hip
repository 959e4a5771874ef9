// MFMA contraction of the TensCol step on gfx950:
//   G = A . S_cat  (+ P . S_cat when the penalty is active),
// with S_cat = [S_1 ... S_D] (n x D*k, stored transposed as S^T [D*k][n_pad])
// and P the penalty operand built by the group-concentration kernel.
//
// A and S are 0/1, so A.S is exact in fp32, bf16 and fp8 operands with FP32
// accumulation; between the two passes each block gathers (A.S_d)[i, c_d(i)]
// into 2 f_color(S_d) (the gradient's first term is the TabuCol gamma matrix,
// whose entry at the vertex's own colour counts its conflicts).
//
// Layout: 256 threads = 4 waves as 2 (rows) x 2 (columns); block tile BM x BN
// with BN = 32 * NTW; each wave owns (BM/2) x (16 NTW) as 16x16 MFMA subtiles.
// Both operands are K-contiguous; a K-stage moves 128 bytes of every operand
// row into LDS (stride 144 B), double buffered, prefetching the next stage
// into registers while the current one feeds the MFMAs.
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
__device__ inline f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_f32(float a, float b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int BM, int NTW>
struct Tile {
    static constexpr int BN = 32 * NTW;
    static constexpr int MT = BM / 32;                       // 16-row subtiles per wave
    static constexpr int STAGE = (BM + BN) * kLdsStride;     // bytes per LDS stage
    static constexpr int NCH = (BM + BN) * 8 / 256;          // 16-byte chunks per thread per stage
    static_assert((BM + BN) * 8 % 256 == 0, "chunk split");
};

// compute one LDS stage into acc (operand format PREC)
template <int PREC, int BM, int NTW>
__device__ inline void stage_mma(f32x4 (&acc)[BM / 32][NTW], const uint8_t* L, int lane, int wm, int wn) {
    constexpr int MT = BM / 32;
    const int ra = wm * (BM / 2) + (lane & 15);
    const int rb = BM + wn * (NTW * 16) + (lane & 15);
    const int q = lane >> 4;
    if constexpr (PREC == kPrecFP8) {
        i32x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const uint4* p = (const uint4*)(L + (ra + mt * 16) * kLdsStride + q * 32);
            uint4 x0 = p[0], x1 = p[1];
            a[mt] = i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
        }
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
            const uint4* p = (const uint4*)(L + (rb + nt * 16) * kLdsStride + q * 32);
            uint4 x0 = p[0], x1 = p[1];
            i32x8 b{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_fp8(a[mt], b, acc[mt][nt]);
        }
    } else if constexpr (PREC == kPrecBF16) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                a[mt] = *(const bf16x8*)(L + (ra + mt * 16) * kLdsStride + ks * 64 + q * 16);
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                bf16x8 b = *(const bf16x8*)(L + (rb + nt * 16) * kLdsStride + ks * 64 + q * 16);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_bf16(a[mt], b, acc[mt][nt]);
            }
        }
    } else {
        // fp32: a float4 at k = 16 ks + 4 q .. +4 feeds four 16x16x4 steps; A and B
        // use the same k order, so the sum is the plain product
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            float4 a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                a[mt] = *(const float4*)(L + (ra + mt * 16) * kLdsStride + ks * 64 + q * 16);
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                float4 b = *(const float4*)(L + (rb + nt * 16) * kLdsStride + ks * 64 + q * 16);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    acc[mt][nt] = mfma_f32(a[mt].x, b.x, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a[mt].y, b.y, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a[mt].z, b.z, acc[mt][nt]);
                    acc[mt][nt] = mfma_f32(a[mt].w, b.w, acc[mt][nt]);
                }
            }
        }
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 gbl_u32x4;

template <int BM, int NCH>
__device__ __forceinline__ void stage_gload(u32x4 (&pre)[NCH], const uint8_t* __restrict__ Arow,
                                            const uint8_t* __restrict__ Brow, size_t ld, int s, int tid) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int ch = tid + c * 256;
        const int row = ch >> 3, part = ch & 7;
        const uint8_t* src = row < BM ? Arow + (size_t)row * ld : Brow + (size_t)(row - BM) * ld;
        pre[c] = *(gbl_u32x4*)(src + (size_t)s * kStageRowBytes + part * 16);
    }
}

template <int NCH>
__device__ __forceinline__ void stage_lstore(const u32x4 (&pre)[NCH], uint8_t* buf, int tid) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int ch = tid + c * 256;
        const int row = ch >> 3, part = ch & 7;
        *(u32x4*)(buf + row * kLdsStride + part * 16) = pre[c];
    }
}

// One K-sweep: acc += Arows[m0.., :] . Brows[n0.., :]^T over `nstages` stages
// of 128 bytes.  Arow / Brow point at the first row of the tile; ld in bytes.
template <int PREC, int BM, int NTW>
__device__ __forceinline__ void gemm_sweep(f32x4 (&acc)[BM / 32][NTW], const uint8_t* __restrict__ Arow,
                                           const uint8_t* __restrict__ Brow, size_t ld, int nstages,
                                           uint8_t* lds) {
    using T = Tile<BM, NTW>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    u32x4 pre[T::NCH];
    stage_gload<BM, T::NCH>(pre, Arow, Brow, ld, 0, tid);
    stage_lstore<T::NCH>(pre, lds, tid);
    __syncthreads();
    for (int s = 0; s < nstages; ++s) {
        const int buf = s & 1;
        // the last iteration reloads its own stage into the idle buffer; nobody reads it
        stage_gload<BM, T::NCH>(pre, Arow, Brow, ld, min(s + 1, nstages - 1), tid);
        stage_mma<PREC, BM, NTW>(acc, lds + buf * T::STAGE, lane, wm, wn);
        stage_lstore<T::NCH>(pre, lds + (buf ^ 1) * T::STAGE, tid);
        __syncthreads();
    }
}

__device__ inline int elem_bytes(int prec) { return prec == kPrecFP32 ? 4 : (prec == kPrecBF16 ? 2 : 1); }

// XCD-aware order: hardware deals block b to XCD b mod 8, so give each XCD a
// contiguous range of tiles (neighbouring tiles share operand panels in its L2)
__device__ inline int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

template <int BM, int NTW>
__device__ inline void decode_tile(const GraphDev* gd, int G, int tile, int& g, int& tm, int& tn) {
    g = find_graph(gd, G, tile, [](const GraphDev& x) { return x.gm_begin; });
    const GraphDev& d = gd[g];
    const int local = tile - d.gm_begin;
    // groups of 4 row tiles sweep the column tiles together
    constexpr int GM = 4;
    const int per_group = GM * d.gm_tn;
    const int grp = local / per_group;
    const int rows_in = min(GM, d.gm_tm - grp * GM);
    const int w = local - grp * per_group;
    tm = grp * GM + w % rows_in;
    tn = w / rows_in;
}

template <int PREC, int BM, int NTW, int MODE>
__global__ __launch_bounds__(256) void k_gemm(const GraphDev* __restrict__ gd, int G, int total_tiles,
                                              int honor_stop, int passes) {
    using T = Tile<BM, NTW>;
    constexpr int MT = T::MT;
    constexpr int BN = T::BN;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    int* f2l = (int*)(lds + 2 * T::STAGE);     // BN + 2 gather counters

    const int tile = xcd_remap(blockIdx.x, total_tiles);
    int g, tm, tn;
    decode_tile<BM, NTW>(gd, G, tile, g, tm, tn);
    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const int pS = st->pS;
    const float tf = (float)st->t;
    const bool pen = (d.lambda * tf != 0.0f) || (d.mu * tf != 0.0f);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = tm * BM;
    // column range of the tile in the flattened (d, l) space
    int n0, ncol_end;
    if (MODE == 1) {
        n0 = tn * d.gm_mpb * d.k;
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

    const int eb = elem_bytes(PREC);
    const size_t ld = (size_t)d.n_pad * eb;
    const int nst = d.n_pad * eb / kStageRowBytes;

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
        gemm_sweep<PREC, BM, NTW>(acc, (const uint8_t*)d.Aop + (size_t)m0 * ld,
                                  (const uint8_t*)d.Sop[pS] + (size_t)n0 * ld, ld, nst, lds);
        // gather 2 f_color: sum over rows i of (A.S_d)[i, c_d(i)]
        for (int e = tid; e < BN + 2; e += 256) f2l[e] = 0;
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * (BM / 2) + mt * 16 + (lane >> 4) * 4 + r;
                if (i < d.n) {
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt) {
                        if (cm[nt] >= 0 && d.c[pS][(size_t)cm[nt] * d.n + i] == cl[nt])
                            atomicAdd(&f2l[cm[nt] - dfirst], (int)acc[mt][nt][r]);
                    }
                }
            }
        __syncthreads();
        const int dlast = (ncol_end - 1) / d.k;
        for (int e = tid; e <= dlast - dfirst; e += 256)
            if (f2l[e]) atomicAdd(&d.f2[dfirst + e], f2l[e]);
    }
    if ((passes & 2) && pen) {
        __syncthreads();
        if constexpr (PREC == kPrecFP8) {
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
        // G[d][i][l] = acc
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * (BM / 2) + mt * 16 + (lane >> 4) * 4 + r;
                if (i < d.n) {
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
                        if (cm[nt] >= 0)
                            d.G[((size_t)cm[nt] * d.n + i) * d.k + cl[nt]] = acc[mt][nt][r];
                }
            }
    }
}

// ------------------------------------------------------------- dispatch ------

template <int PREC, int BM, int NTW, int MODE>
static size_t lds_bytes() {
    return 2 * Tile<BM, NTW>::STAGE + sizeof(int) * (Tile<BM, NTW>::BN + 2);
}

template <int PREC, int BM, int NTW, int MODE>
static hipError_t prep_one() {
    return hipFuncSetAttribute((const void*)k_gemm<PREC, BM, NTW, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes<PREC, BM, NTW, MODE>());
}

template <int PREC, int BM, int NTW, int MODE>
static hipError_t launch_one(const GraphDev* gd, int G, int total_tiles, int honor_stop, int passes, hipStream_t s) {
    const size_t shm = lds_bytes<PREC, BM, NTW, MODE>();
    k_gemm<PREC, BM, NTW, MODE><<<dim3(total_tiles), dim3(256), shm, s>>>(gd, G, total_tiles, honor_stop, passes);
    return hipGetLastError();
}

// instantiated tile shapes: (BM, NTW)
#define TCOL_GEMM_SHAPES(X, PREC, MODE) \
    X(PREC, 64, 2, MODE) X(PREC, 64, 4, MODE) X(PREC, 128, 4, MODE) X(PREC, 128, 8, MODE) X(PREC, 64, 9, MODE) \
    X(PREC, 128, 9, MODE)

#define TCOL_GEMM_CASE(PREC, BM, NTW, MODE)                                                             \
    if (s.prec == PREC && s.bm == BM && s.ntw == NTW && s.mode == MODE) {                               \
        if (op == 0) return hipSuccess;                                                                 \
        if (op == 1) return prep_one<PREC, BM, NTW, MODE>();                                             \
        return launch_one<PREC, BM, NTW, MODE>(gd, G, total_tiles, honor_stop, passes, st);            \
    }

static hipError_t gemm_dispatch(int op, const GemmShape& s, const GraphDev* gd, int G, int total_tiles,
                                int honor_stop, int passes, hipStream_t st) {
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP32, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecBF16, 0)
    TCOL_GEMM_SHAPES(TCOL_GEMM_CASE, kPrecFP8, 0)
    return hipErrorInvalidValue;
}

bool gemm_supported(const GemmShape& s) { return gemm_dispatch(0, s, nullptr, 0, 0, 0, 0, nullptr) == hipSuccess; }
hipError_t gemm_prepare(const GemmShape& s) { return gemm_dispatch(1, s, nullptr, 0, 0, 0, 0, nullptr); }
hipError_t launch_gemm(const GemmShape& s, const GraphDev* gd, int G, int total_tiles, int honor_stop, int passes,
                       hipStream_t st) {
    if (total_tiles <= 0) return hipSuccess;
    return gemm_dispatch(2, s, gd, G, total_tiles, honor_stop, passes, st);
}
int gemm_bn(int ntw) { return 32 * ntw; }

}  // namespace tcol
