// Internal definitions shared by the gfx950 kernels and the host runtime of libtcol.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcol {

constexpr int kPrecFP32 = 0;
constexpr int kPrecBF16 = 1;
constexpr int kPrecFP8 = 2;
constexpr int kPrecFP4 = 3;

// problems (the public enum's values)
constexpr int kProbKCOL = 0, kProbECP = 1, kProbKPART = 2, kProbBKPART = 3, kProbMSCP = 4, kProbMCOL = 5;
// multicolouring: at most this many colours per vertex
constexpr int kMaxDemand = 8;
// partitioning: the fitness term is -A.S and the group concentration enters as D - Mt
__host__ __device__ inline bool prob_partition(int p) { return p == kProbKPART || p == kProbBKPART; }
// problems whose fitness and loss carry an added term (equity or colour cost)
__host__ __device__ inline bool prob_added(int p) { return p == kProbECP || p == kProbBKPART || p == kProbMSCP; }
// the added term is the equity fitness
__host__ __device__ inline bool prob_equity(int p) { return p == kProbECP || p == kProbBKPART; }
// derivative of the added fitness with respect to s_{d,i,l} (times nu t in the
// gradient): the equity term (+1 above c2, -1 below c1, else 0) or the colour
// cost z_l = l + 1 of minimum sum colouring
__device__ inline float added_grad(int problem, int32_t v, int l, int c1, int c2) {
    if (problem == kProbMSCP) return (float)(l + 1);
    return (float)((v > c2) - (v < c1));
}

// A.S in fp8: the penalty pass then runs on a bf16 copy of S (in fp4 it expands the fp4
// operand to bf16 in registers)
__host__ __device__ inline bool prec_split(int prec) { return prec == kPrecFP8; }
// bytes of one operand row of n_pad elements (n_pad a multiple of 256)
__host__ __device__ inline size_t op_row_bytes(int prec, int n_pad) {
    return prec == kPrecFP32 ? 4 * (size_t)n_pad
                             : (prec == kPrecBF16 ? 2 * (size_t)n_pad : (prec == kPrecFP8 ? (size_t)n_pad : (size_t)n_pad / 2));
}

constexpr int kF2Slots = 64;

constexpr int kMaxN = 32768;
constexpr int kMaxK = 4096;
constexpr int kMaxD = 1024;

// operand rows and columns are padded to this multiple (GEMM tile in M and K)
constexpr int kPadN = 256;
// extra zero rows after the D*k rows of S^T so any column tile can read a full tile
constexpr int kSRowSlack = 576;
// bytes per operand row per GEMM K-stage (one LDS row)
constexpr int kStageRowBytes = 128;

// device-resident per-graph state (iteration counter, stop flags, parities)
struct GraphState {
    long long t;        // iteration counter of Algorithm 1 (starts at 0)
    int stopped;        // a legal member was found (stop_on_legal) or an error occurred
    int error;          // 0 or a negative tcol status (non-finite weight)
    int legal_d;        // lowest legal member of the stopping iteration, or -1
    int steps_done;     // updates made since the last reset by the host
    int pW;             // fused path: which W buffer holds the current weights (0 = caller's)
    int pS;             // fused path: which colour / S buffer set is current
    int next_bad;       // fused path: the update produced a non-finite weight
    int pdense;         // sparse penalty graphs: this iteration takes the dense operand pass
    int prep_ticket;    // member blocks of the class-size kernel done this iteration (the
                        // last one takes the penalty choice and sets it back to 0)
    // iterations evaluated since init, by the route of their penalty product: none (lambda t =
    // mu t = 0), the dense operand pass, the sparse rows (counted by the fitness kernel)
    long long it_nopen, it_dense, it_sparse;
};

// per-graph descriptor, uploaded once at init
struct GraphDev {
    int n, k, D;
    int n_pad;          // padded n (rows and K of the operands)
    int cs;             // row stride of the colour arrays c[p] (n rounded up to 64)
    int ncols;          // D * k
    int rows_S;         // rows of S^T (D*k + slack)
    int problem, precision, bonus_diag, stop_on_legal, nb_iter;
    int c1, c2;         // equity bounds
    float eta, rho, nu, lambda, mu;
    float momentum;           // heavy-ball coefficient (0: plain step)
    long long edges;          // |E|
    const unsigned long long* ones_dev;   // when set: the number of ones of A (2 |E|) on the device,
                                          // read in place of `edges`
    // look-up tables over m = 0..D, with x = m (colouring) or D - m (partitioning)
    const float* lut_pen;     // 2 alpha lambda x^(alpha-1)   (0 at x = 0)
    const float* lut_bon;     // 2 beta mu x^(beta-1)         (0 at x = 0)
    const double* lut_ka;     // x^alpha
    const double* lut_vb;     // x^beta
    // buffers
    float* W[2];              // [0] caller's weights, [1] fused-path ping-pong buffer
    const uint8_t* A8;        // [n_pad][n_pad] 0/1 bytes (zero padded)
    void* Aop;                // [n_pad][n_pad] A in the operand precision
    void* Pop;                // [n_pad][n_pad] penalty operand (fp32; bf16 for BF16/FP8; bf16, halved, for FP4)
    void* Sop[2];             // [rows_S][n_pad] S^T in the A.S operand precision
    void* Sp2[2];             // [rows_S][n_pad] S^T in bf16 for the FP8 penalty pass (else null)
    int16_t* c[2];            // colours [D][cs] (member-major; entries n..cs-1 unused)
    int32_t* V[2];            // class sizes [D][k]
    float* G;                 // [D][n][k] gradient with respect to S (separate-kernel path)
    float* vel;               // [D][n][k] momentum velocity (null when momentum is 0)
    int32_t* f2;              // [D] 2 * f_color accumulated by the GEMM
    int32_t* f2p;             // [D][kF2Slots] 2 * f_color gathered by the sparse rows, spread over
                              // slots (row i adds to slot i mod kF2Slots) so their atomics do not
                              // pile onto one address; folded into f2 by the rows' last block
    int64_t* fcol;            // [D] main fitness: f_color, or the cut for partitioning
    int64_t* feq;             // [D] added fitness: f_eq, the colour cost, or 0
    int64_t* f;               // [D] fcol + feq
    double* part;             // [mt_tiles][2] kappa / varpi partial sums
    int16_t* snap;            // [n] colouring of the legal member ([n][cmax] for multicolouring)
    // multicolouring (cmax > 1, or problem kProbMCOL): vertex i takes dem[i] <= cmax colours;
    // sel[d][s][i] (s < cmax, rows of cs) is the s-th colour of vertex i in member d, in
    // decreasing weight, -1 past dem[i]; c[p] holds slot 0 (the argmax)
    int cmax;
    const int32_t* dem;
    int16_t* sel;
    GraphState* st;
    int16_t* cT;              // [n][cTs] colours of the current iteration, vertex-major
    int cTs;                  // row stride of cT (D rounded up to 8)
    int psparse;              // fast / epilogue paths: penalty rows from the nonzeros of P, in
                              // every iteration or in those that ask for them (ps_mode); else
                              // the dense operand pass of the contraction
    int16_t* cls_v;           // [D][cs] vertices of each member grouped by colour
    int32_t* cls_off;         // [D][k + 1] start of colour l's vertices in cls_v (last entry n)
    int2* cinfo;              // [D][cs] start in cls_v and size of the class of vertex i in member d
    long long* sq;            // [D] sum over colours of the squared class sizes of each member
    int ps_mode;              // sparse penalty: 1 every iteration, 2 when the classes are small
    int pfuse;                // fast path: the sparse-rows launch also takes this graph's row update
                              // (softmax, straight-through gradient, update, next colours) in
                              // every iteration, writing the other W and colour buffers, and the
                              // A.S counts of its sparse iterations are stored as uint16 in G
    // flattened work offsets (prefix sums over graphs)
    int row_begin;            // rows (d, i) for row kernels
    int mem_begin;            // members d for per-member kernels
    int ps_begin;             // blocks (rows) of the sparse penalty kernel
    int mt_begin;             // tiles of the group-concentration kernel
    int mt_T;                 // tiles per side
    int mt_ts;                // tile side of the group-concentration kernel (32 or 64)
    int ex_begin;             // blocks of the S^T expansion kernel
    int ex_cblocks;           // column blocks per S^T row group
    int gm_begin[2];          // GEMM tiles of the separate (0) and fused (1) tilings
    int gm_tm[2], gm_tn[2];   // tiles along rows and along columns
    int gm_mpb;               // fused tiling: members per column tile
};

// run-time flags passed to the kernels of one launch sequence
enum : int {
    kFlagLoss = 1,        // group-concentration kernel also writes kappa/varpi partials
    kFlagMtOut = 2,       // ... and Mt to an output buffer
    kFlagForcePen = 4,    // build the penalty operand even when lambda t = mu t = 0
    kFlagReport = 8,      // fitness kernel only reports (no stop, no state change)
    kFlagGate = 16,       // group-concentration kernel runs only for graphs on the dense penalty this iteration
    kFlagFused = 32,      // fitness kernel of the fused path: accept the update by flipping buffers
    kFlagPlainPen = 64,   // fitness kernel of the plain path: the penalty took the dense pass
    kFlagFoldSparse = 256,  // fitness kernel of the fast path: graphs whose iteration took the
                            // sparse rows have their f_color in the rows' slots (f2p)
    kFlagFlipFused = 512,   // fitness kernel of the fast path: graphs whose row update rode on the
                            // sparse-rows launch (pfuse) accept it by flipping their W and colour
                            // buffers, unless they stop
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline int round_up(int a, int b) { return ceil_div(a, b) * b; }

// S^T expansion: colour rows per thread (the member's colours are loaded once for them), and
// the launch's blocks of 256 threads for a graph
constexpr int kExpandRows = 4;
inline int expand_blocks(int D, int k, int n_pad) {
    const long long items = (long long)D * ((k + kExpandRows - 1) / kExpandRows) * (n_pad / 16);
    return (int)((items + 255) / 256);
}

// ---- softmax arithmetic of the row updates ----
// e^x on the hardware base-2 exponential of x log2(e): for the arguments of a softmax (x <= 0,
// a few tens at most in magnitude) the relative error is below about 2^-21
__device__ __forceinline__ float exp_soft(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// Lane reductions in DPP steps, over lanes that are all active.  Floats take part as
// integers of the same order (an involution on the bit patterns of finite values and
// infinities), so that every step is one integer max or min.
__device__ __forceinline__ int f32_ord(float x) {
    const int b = __float_as_int(x);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float f32_from_ord(int o) { return __int_as_float(o ^ ((o >> 31) & 0x7FFFFFFF)); }
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int ident, int v) {
    return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float ident, float v) {
    return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(ident), __float_as_int(v)));
}
// within each 16-lane row: xor 1 and 2 inside each quad, then rotations by 4 and 8; every lane
// of the row ends with the row's result
__device__ __forceinline__ int row16_max_i(int v) {
    constexpr int I = (int)0x80000000;
    v = max(v, dpp_i<0xB1, 0xF>(I, v));    // quad_perm [1, 0, 3, 2]
    v = max(v, dpp_i<0x4E, 0xF>(I, v));    // quad_perm [2, 3, 0, 1]
    v = max(v, dpp_i<0x124, 0xF>(I, v));   // row_ror 4
    return max(v, dpp_i<0x128, 0xF>(I, v));   // row_ror 8
}
__device__ __forceinline__ int row16_min_i(int v) {
    constexpr int I = 0x7FFFFFFF;
    v = min(v, dpp_i<0xB1, 0xF>(I, v));
    v = min(v, dpp_i<0x4E, 0xF>(I, v));
    v = min(v, dpp_i<0x124, 0xF>(I, v));
    return min(v, dpp_i<0x128, 0xF>(I, v));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_f<0xB1, 0xF>(0.0f, v);
    v += dpp_f<0x4E, 0xF>(0.0f, v);
    v += dpp_f<0x124, 0xF>(0.0f, v);
    return v + dpp_f<0x128, 0xF>(0.0f, v);
}
__device__ __forceinline__ float row16_max(float v) { return f32_from_ord(row16_max_i(f32_ord(v))); }
// over the 64 lanes: the row results, then lane 15 of rows 0 and 2 into rows 1 and 3 and lane
// 31 into rows 2 and 3; lane 63 ends with the wave's result, returned from a scalar register
__device__ __forceinline__ int wave_max_i(int v) {
    constexpr int I = (int)0x80000000;
    v = row16_max_i(v);
    v = max(v, dpp_i<0x142, 0xA>(I, v));   // row_bcast 15 into rows 1 and 3
    v = max(v, dpp_i<0x143, 0xC>(I, v));   // row_bcast 31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_min_i(int v) {
    constexpr int I = 0x7FFFFFFF;
    v = row16_min_i(v);
    v = min(v, dpp_i<0x142, 0xA>(I, v));
    v = min(v, dpp_i<0x143, 0xC>(I, v));
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ float wave_sum(float v) {
    v = row16_sum(v);
    v += dpp_f<0x142, 0xA>(0.0f, v);
    v += dpp_f<0x143, 0xC>(0.0f, v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_max(float v) { return f32_from_ord(wave_max_i(f32_ord(v))); }

// find the graph that owns flattened work item `w` given a begin offset per graph
template <typename F>
__device__ inline int find_graph(const GraphDev* gd, int G, int w, F begin_of) {
    int g = 0;
    while (g + 1 < G && begin_of(gd[g + 1]) <= w) ++g;
    return g;
}

}  // namespace tcol
